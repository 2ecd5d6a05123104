"""Off-grid FP64 kernels through the C ABI: the Cartesian midpoint-rule
projection (Sect. 5's foil) and synthesis at arbitrary points, against the
oracle, the golden closed forms and the sampling-theorem transforms."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from closed_forms import DEGREE, load_closed_forms, poly  # noqa: E402
from oracle import direct as D, points as PT  # noqa: E402
from paper_1604_05140_amd import sgl, synth  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SEED = synth.BASE_SEED + 900


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def t(x, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV, dtype)


def einf(ref, got):
    return D.error_metrics(np.asarray(ref), np.asarray(got))["e_inf"]


@pytest.mark.parametrize("B,nx,h,s", [(3, 10, 4.0, 1.0), (6, 20, 5.0, 1.0), (5, 16, 6.0, 1.6)])
def test_midpoint_matches_oracle(B, nx, h, s):
    """Same cells, same sum: every coefficient against the oracle's midpoint rule."""
    g = np.random.default_rng(SEED + B)
    vals = (g.standard_normal((2, nx ** 3)) + 1j * g.standard_normal((2, nx ** 3))) / np.sqrt(2)
    plan = sgl.sgl_plan_scaled([B, B], "f64", 0, s)
    out = torch.empty(plan.total_coeffs, dtype=torch.complex128, device=DEV)
    sgl.sgl_midpoint_forward(plan, t(vals.reshape(-1)), nx, h, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(2, -1)
    for b in range(2):
        assert einf(PT.midpoint_forward(vals[b], B, nx, h, radial_scale=s), got[b]) <= 1e-12


@pytest.mark.parametrize("s", [1.0, 2.2])
def test_synthesis_matches_oracle_and_closed_forms(s):
    B = 7
    xyz = np.random.default_rng(SEED + 3).uniform(-4 * s, 4 * s, (1000, 3))
    c = synth.complex_normal_coeffs(B, 2, seed=SEED + 4)
    plan = sgl.sgl_plan_scaled([B, B], "f64", 0, s)
    out = torch.empty(2 * len(xyz), dtype=torch.complex128, device=DEV)
    sgl.sgl_synthesize_points(plan, t(c.reshape(-1)), t(xyz, torch.float64), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(2, -1)
    for b in range(2):
        assert einf(PT.synthesize(c[b], B, xyz, radial_scale=s), got[b]) <= 1e-12
    # closed forms: synthesis of the exact coefficients of x + iy is x + iy
    ref = np.zeros(D.num_coeffs(B), dtype=np.complex128)
    for (nm, n, l, m, v) in load_closed_forms():
        if nm == "x+iy":
            ref[D.omega(n, l, m)] = v * s ** (1.5 + DEGREE[nm])
    plan1 = sgl.sgl_plan_scaled([B], "f64", 0, s)
    out1 = torch.empty(len(xyz), dtype=torch.complex128, device=DEV)
    sgl.sgl_synthesize_points(plan1, t(ref), t(xyz, torch.float64), out1)
    torch.cuda.synchronize()
    poly_v = poly("x+iy", xyz[:, 0], xyz[:, 1], xyz[:, 2])
    assert np.abs(out1.cpu().numpy() - poly_v).max() <= 1e-12 * np.abs(poly_v).max()


def test_synthesis_at_grid_points_is_the_inverse_transform():
    B = 16
    c = synth.complex_normal_coeffs(B, 1, seed=SEED + 5, decay=1.0)[0]
    plan = sgl.sgl_plan_ex([B], "f64", sgl.SGL_SAMPLES_RAW)
    xyz = t(D.sample_grid_points(B), torch.float64)
    out = torch.empty(D.num_samples(B), dtype=torch.complex128, device=DEV)
    sgl.sgl_synthesize_points(plan, t(c), xyz, out)
    raw = torch.empty_like(out)
    sgl.sgl_inverse(plan, t(c), raw)
    torch.cuda.synchronize()
    assert einf(raw.cpu().numpy(), out.cpu().numpy()) <= 1e-12


def test_midpoint_foil_converges_on_a_bandlimited_function():
    """A bandlimited function synthesized on Cartesian cells: the midpoint rule
    recovers its coefficients only as the cells shrink (the sampling-theorem
    transform recovers them exactly on its own grid)."""
    B, h = 8, 9.0  # the cube must hold the Gaussian-weighted degree-15 terms (h = 7 truncates at ~5e-9)
    c = synth.complex_normal_coeffs(B, 1, seed=SEED + 6, decay=1.0)[0]
    plan = sgl.sgl_plan(B, 1, "f64")
    errs = []
    for nx in (12, 24, 64):
        xyz = t(PT.cartesian_midpoints(nx, h), torch.float64)
        vals = torch.empty(nx ** 3, dtype=torch.complex128, device=DEV)
        sgl.sgl_synthesize_points(plan, t(c), xyz, vals)
        out = torch.empty(plan.total_coeffs, dtype=torch.complex128, device=DEV)
        sgl.sgl_midpoint_forward(plan, vals, nx, h, out)
        torch.cuda.synchronize()
        errs.append(einf(c, out.cpu().numpy()))
    assert errs[2] <= 1e-12
    assert errs[0] > 1e3 * errs[2]


def test_off_grid_needs_fp64_and_valid_grid():
    plan = sgl.sgl_plan(4, 1, "f32")
    v = torch.zeros(8, dtype=torch.complex64, device=DEV)
    c = torch.empty(plan.total_coeffs, dtype=torch.complex64, device=DEV)
    with pytest.raises(sgl.SglError) as e:
        sgl.sgl_midpoint_forward(plan, v, 2, 1.0, c)
    assert e.value.status == 2
    p64 = sgl.sgl_plan(4, 1, "f64")
    v64 = torch.zeros(8, dtype=torch.complex128, device=DEV)
    c64 = torch.empty(p64.total_coeffs, dtype=torch.complex128, device=DEV)
    with pytest.raises(sgl.SglError) as e:
        sgl.sgl_midpoint_forward(p64, v64, 2, -1.0, c64)
    assert e.value.status == 1
