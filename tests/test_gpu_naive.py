"""GPU naive transforms (Alg. 1 forward, Alg. 2 inverse; plain FP64) through the
C ABI: against the CPU oracle at small bandlimits (every value), against the
fast FP64 GPU path at larger ones, batched uneven bandlimits, raw samples, and
the FP64-only contract.  Error metric as elsewhere: e_inf = max|delta| /
max|reference| per function, bar 1e-12 in FP64."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import direct as D  # noqa: E402
from paper_1604_05140_amd import sgl, synth  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SEED = synth.BASE_SEED + 700


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(x, ct=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x).reshape(-1)).to(DEV, ct)


def run(fn, plan, x, n_out):
    out = torch.empty(n_out, dtype=plan.complex_dtype, device=DEV)
    fn(plan, x if isinstance(x, torch.Tensor) else dev(x), out)
    torch.cuda.synchronize()
    return out


def einf(ref, got):
    return D.error_metrics(np.asarray(ref), np.asarray(got))["e_inf"]


@pytest.mark.parametrize("B,batch", [(1, 1), (3, 2), (4, 1), (8, 1)])
def test_naive_matches_oracle(B, batch):
    """Every coefficient and every sample against the oracle's quadrature and
    synthesis sums, on arbitrary (not bandlimited) samples and coefficients."""
    s = synth.complex_normal_samples(B, batch, seed=SEED + B)
    c = synth.complex_normal_coeffs(B, batch, seed=SEED + 10 + B)
    plan = sgl.sgl_plan(B, batch, "f64")
    cg = run(sgl.sgl_naive_forward, plan, s, plan.total_coeffs).cpu().numpy().reshape(batch, -1)
    sg = run(sgl.sgl_naive_inverse, plan, c, plan.total_samples).cpu().numpy().reshape(batch, -1)
    for b in range(batch):
        assert einf(D.forward(s[b], B), cg[b]) <= 1e-12, b
        assert einf(D.inverse(c[b], B), sg[b]) <= 1e-12, b


@pytest.mark.parametrize("B", [12, 16, 32])
def test_naive_matches_fast_path_and_round_trip(B):
    """Naive and fast FP64 GPU paths are the same linear maps; bandlimited
    coefficients survive naive synthesis + naive analysis (Thm. 3.4)."""
    c = synth.complex_normal_coeffs(B, 2, seed=SEED + 20 + B, decay=1.0)
    s = synth.complex_normal_samples(B, 2, seed=SEED + 30 + B)
    plan = sgl.sgl_plan(B, 2, "f64")
    cn = run(sgl.sgl_naive_forward, plan, s, plan.total_coeffs)
    cf = run(sgl.sgl_forward, plan, s, plan.total_coeffs)
    sn = run(sgl.sgl_naive_inverse, plan, c, plan.total_samples)
    sf = run(sgl.sgl_inverse, plan, c, plan.total_samples)
    nc, ns = D.num_coeffs(B), D.num_samples(B)
    for b in range(2):
        assert einf(cf.cpu().numpy()[b * nc:(b + 1) * nc], cn.cpu().numpy()[b * nc:(b + 1) * nc]) <= 1e-12
        assert einf(sf.cpu().numpy()[b * ns:(b + 1) * ns], sn.cpu().numpy()[b * ns:(b + 1) * ns]) <= 1e-12
    back = run(sgl.sgl_naive_forward, plan, sn, plan.total_coeffs).cpu().numpy()
    assert einf(c.reshape(-1), back) <= 1e-12


def test_naive_batched_uneven_bandlimits():
    Bs = [3, 5, 3, 8, 1, 5]
    plan = sgl.sgl_plan_ex(Bs, "f64")
    so, co = plan.offsets()
    cs = [synth.complex_normal_coeffs(B, 1, seed=SEED + 40 + q)[0] for q, B in enumerate(Bs)]
    ss = [synth.complex_normal_samples(B, 1, seed=SEED + 50 + q)[0] for q, B in enumerate(Bs)]
    cg = run(sgl.sgl_naive_forward, plan, np.concatenate(ss), plan.total_coeffs).cpu().numpy()
    sg = run(sgl.sgl_naive_inverse, plan, np.concatenate(cs), plan.total_samples).cpu().numpy()
    for q, B in enumerate(Bs):
        assert einf(D.forward(ss[q], B), cg[co[q]:co[q] + D.num_coeffs(B)]) <= 1e-12
        assert einf(D.inverse(cs[q], B), sg[so[q]:so[q] + D.num_samples(B)]) <= 1e-12


def test_naive_raw_samples():
    B = 7
    c = synth.complex_normal_coeffs(B, 1, seed=SEED + 60)[0]
    f = D.inverse(c, B, raw=True)
    plan = sgl.sgl_plan_ex([B], "f64", sgl.SGL_SAMPLES_RAW)
    assert einf(c, run(sgl.sgl_naive_forward, plan, f, plan.total_coeffs).cpu().numpy()) <= 1e-12
    assert einf(f, run(sgl.sgl_naive_inverse, plan, c, plan.total_samples).cpu().numpy()) <= 1e-12


@pytest.mark.parametrize("dtype", ["f32", "split_bf16"])
def test_naive_needs_fp64_plan(dtype):
    plan = sgl.sgl_plan(4, 1, dtype)
    s = torch.zeros(plan.total_samples, dtype=plan.complex_dtype, device=DEV)
    c = torch.empty(plan.total_coeffs, dtype=plan.complex_dtype, device=DEV)
    with pytest.raises(sgl.SglError) as e:
        sgl.sgl_naive_forward(plan, s, c)
    assert e.value.status == 2
