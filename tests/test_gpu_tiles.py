"""GEMM tile geometries of the stage (b)/(c) launch slots (the per-order and
per-degree grouped contractions of Alg. 3 / Alg. 4, Eq. DLT and Eq. DRT).

The register-staged MFMA GEMM runs with a 128 x 64 (complex) or a 64 x 32 tile,
and the forward radial slot (split and FP32 forms) and the FP32 Legendre slots
also on a copy-fed kernel (128 x 128); the plan-time autotuner picks one per launch slot.
Every geometry must give the default plan's results to the form's tolerance,
hold the oracle's quadrature and synthesis sums on small ragged plans, and
survive graph capture.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import direct as D  # noqa: E402
from paper_1604_05140_amd import sgl, synth  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SEED = synth.BASE_SEED + 7000
GEMM_SLOTS = (3, 4, 5, 6)  # forward Legendre, forward radial, inverse radial, inverse Legendre
TOL = {"f64": 1e-12, "f32": 1e-5, "split_bf16": 1e-6}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(x, ct):
    return torch.from_numpy(np.ascontiguousarray(x).reshape(-1)).to(DEV, ct)


def run(plan, fn, x):
    n = plan.total_coeffs if fn is sgl.sgl_forward else plan.total_samples
    out = torch.full((n,), float("nan"), dtype=plan.complex_dtype, device=DEV)
    fn(plan, x, out)
    torch.cuda.synchronize()
    return out


def einf(ref, got):
    return float((ref - got).abs().max() / ref.abs().max())


def slot_geometries(plan, slot):
    out = []
    for g in (0, 1, 2):
        try:
            plan.set_launch_tile(slot, g)
            out.append(g)
        except sgl.SglError as e:
            assert e.status == 2  # SGL_ERR_UNSUPPORTED
    plan.set_launch_tile(slot, 0)
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32", "split_bf16"])
def test_every_geometry_matches_default(dtype):
    """Ragged groups: two bandlimits (one with a Bluestein ring length), a
    class of two functions, rows and columns that end mid-tile."""
    Bs = [24, 24, 17]
    print(f"tile geometries {dtype} B={Bs}", flush=True)
    ct = torch.complex128 if dtype == "f64" else torch.complex64
    base = sgl.sgl_plan_ex(Bs, dtype)
    s = dev(np.concatenate([synth.complex_normal_samples(B, 1, seed=SEED + q)[0] for q, B in enumerate(Bs)]), ct)
    c = dev(np.concatenate([synth.complex_normal_coeffs(B, 1, seed=SEED + 10 + q, decay=1.0)[0]
                            for q, B in enumerate(Bs)]), ct)
    f0, i0 = run(base, sgl.sgl_forward, s), run(base, sgl.sgl_inverse, c)
    tiles0 = base.launch_tiles()
    assert tiles0[0] == (0, 0) and tiles0[7] == (0, 0)
    assert tiles0[4] == (128, 64) and tiles0[5] == (128, 64)
    geos = {q: slot_geometries(base, q) for q in GEMM_SLOTS}
    assert geos[5] == [0, 1]
    # split form: the forward radial slot also runs the copy-fed kernel, the
    # Legendre slots only it; FP32: the Legendre slots and the forward radial
    # slot also run theirs; other slots: the two register-staged tiles
    assert geos[4] == ([0, 1] if dtype == "f64" else [0, 1, 2])
    assert geos[3] == geos[6] == {"split_bf16": [0], "f32": [0, 1, 2], "f64": [0, 1]}[dtype]
    p = sgl.sgl_plan_ex(Bs, dtype)
    for q in GEMM_SLOTS:
        for g in geos[q]:
            p.set_launch_tile(q, g)
            copy_fed = g == 2 or (dtype == "split_bf16" and q in (3, 6))
            want = (64, 32) if g == 1 else ((128, 128) if copy_fed else (128, 64))
            assert p.launch_tiles()[q] == want
            f1, i1 = run(p, sgl.sgl_forward, s), run(p, sgl.sgl_inverse, c)
            assert torch.isfinite(f1).all() and torch.isfinite(i1).all()
            ef, ei = einf(f0, f1), einf(i0, i1)
            print(f"  slot {q} geometry {g}: forward {ef:.1e}, inverse {ei:.1e}", flush=True)
            assert ef <= TOL[dtype] and ei <= TOL[dtype], (q, g, ef, ei)
        p.set_launch_tile(q, 0)
    # all slots on their last geometry at once
    for q in GEMM_SLOTS:
        p.set_launch_tile(q, geos[q][-1])
    assert einf(f0, run(p, sgl.sgl_forward, s)) <= TOL[dtype]
    assert einf(i0, run(p, sgl.sgl_inverse, c)) <= TOL[dtype]
    p.destroy()
    base.destroy()


def test_small_tile_against_oracle():
    """FP64 plan with every GEMM slot on the 64 x 32 tile against the oracle's
    quadrature sums (forward of non-bandlimited samples, Thm. 3.4) and
    synthesis sums, for two bandlimits at once."""
    Bs = [9, 6]
    p = sgl.sgl_plan_ex(Bs, "f64")
    for q in GEMM_SLOTS:
        p.set_launch_tile(q, 1)
    so, co = p.offsets()
    ss = [synth.complex_normal_samples(B, 1, seed=SEED + 20 + q)[0] for q, B in enumerate(Bs)]
    cs = [synth.complex_normal_coeffs(B, 1, seed=SEED + 30 + q)[0] for q, B in enumerate(Bs)]
    f = run(p, sgl.sgl_forward, dev(np.concatenate(ss), torch.complex128)).cpu().numpy()
    i = run(p, sgl.sgl_inverse, dev(np.concatenate(cs), torch.complex128)).cpu().numpy()
    for q, B in enumerate(Bs):
        ref_f = D.forward(ss[q], B)
        ref_i = D.inverse(cs[q], B)
        got_f = f[co[q]:co[q] + D.num_coeffs(B)]
        got_i = i[so[q]:so[q] + D.num_samples(B)]
        assert np.abs(got_f - ref_f).max() <= 1e-12 * np.abs(ref_f).max(), B
        assert np.abs(got_i - ref_i).max() <= 1e-12 * np.abs(ref_i).max(), B
    p.destroy()


def test_tile_change_recaptures_graphs():
    B, batch = 16, 2
    p = sgl.sgl_plan_ex([B] * batch, "f32", sgl.SGL_GRAPHS)
    s = dev(synth.complex_normal_samples(B, batch, seed=SEED + 40), torch.complex64)
    out = torch.empty(p.total_coeffs, dtype=torch.complex64, device=DEV)
    sgl.sgl_forward(p, s, out)  # captured with geometry 0
    torch.cuda.synchronize()
    ref = out.clone()
    for q in GEMM_SLOTS:
        p.set_launch_tile(q, 1)
    out.fill_(float("nan"))
    sgl.sgl_forward(p, s, out)  # same buffers: captured again with geometry 1
    sgl.sgl_forward(p, s, out)  # and replayed
    torch.cuda.synchronize()
    assert einf(ref, out) <= 1e-5
    p.destroy()


def test_copy_fed_geometries_in_graph_replays():
    """FP32 plan with the Legendre slots and the forward radial slot on the
    copy-fed kernels, captured in hipGraphs: several replays of the forward and
    the inverse, with eager work and synchronizations between them, each equal
    to the eager plan's results on the same tiles."""
    Bs = [40, 24, 40]
    eager = sgl.sgl_plan_ex(Bs, "f32")
    graph = sgl.sgl_plan_ex(Bs, "f32", sgl.SGL_GRAPHS)
    for p in (eager, graph):
        for q in (3, 4, 6):
            p.set_launch_tile(q, 2)
    s = dev(np.concatenate([synth.complex_normal_samples(B, 1, seed=SEED + 100 + q)[0] for q, B in enumerate(Bs)]),
            torch.complex64)
    c = dev(np.concatenate([synth.complex_normal_coeffs(B, 1, seed=SEED + 110 + q, decay=1.0)[0]
                            for q, B in enumerate(Bs)]), torch.complex64)
    f0, i0 = run(eager, sgl.sgl_forward, s), run(eager, sgl.sgl_inverse, c)
    fo = torch.empty_like(f0)
    io = torch.empty_like(i0)
    for rep in range(4):
        fo.fill_(float("nan"))
        io.fill_(float("nan"))
        sgl.sgl_forward(graph, s, fo)
        sgl.sgl_inverse(graph, c, io)
        torch.cuda.synchronize()
        assert torch.equal(fo, f0) and torch.equal(io, i0), rep
        _ = (s.abs() * 2).sum().item()  # eager work between replays
    eager.destroy()
    graph.destroy()


def test_bad_tile_requests():
    p = sgl.sgl_plan(8, 1, "f32")
    for slot, g, status in ((0, 1, 2), (7, 1, 2), (5, 2, 2), (4, 3, 2), (3, 3, 2), (6, 3, 2),
                            (10, 0, 1), (-1, 0, 1), (4, -1, 1)):
        with pytest.raises(sgl.SglError) as ei:
            p.set_launch_tile(slot, g)
        assert ei.value.status == status, (slot, g)
    p.destroy()


def test_autotuner_reports_its_tiles():
    Bs = synth.batched_bandlimits(24, 16, 40, seed=SEED + 50)
    p = sgl.sgl_plan_ex(list(Bs), "f32", sgl.SGL_AUTOTUNE)
    tiles = p.launch_tiles()
    print(f"autotuned tiles {tiles}", flush=True)
    for q in GEMM_SLOTS:
        copy_fed = q in (3, 4, 6)  # FP32 slots with a copy-fed geometry
        assert tiles[q] in (((128, 64), (64, 32)) + (((128, 128),) if copy_fed else ())), (q, tiles[q])
    p.destroy()


@pytest.mark.parametrize("dtype", ["split_bf16", "f32"])
def test_copy_fed_radial_against_oracle(dtype):
    """Split and FP32 plans with the forward radial contraction on the copy-fed
    kernel (Eq. DRT, 128 x 128 tiles) against the oracle's quadrature sums of
    non-bandlimited samples (Thm. 3.4): bandlimits whose K = 2B ends mid-chunk
    (B = 9, 21) and whose degree groups span several column tiles (B = 40,
    batch 2: up to 316 columns).  The two B = 40 functions are not stored one
    after another, so the kernel reads their coefficient offsets (the other
    tests' classes take the closed form)."""
    Bs = [40, 9, 21, 40]
    p = sgl.sgl_plan_ex(Bs, dtype)
    p.set_launch_tile(4, 2)
    assert p.launch_tiles()[4] == (128, 128)
    so, co = p.offsets()
    ss = [synth.complex_normal_samples(B, 1, seed=SEED + 60 + q)[0] for q, B in enumerate(Bs)]
    f = run(p, sgl.sgl_forward, dev(np.concatenate(ss), torch.complex64)).cpu().numpy()
    for q, B in enumerate(Bs):
        n = D.num_coeffs(B)
        # the highest degrees (the widest column groups, their last tiles), the
        # lowest, and a stride through the rest
        om = np.unique(np.concatenate([np.arange(min(n, 40)), np.arange(max(0, n - 200), n),
                                       np.arange(0, n, 1 if B < 10 else 53)]))
        ref = D.forward(ss[q].astype(np.complex128), B, omegas=om)
        got = f[co[q]:co[q] + n][om]
        e = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"copy-fed radial {dtype} B={B}: e_inf {e:.2e}", flush=True)
        assert e <= 2e-6, (B, e)
    p.destroy()


def test_copy_fed_f32_legendre_against_oracle():
    """FP32 plan with both Legendre contractions on the copy-fed kernel (Eq. DLT
    and its inverse, 128 x 128 tiles) against the oracle: quadrature sums of
    non-bandlimited samples (Thm. 3.4) and synthesis sums (Alg. 2) at grid
    points on every polar row.  Bandlimits whose polar contraction ends
    mid-chunk (2B = 18, 42; inverse K = B - m of every length up to B), order
    groups over several column tiles (B = 40, batch 2: 320 columns) and an
    inverse with two row tiles (2B = 140, the second ragged)."""
    Bs = [9, 21, 40, 40, 70]
    p = sgl.sgl_plan_ex(Bs, "f32")
    for q in (3, 6):
        p.set_launch_tile(q, 2)
        assert p.launch_tiles()[q] == (128, 128)
    so, co = p.offsets()
    ss = [synth.complex_normal_samples(B, 1, seed=SEED + 70 + q)[0] for q, B in enumerate(Bs)]
    cs = [synth.complex_normal_coeffs(B, 1, seed=SEED + 80 + q, decay=1.0)[0] for q, B in enumerate(Bs)]
    f = run(p, sgl.sgl_forward, dev(np.concatenate(ss), torch.complex64)).cpu().numpy()
    s = run(p, sgl.sgl_inverse, dev(np.concatenate(cs), torch.complex64)).cpu().numpy()
    rng = np.random.default_rng(SEED + 90)
    for q, B in enumerate(Bs):
        n, L = D.num_coeffs(B), 2 * B
        om = np.unique(np.concatenate([np.arange(min(n, 40)), np.arange(max(0, n - 200), n),
                                       np.arange(0, n, 1 if B < 10 else 53)]))
        ref = D.forward(ss[q].astype(np.complex128), B, omegas=om)
        ef = np.abs(f[co[q]:co[q] + n][om] - ref).max() / np.abs(ref).max()
        # every polar row j at a few (radius, azimuth) pairs
        ik = rng.integers(0, L, size=(3 if B > 40 else 6, 2))
        pts = np.array([(i, j, k) for i, k in ik for j in range(L)])
        sref = D.inverse(cs[q], B, points=pts)
        flat = (pts[:, 0] * L + pts[:, 1]) * L + pts[:, 2]
        ei = np.abs(s[so[q]:so[q] + D.num_samples(B)][flat] - sref).max() / np.abs(sref).max()
        print(f"copy-fed FP32 Legendre B={B}: forward e_inf {ef:.2e}, inverse e_inf {ei:.2e}", flush=True)
        assert ef <= 1e-5 and ei <= 1e-5, (B, ef, ei)
    p.destroy()
