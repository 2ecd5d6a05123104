"""GPU parity: libsgl (HIP, through the C ABI) against the CPU oracle.

Error metric (a reading of Sect. 4's relative error, which the paper does not
define further): e_inf = max|delta| / max|reference| per function.  Bars: FP64 1e-12 against the
oracle; FP32 1e-5 and split-bf16 1e-6 against the plain FP64 GPU path on the
same inputs (which is itself held to 1e-12 against the oracle).
"""

import ctypes
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import basis as BS, direct as D, quadrature as Q  # noqa: E402
from paper_1604_05140_amd import sgl, synth  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SEED = synth.BASE_SEED


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(x, ct):
    return torch.from_numpy(np.ascontiguousarray(x).reshape(-1)).to(DEV, ct)


def gpu_forward(plan, samples):
    out = torch.empty(plan.total_coeffs, dtype=plan.complex_dtype, device=DEV)
    s = samples if isinstance(samples, torch.Tensor) else dev(samples, plan.complex_dtype)
    sgl.sgl_forward(plan, s, out)
    torch.cuda.synchronize()
    return out


def gpu_inverse(plan, coeffs):
    out = torch.empty(plan.total_samples, dtype=plan.complex_dtype, device=DEV)
    c = coeffs if isinstance(coeffs, torch.Tensor) else dev(coeffs, plan.complex_dtype)
    sgl.sgl_inverse(plan, c, out)
    torch.cuda.synchronize()
    return out


def einf(ref, got):
    return D.error_metrics(np.asarray(ref), np.asarray(got))["e_inf"]


# ---------------------------------------------------------------------------
# GEMM core (MFMA lane layouts, ragged tiles, the three precisions)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-14), ("f32", 2e-6), ("split_bf16", 2e-6)])
@pytest.mark.parametrize("M,K,N", [(70, 45, 100), (64, 256, 128), (1, 1, 2), (130, 33, 17)])
def test_gemm_core(dtype, tol, M, K, N):
    g = np.random.default_rng(M * 1000 + K + N)
    A = g.standard_normal((M, K))
    X = g.standard_normal((K, N))
    ref = A @ X
    Ag, Xg = torch.from_numpy(A).to(DEV), torch.from_numpy(X).to(DEV)
    Cg = torch.full((M, N), float("nan"), dtype=torch.float64, device=DEV)
    sgl.sgl_debug_gemm(dtype, Ag, Xg, Cg)
    C = Cg.cpu().numpy()
    scale = np.abs(A).max() * np.abs(X).max() * math.sqrt(K)
    assert np.isfinite(C).all()
    assert np.abs(C - ref).max() <= tol * scale


# ---------------------------------------------------------------------------
# Plan-time FP64 grid and tables
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("B", [1, 2, 8, 17, 64, 128, 256])
def test_grid_matches_oracle(B):
    """The GPU rule (double-double Lanczos, Newton and Christoffel sums, rounded
    once to FP64) against the oracle's 40-digit rule rounded to FP64: nodes to a
    few units in the last place, ln a_i to a few ulps of its magnitude."""
    plan = sgl.sgl_plan(B, 1, "f64")
    g = plan.grid(B)
    o = Q.sgl_grid(B)
    rel_r = np.abs(g["r"] / o["r"] - 1)
    d_la = np.abs(g["log_a"] - o["log_a"]) / np.maximum(1.0, np.abs(o["log_a"]))
    d_ls = np.abs(g["log_sigma"] - o["log_sigma"]) / np.maximum(1.0, np.abs(o["log_sigma"]))
    print(f"B={B}: nodes max rel {rel_r.max():.2e}, ln a max {d_la.max():.2e}, ln sigma max {d_ls.max():.2e}",
          flush=True)
    assert rel_r.max() < 4e-15, rel_r.max()
    assert d_la.max() < 4e-15, d_la.max()
    assert d_ls.max() < 4e-15, d_ls.max()
    assert np.abs(g["theta"] - o["theta"]).max() < 1e-15
    assert np.abs(g["btilde"] / o["btilde"] - 1).max() < 1e-13
    plan.destroy()


def _oracle_tables(B):
    g = Q.sgl_grid(B)
    P = BS.legendre_table(B, g["theta"])
    R = BS.radial_table(B, g["r"], g["log_sigma"])
    Pt, Rt = [], []
    for m in range(B):
        Pt.append(P[m, m:B].reshape(-1))
    for l in range(B):
        Rt.append(R[l + 1:B + 1, l].reshape(-1))
    return np.concatenate(Pt), np.concatenate(Rt)


@pytest.mark.parametrize("B", [1, 3, 8, 64, 128, 256])
def test_tables_match_oracle(B):
    plan = sgl.sgl_plan(B, 1, "f64")
    Pg, Rg = plan.table(B, 0), plan.table(B, 1)
    Po, Ro = _oracle_tables(B)
    dP, dR = np.abs(Pg - Po).max(), np.abs(Rg - Ro).max()
    print(f"B={B}: Legendre table max abs diff {dP:.2e}, radial table {dR:.2e}", flush=True)
    # both sides run FP64 three-term recurrences of up to B steps on values up
    # to sqrt((2B-1)/(4 pi)) (Legendre) and 1 (radial, orthonormal rows), in a
    # different order of operations; rounding grows like B * eps * max|value|
    assert dP < 2e-15 * B * max(1.0, math.sqrt((2 * B - 1) / (4 * math.pi)))
    assert dR < 2e-15 * B
    plan.destroy()


@pytest.mark.parametrize("B", [8, 64, 128, 256])
def test_gpu_radial_rule_is_exact(B):
    """Thm. 3.3 for the GPU-built rule itself: sum_i a_i r_i^k = Gamma((k+1)/2)/2 for
    k <= 4B-1 (log-sum form, a_i underflows), and the GPU radial table has
    orthonormal rows (the iDRT identity, Sect. 3.3.2)."""
    plan = sgl.sgl_plan(B, 1, "f64")
    g = plan.grid(B)
    la, lr = g["log_a"], np.log(g["r"])
    for k in range(0, 4 * B, max(1, B // 8)):
        t = la + k * lr
        mx = t.max()
        lsum = mx + math.log(np.exp(t - mx).sum())
        assert abs(lsum - (math.lgamma((k + 1) / 2) - math.log(2.0))) < 1e-12 * max(1.0, abs(lsum)), k
    R = plan.table(B, 1)
    off = 0
    for l in range(B):
        blk = R[off:off + (B - l) * 2 * B].reshape(B - l, 2 * B)
        off += (B - l) * 2 * B
        assert np.abs(blk @ blk.T - np.eye(B - l)).max() < 1e-13, l  # 2B-term FP64 sums
    plan.destroy()


# ---------------------------------------------------------------------------
# FP64 transforms against the oracle
# ---------------------------------------------------------------------------
def test_fp64_config1_b8_recovers_coefficients():
    """B = 8, one function, CN(0,1) coefficients: oracle synthesis -> GPU forward
    recovers them; GPU inverse reproduces the oracle's samples."""
    B = 8
    c = synth.complex_normal_coeffs(B, 1, seed=SEED + 1)[0]
    s = D.inverse(c, B)
    plan = sgl.sgl_plan(B, 1, "f64")
    cg = gpu_forward(plan, s).cpu().numpy()
    sg = gpu_inverse(plan, c).cpu().numpy()
    assert einf(c, cg) <= 1e-12
    assert einf(s, sg) <= 1e-12
    assert einf(D.forward(s, B), cg) <= 1e-12


@pytest.mark.parametrize("B,batch", [(1, 1), (2, 3), (3, 2), (5, 2), (6, 1), (12, 2)])
def test_fp64_arbitrary_samples_and_coefficients(B, batch):
    """The forward map is the quadrature sum for any samples (not only bandlimited
    ones); the inverse is the synthesis sum for any coefficients."""
    s = synth.complex_normal_samples(B, batch, seed=SEED + 10 + B)
    c = synth.complex_normal_coeffs(B, batch, seed=SEED + 20 + B)
    plan = sgl.sgl_plan(B, batch, "f64")
    cg = gpu_forward(plan, s).cpu().numpy().reshape(batch, -1)
    sg = gpu_inverse(plan, c).cpu().numpy().reshape(batch, -1)
    for b in range(batch):
        assert einf(D.forward(s[b], B), cg[b]) <= 1e-12, b
        assert einf(D.inverse(c[b], B), sg[b]) <= 1e-12, b


def test_fp64_raw_samples():
    B = 7
    c = synth.complex_normal_coeffs(B, 1, seed=SEED + 30)[0]
    f = D.inverse(c, B, raw=True)
    plan = sgl.sgl_plan_ex([B], "f64", sgl.SGL_SAMPLES_RAW)
    cg = gpu_forward(plan, f).cpu().numpy()
    fg = gpu_inverse(plan, c).cpu().numpy()
    assert einf(c, cg) <= 1e-12
    assert einf(f, fg) <= 1e-12


@pytest.mark.parametrize("B", [65, 67, 127])
def test_fp64_512_point_rings(B):
    """Ring lengths 130..254 run Bluestein's convolution of length 512 on the
    one-wavefront 512-point kernels (the ragged column tail included: 2 x 2B
    columns are not a multiple of the 16 rings of a block): forward against the
    quadrature sum at seeded coefficients, inverse against the synthesis sum at
    seeded grid points, for arbitrary samples and coefficients."""
    batch = 2
    s = synth.complex_normal_samples(B, batch, seed=SEED + 110 + B)
    c = synth.complex_normal_coeffs(B, batch, seed=SEED + 120 + B)
    plan = sgl.sgl_plan(B, batch, "f64")
    assert plan.launch_grids()[1] > 0 and plan.launch_grids()[8] > 0
    cg = gpu_forward(plan, s).cpu().numpy().reshape(batch, -1)
    sg = gpu_inverse(plan, c).cpu().numpy().reshape(batch, -1)
    for b in range(batch):
        oms = synth.subset(6, D.num_coeffs(B), seed=SEED + 130 + b)
        f_or = D.forward(s[b], B, omegas=oms)
        assert np.abs(cg[b][oms] - f_or).max() <= 1e-12 * np.abs(cg[b]).max(), b
        pts = synth.grid_points(64, B, seed=SEED + 140 + b)
        s_or = D.inverse(c[b], B, points=pts)
        s_at = sg[b].reshape(2 * B, 2 * B, 2 * B)[pts[:, 0], pts[:, 1], pts[:, 2]]
        assert np.abs(s_at - s_or).max() <= 1e-12 * np.abs(sg[b]).max(), b
    plan.destroy()


def test_fp64_raw_samples_512_point_rings():
    """Raw samples through the 512-point kernels: synthesis of raw values and
    analysis back to the coefficients (B = 70, rings of 140 points)."""
    B = 70
    c = synth.complex_normal_coeffs(B, 1, seed=SEED + 150, decay=1.0)[0]
    plan = sgl.sgl_plan_ex([B], "f64", sgl.SGL_SAMPLES_RAW)
    f = gpu_inverse(plan, c)
    cg = gpu_forward(plan, f).cpu().numpy()
    assert einf(c, cg) <= 1e-12
    pts = synth.grid_points(32, B, seed=SEED + 151)
    f_or = D.inverse(c, B, points=pts, raw=True)
    f_at = f.cpu().numpy().reshape(2 * B, 2 * B, 2 * B)[pts[:, 0], pts[:, 1], pts[:, 2]]
    assert np.abs(f_at - f_or).max() <= 1e-12 * np.abs(f_or).max()
    plan.destroy()


def test_fp64_config2_b64_subsets_and_round_trip():
    """B = 64, batch 1, CN(0,1)/n: GPU inverse at 200 seeded grid points against
    the oracle's synthesis sum; round trip; GPU forward of seeded CN(0,1) samples
    at 200 seeded coefficients against the oracle's quadrature sum."""
    B = 64
    c = synth.complex_normal_coeffs(B, 1, seed=SEED + 2, decay=1.0)[0]
    plan = sgl.sgl_plan(B, 1, "f64")
    s_gpu = gpu_inverse(plan, c)
    s = s_gpu.cpu().numpy()
    pts = synth.grid_points(200, B, seed=SEED + 1002)
    s_or = D.inverse(c, B, points=pts)
    s_at = s.reshape(2 * B, 2 * B, 2 * B)[pts[:, 0], pts[:, 1], pts[:, 2]]
    assert np.abs(s_at - s_or).max() <= 1e-12 * np.abs(s_or).max()
    c2 = gpu_forward(plan, s_gpu).cpu().numpy()
    assert einf(c, c2) <= 1e-12
    s_arb = synth.complex_normal_samples(B, 1, seed=SEED + 1006)[0]
    c_arb = gpu_forward(plan, s_arb).cpu().numpy()
    oms = synth.subset(200, D.num_coeffs(B), seed=SEED + 1003)
    f_or = D.forward(s_arb, B, omegas=oms)
    assert np.abs(c_arb[oms] - f_or).max() <= 1e-12 * np.abs(f_or).max()


def test_batched_uneven_bandlimits_fp64():
    Bs = [3, 5, 3, 8, 1, 5]
    plan = sgl.sgl_plan_ex(Bs, "f64")
    so, co = plan.offsets()
    cs = [synth.complex_normal_coeffs(B, 1, seed=SEED + 40 + q)[0] for q, B in enumerate(Bs)]
    ss = [synth.complex_normal_samples(B, 1, seed=SEED + 50 + q)[0] for q, B in enumerate(Bs)]
    cg = gpu_forward(plan, np.concatenate(ss)).cpu().numpy()
    sg = gpu_inverse(plan, np.concatenate(cs)).cpu().numpy()
    for q, B in enumerate(Bs):
        assert einf(D.forward(ss[q], B), cg[co[q]:co[q] + D.num_coeffs(B)]) <= 1e-12
        assert einf(D.inverse(cs[q], B), sg[so[q]:so[q] + D.num_samples(B)]) <= 1e-12


# ---------------------------------------------------------------------------
# Precision forms against the plain FP64 GPU path
# ---------------------------------------------------------------------------
def einf_dev(ref, got):
    """e_inf on the device (large cases), in float64."""
    ref = ref.to(torch.complex128)
    got = got.to(torch.complex128)
    return float((got - ref).abs().max() / ref.abs().max())


def _precision_case(B, batch, decay, seed, dtypes=(("f32", 1e-5), ("split_bf16", 1e-6)), host_fn=0):
    c = synth.complex_normal_coeffs(B, batch, seed=seed, decay=decay)
    c_dev = dev(c, torch.complex128)
    p64 = sgl.sgl_plan(B, batch, "f64")
    s64 = gpu_inverse(p64, c_dev)
    c64 = gpu_forward(p64, s64)
    ns, nc = D.num_samples(B), D.num_coeffs(B)
    for b in range(batch):
        assert einf_dev(c_dev[b * nc:(b + 1) * nc], c64[b * nc:(b + 1) * nc]) <= 1e-12
    res = {}
    s32 = s64.to(torch.complex64)
    c32 = c_dev.to(torch.complex64)
    for dtype, tol in dtypes:
        p = sgl.sgl_plan(B, batch, dtype)
        cf = gpu_forward(p, s32)
        sf = gpu_inverse(p, c32)
        ef = max(einf_dev(c64[b * nc:(b + 1) * nc], cf[b * nc:(b + 1) * nc]) for b in range(batch))
        ei = max(einf_dev(s64[b * ns:(b + 1) * ns], sf[b * ns:(b + 1) * ns]) for b in range(batch))
        res[dtype] = (ef, ei)
        print(f"B={B} batch={batch} {dtype}: forward e_inf {ef:.2e}, inverse e_inf {ei:.2e}", flush=True)
        assert ef <= tol and ei <= tol, (dtype, ef, ei)
        del cf, sf
        p.destroy()
    s_host = s64[host_fn * ns:(host_fn + 1) * ns].cpu().numpy()
    del s64, c64, s32
    p64.destroy()
    torch.cuda.empty_cache()
    return c, s_host, res


def test_precision_forms_uneven_bandlimits():
    """Reduced-precision plans over functions of uneven bandlimits (work items of
    1 to 5 contraction chunks, ragged column tiles, items of different classes in
    one persistent launch) against the FP64 plan on the same inputs; the FP64
    results of the largest function checked against the oracle on seeded subsets."""
    Bs = [5, 17, 40, 3, 64, 9, 33, 70]
    p64 = sgl.sgl_plan_ex(Bs, "f64")
    so, co = p64.offsets()
    cs = [synth.complex_normal_coeffs(B, 1, seed=SEED + 300 + q, decay=1.0)[0] for q, B in enumerate(Bs)]
    c_all = np.concatenate(cs)
    s64 = gpu_inverse(p64, dev(c_all, torch.complex128))
    c64 = gpu_forward(p64, s64)
    q = Bs.index(70)
    s_host = s64[so[q]:so[q] + D.num_samples(70)].cpu().numpy()
    pts = synth.grid_points(12, 70, seed=SEED + 310)
    ref = D.inverse(cs[q], 70, points=pts)
    assert np.abs(s_host[psi_of(pts, 70)] - ref).max() <= 1e-12 * np.abs(ref).max()
    oms = synth.subset(40, D.num_coeffs(70), seed=SEED + 311)
    f_or = D.forward(s_host, 70, omegas=oms)
    c_host = c64[co[q]:co[q] + D.num_coeffs(70)].cpu().numpy()
    assert np.abs(c_host[oms] - f_or).max() <= 1e-12 * np.abs(f_or).max()
    for dtype, tol in (("f32", 1e-5), ("split_bf16", 1e-6)):
        for flags in (0, sgl.SGL_AUTOTUNE | sgl.SGL_GRAPHS):
            p = sgl.sgl_plan_ex(Bs, dtype, flags)
            cf = gpu_forward(p, s64.to(torch.complex64))
            sf = gpu_inverse(p, dev(c_all, torch.complex64))
            for q, B in enumerate(Bs):
                ns, nc = D.num_samples(B), D.num_coeffs(B)
                ef = einf_dev(c64[co[q]:co[q] + nc], cf[co[q]:co[q] + nc])
                ei = einf_dev(s64[so[q]:so[q] + ns], sf[so[q]:so[q] + ns])
                assert ef <= tol and ei <= tol, (dtype, flags, B, ef, ei)
            p.destroy()
    p64.destroy()


def psi_of(pts, B):
    """psi index of (i, j, k) grid triples (Sect. 3.4 ordering)."""
    return (pts[:, 0] * 2 * B + pts[:, 1]) * 2 * B + pts[:, 2]


def test_precision_forms_small_b():
    _precision_case(12, 3, 1.0, SEED + 60)


def test_precision_forms_config3_b128():
    """B = 128, batch 4, CN(0,1)/n: FP32 MFMA (1e-5) and split-bf16 (1e-6) against
    FP64; the FP64 synthesis of function 1 checked against the oracle's synthesis
    of the same seeded coefficients at 24 seeded grid points."""
    B, batch = 128, 4
    c, s1, _ = _precision_case(B, batch, 1.0, SEED + 3, host_fn=1)
    pts = synth.grid_points(24, B, seed=SEED + 1004)
    ref = D.inverse(c[1], B, points=pts)
    assert np.abs(s1[psi_of(pts, B)] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_precision_config5_b256_split():
    """B = 256, batch 8, CN(0,1) n^-1.5: split-bf16 against FP64 (1e-6)."""
    B, batch = 256, 8
    c, s0, _ = _precision_case(B, batch, 1.5, SEED + 5, dtypes=(("split_bf16", 1e-6),), host_fn=0)
    pts = synth.grid_points(6, B, seed=SEED + 1005)
    ref = D.inverse(c[0], B, points=pts)
    assert np.abs(s0[psi_of(pts, B)] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_bench_launch_configuration_split_vs_oracle():
    """The timed configuration of the benchmark: B = 128, batch 4, split-bf16 plan
    built with SGL_AUTOTUNE | SGL_GRAPHS, eager capture and a graph replay.
    Forward: seeded CN(0,1) samples (rounded to complex64, the same values fed
    to the oracle) at 24 seeded coefficients of function 2 against the oracle's
    quadrature sums, 1e-6 of the largest of those 24.  Inverse: seeded
    CN(0,1)/n coefficients (complex64) at 24 seeded grid points of function 3
    against the oracle's synthesis, 1e-6 of the largest sample magnitude (the
    e_inf denominator, taken from the FP64 GPU synthesis of the same
    coefficients, itself pinned to the oracle above)."""
    B, batch = 128, 4
    ns, nc = D.num_samples(B), D.num_coeffs(B)
    s = synth.complex_normal_samples(B, batch, seed=SEED + 2001).astype(np.complex64)
    c = synth.complex_normal_coeffs(B, batch, seed=SEED + 2002, decay=1.0).astype(np.complex64)
    plan = sgl.sgl_plan_ex([B] * batch, "split_bf16", sgl.SGL_AUTOTUNE | sgl.SGL_GRAPHS)
    s_dev, c_dev = dev(s, torch.complex64), dev(c, torch.complex64)
    oms = synth.subset(24, nc, seed=SEED + 2003)
    f_ref = D.forward(s[2].astype(np.complex128), B, omegas=oms)
    pts = synth.grid_points(24, B, seed=SEED + 2004)
    s_ref = D.inverse(c[3].astype(np.complex128), B, points=pts)
    p64 = sgl.sgl_plan(B, 1, "f64")
    smax = float(gpu_inverse(p64, dev(c[3], torch.complex128)).abs().max())
    p64.destroy()
    for call in range(2):  # capture, then replay
        cf = gpu_forward(plan, s_dev)[2 * nc:3 * nc].cpu().numpy()
        sf = gpu_inverse(plan, c_dev)[3 * ns:4 * ns].cpu().numpy()
        ef = np.abs(cf[oms] - f_ref).max() / np.abs(f_ref).max()
        ei = np.abs(sf[psi_of(pts, B)] - s_ref).max() / smax
        print(f"bench configuration, call {call}: forward {ef:.2e}, inverse {ei:.2e}", flush=True)
        assert ef <= 1e-6 and ei <= 1e-6, (call, ef, ei)
    plan.destroy()


# ---------------------------------------------------------------------------
# hipGraph replay and the plan-time autotuner
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f64", "split_bf16"])
def test_graph_replays_match_eager(dtype):
    """SGL_GRAPHS: every replay equals the eager launch sequence on the same inputs,
    with eager work (another plan, torch kernels) and input changes in between."""
    B, batch = 12, 2
    eager = sgl.sgl_plan(B, batch, dtype)
    graph = sgl.sgl_plan_ex([B] * batch, dtype, sgl.SGL_GRAPHS)
    ct = eager.complex_dtype
    s_in = torch.empty(eager.total_samples, dtype=ct, device=DEV)
    c_in = torch.empty(eager.total_coeffs, dtype=ct, device=DEV)
    c_out = torch.empty(eager.total_coeffs, dtype=ct, device=DEV)
    s_out = torch.empty(eager.total_samples, dtype=ct, device=DEV)
    for rep in range(4):
        s_in.copy_(dev(synth.complex_normal_samples(B, batch, seed=SEED + 70 + rep), ct))
        c_in.copy_(dev(synth.complex_normal_coeffs(B, batch, seed=SEED + 80 + rep), ct))
        ref_c = gpu_forward(eager, s_in)
        ref_s = gpu_inverse(eager, c_in)
        _ = (torch.randn(1 << 20, device=DEV) * 2).sum()  # unrelated eager work
        sgl.sgl_forward(graph, s_in, c_out)
        sgl.sgl_inverse(graph, c_in, s_out)
        torch.cuda.synchronize()
        assert torch.equal(c_out, ref_c), rep
        assert torch.equal(s_out, ref_s), rep
    # a second buffer pair is captured separately and does not disturb the first
    c_out2 = torch.empty_like(c_out)
    sgl.sgl_forward(graph, s_in, c_out2)
    sgl.sgl_forward(graph, s_in, c_out)
    torch.cuda.synchronize()
    assert torch.equal(c_out2, c_out)


def test_graph_cache_eviction_and_caller_streams():
    """SGL_GRAPHS keeps at most eight instantiated graphs: ten output buffers used in
    turn (each call a capture or a replay after eviction) all equal the eager result,
    on the default stream and on a caller-created stream."""
    B, batch = 16, 1
    eager = sgl.sgl_plan(B, batch, "split_bf16")
    graph = sgl.sgl_plan_ex([B] * batch, "split_bf16", sgl.SGL_GRAPHS)
    ct = eager.complex_dtype
    s_in = dev(synth.complex_normal_samples(B, batch, seed=SEED + 95), ct)
    c_in = dev(synth.complex_normal_coeffs(B, batch, seed=SEED + 96), ct)
    ref_c = gpu_forward(eager, s_in)
    ref_s = gpu_inverse(eager, c_in)
    outs_c = [torch.empty(graph.total_coeffs, dtype=ct, device=DEV) for _ in range(10)]
    outs_s = [torch.empty(graph.total_samples, dtype=ct, device=DEV) for _ in range(10)]
    side = torch.cuda.Stream()
    for rnd in range(2):
        for q in range(10):
            for o in (outs_c[q], outs_s[q]):
                o.fill_(float("nan"))
            st = side if (q + rnd) % 2 else None
            if st is not None:
                st.wait_stream(torch.cuda.current_stream())
            sgl.sgl_forward(graph, s_in, outs_c[q], st)
            sgl.sgl_inverse(graph, c_in, outs_s[q], st)
            if st is not None:
                torch.cuda.current_stream().wait_stream(st)
            torch.cuda.synchronize()
            assert torch.equal(outs_c[q], ref_c), (rnd, q)
            assert torch.equal(outs_s[q], ref_s), (rnd, q)
    graph.destroy()
    eager.destroy()


def test_call_argument_errors_leave_outputs_untouched():
    """Through the C ABI on a live plan: null data pointers and overlapping input and
    output are rejected with SGL_ERR_INVALID_ARG, the naive transforms of a non-FP64
    plan with SGL_ERR_UNSUPPORTED, and no output element is written."""
    lib = sgl._load()
    B = 8
    plan = sgl.sgl_plan(B, 1, "split_bf16")
    ct = plan.complex_dtype
    s = dev(synth.complex_normal_samples(B, 1, seed=SEED + 97), ct)
    c = torch.full((plan.total_coeffs,), 7.0, dtype=ct, device=DEV)
    buf = torch.zeros(plan.total_samples + plan.total_coeffs, dtype=ct, device=DEV)
    torch.cuda.synchronize()
    P = ctypes.c_void_p
    h, st = plan.handle, P(torch.cuda.current_stream().cuda_stream)
    assert lib.sgl_forward(h, None, P(c.data_ptr()), st) == 1
    assert b"null" in lib.sgl_last_error()
    assert lib.sgl_inverse(h, P(c.data_ptr()), None, st) == 1
    # output overlapping the input: coefficients written over the samples' tail
    over = buf.data_ptr() + (plan.total_samples - 1) * buf.element_size()
    assert lib.sgl_forward(h, P(buf.data_ptr()), P(over), st) == 1
    assert b"overlap" in lib.sgl_last_error()
    assert lib.sgl_naive_forward(h, P(s.data_ptr()), P(c.data_ptr()), st) == 2
    torch.cuda.synchronize()
    assert bool((c == 7.0).all()) and bool((buf == 0).all())
    plan.destroy()


def test_autotuned_plan_matches_default():
    B, batch = 16, 3
    s = synth.complex_normal_samples(B, batch, seed=SEED + 90)
    c = synth.complex_normal_coeffs(B, batch, seed=SEED + 91)
    for dtype in ("f64", "split_bf16"):
        p0 = sgl.sgl_plan(B, batch, dtype)
        p1 = sgl.sgl_plan_ex([B] * batch, dtype, sgl.SGL_AUTOTUNE | sgl.SGL_GRAPHS)
        grids = p1.launch_grids()
        assert len(grids) == sgl.SGL_NUM_SLOTS
        # B = 16: 32-point rings (slot 0 / 7); no 512-point or Bluestein rings
        assert all(g >= 1 for g in grids[:1] + grids[3:8]), grids
        assert grids[1] == grids[2] == grids[8] == grids[9] == 0, grids
        assert torch.equal(gpu_forward(p0, s), gpu_forward(p1, s))
        assert torch.equal(gpu_inverse(p0, c), gpu_inverse(p1, c))


# ---------------------------------------------------------------------------
# Batched form: uneven bandlimits through one launch per stage
# ---------------------------------------------------------------------------
def test_batched_config4_256_functions_f32():
    """256 functions with bandlimits uniform in {16..96}, CN(0,1)/n coefficients:
    FP32 MFMA batched plan (autotuned, graphs) against the FP64 batched plan
    (1e-5), and the FP64 plan against the oracle on a few coefficients."""
    Bs = synth.batched_bandlimits(256, 16, 96, seed=SEED + 4)
    p64 = sgl.sgl_plan_ex(list(Bs), "f64")
    p32 = sgl.sgl_plan_ex(list(Bs), "f32", sgl.SGL_AUTOTUNE | sgl.SGL_GRAPHS)
    so, co = p64.offsets()
    cs = [synth.complex_normal_coeffs(int(B), 1, seed=SEED + 4000 + q, decay=1.0)[0] for q, B in enumerate(Bs)]
    c_dev = dev(np.concatenate(cs), torch.complex128)
    s64 = gpu_inverse(p64, c_dev)
    c64 = gpu_forward(p64, s64)
    s32 = gpu_inverse(p32, c_dev.to(torch.complex64))
    c32 = gpu_forward(p32, s64.to(torch.complex64))
    worst_f = worst_i = worst_rt = 0.0
    for q, B in enumerate(Bs):
        nc, ns = D.num_coeffs(int(B)), D.num_samples(int(B))
        cr = c_dev[co[q]:co[q] + nc]
        worst_rt = max(worst_rt, einf_dev(cr, c64[co[q]:co[q] + nc]))
        worst_f = max(worst_f, einf_dev(c64[co[q]:co[q] + nc], c32[co[q]:co[q] + nc]))
        worst_i = max(worst_i, einf_dev(s64[so[q]:so[q] + ns], s32[so[q]:so[q] + ns]))
    print(f"config4: FP64 round trip {worst_rt:.2e}; FP32 forward {worst_f:.2e}, inverse {worst_i:.2e}", flush=True)
    assert worst_rt <= 1e-12
    assert worst_f <= 1e-5 and worst_i <= 1e-5
    # oracle spot check on the two smallest functions: FP64 synthesis at seeded
    # grid points against the oracle's synthesis of the same coefficients
    for q in np.argsort(Bs)[:2]:
        B = int(Bs[q])
        pts = synth.grid_points(8, B, seed=SEED + 4100 + int(q))
        s_or = D.inverse(cs[q], B, points=pts)
        got = s64[so[q]:so[q] + D.num_samples(B)].cpu().numpy()[psi_of(pts, B)]
        assert np.abs(got - s_or).max() <= 1e-12 * np.abs(s_or).max()
