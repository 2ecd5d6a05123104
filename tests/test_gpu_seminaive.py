"""GPU parity of the seminaive Legendre step (SGL_SEMINAIVE plans, Sect. 3.3.1).

The cosine-domain table against the oracle's (oracle/seminaive.py); whole FP64
transforms against the quadrature and synthesis sums of the direct oracle at
small B; at larger B and in the FP32 / split-bf16 forms against the plain FP64
GPU path (itself held to 1e-12 against the oracle), with the bars of the
direct path: FP64 1e-12, FP32 1e-5, split-bf16 1e-6 (e_inf per function).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import direct as D, seminaive as S  # noqa: E402
from paper_1604_05140_amd import sgl, synth  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SEED = synth.BASE_SEED + 500


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(x, ct):
    return torch.from_numpy(np.ascontiguousarray(x).reshape(-1)).to(DEV, ct)


def run(plan, x, forward):
    n = plan.total_coeffs if forward else plan.total_samples
    out = torch.empty(n, dtype=plan.complex_dtype, device=DEV)
    xin = x if isinstance(x, torch.Tensor) else dev(x, plan.complex_dtype)
    (sgl.sgl_forward if forward else sgl.sgl_inverse)(plan, xin, out)
    torch.cuda.synchronize()
    return out


def einf_dev(ref, got):
    ref = ref.to(torch.complex128)
    got = got.to(torch.complex128)
    return float((got - ref).abs().max() / ref.abs().max())


@pytest.mark.parametrize("B", [8, 32])
def test_cosine_legendre_table_matches_oracle(B):
    plan = sgl.sgl_plan_ex([B], "f64", sgl.SGL_SEMINAIVE)
    got = plan.table(B, 2)
    T = S.get_tables(B)
    off = 0
    for m in range(B):
        blk = got[off:off + (B - m) * B].reshape(B - m, B)
        off += (B - m) * B
        ref = T.Cq[m, m:B, :B].copy()
        for r in range(B - m):  # the table stops at the degree l - par
            ref[r, m + r - S.parity(m) + 1:] = 0.0
        assert np.abs(blk - ref).max() < 1e-12, m
    plan.destroy()


@pytest.mark.parametrize("B,batch", [(8, 2), (16, 1)])
def test_fp64_seminaive_matches_quadrature_sums(B, batch):
    s = synth.complex_normal_samples(B, batch, seed=SEED + B)
    c = synth.complex_normal_coeffs(B, batch, seed=SEED + 10 + B)
    plan = sgl.sgl_plan_ex([B] * batch, "f64", sgl.SGL_SEMINAIVE)
    cg = run(plan, s, True).cpu().numpy().reshape(batch, -1)
    sg = run(plan, c, False).cpu().numpy().reshape(batch, -1)
    for b in range(batch):
        ref_c = D.forward(s[b], B)
        assert np.abs(cg[b] - ref_c).max() <= 1e-12 * np.abs(ref_c).max(), b
        ref_s = D.inverse(c[b], B)
        assert np.abs(sg[b] - ref_s).max() <= 1e-12 * np.abs(ref_s).max(), b
    plan.destroy()


def test_fp64_seminaive_matches_direct_plan_uneven_batch():
    """Several bandlimit classes in one seminaive plan, odd and even orders,
    arbitrary samples and coefficients, against the direct FP64 plan."""
    Bs = [8, 64, 16, 64, 32]
    direct = sgl.sgl_plan_ex(Bs, "f64")
    semi = sgl.sgl_plan_ex(Bs, "f64", sgl.SGL_SEMINAIVE)
    so, co = direct.offsets()
    s = np.concatenate([synth.complex_normal_samples(B, 1, seed=SEED + 100 + q)[0] for q, B in enumerate(Bs)])
    c = np.concatenate([synth.complex_normal_coeffs(B, 1, seed=SEED + 200 + q)[0] for q, B in enumerate(Bs)])
    s_dev, c_dev = dev(s, torch.complex128), dev(c, torch.complex128)
    cd, cs = run(direct, s_dev, True), run(semi, s_dev, True)
    sd, ss = run(direct, c_dev, False), run(semi, c_dev, False)
    for q, B in enumerate(Bs):
        nc, ns = D.num_coeffs(B), D.num_samples(B)
        assert einf_dev(cd[co[q]:co[q] + nc], cs[co[q]:co[q] + nc]) <= 1e-12, (q, B)
        assert einf_dev(sd[so[q]:so[q] + ns], ss[so[q]:so[q] + ns]) <= 1e-12, (q, B)
    direct.destroy()
    semi.destroy()


@pytest.mark.parametrize("B,batch", [(128, 2), (256, 1)])
def test_fp64_seminaive_large_b(B, batch):
    """B = 128 (16-column DCT tiles) and B = 256 (8-column tiles in FP64):
    round trip of CN(0,1)/n coefficients and agreement with the direct plan."""
    c = synth.complex_normal_coeffs(B, batch, seed=SEED + 300 + B, decay=1.0)
    c_dev = dev(c, torch.complex128)
    semi = sgl.sgl_plan_ex([B] * batch, "f64", sgl.SGL_SEMINAIVE)
    s_semi = run(semi, c_dev, False)
    c_back = run(semi, s_semi, True)
    nc, ns = D.num_coeffs(B), D.num_samples(B)
    for b in range(batch):
        assert einf_dev(c_dev[b * nc:(b + 1) * nc], c_back[b * nc:(b + 1) * nc]) <= 1e-12, b
    semi.destroy()
    direct = sgl.sgl_plan(B, batch, "f64")
    s_dir = run(direct, c_dev, False)
    for b in range(batch):
        assert einf_dev(s_dir[b * ns:(b + 1) * ns], s_semi[b * ns:(b + 1) * ns]) <= 1e-12, b
    direct.destroy()


@pytest.mark.parametrize("dtype,tol,copy_fed", [("f32", 1e-5, False), ("f32", 1e-5, True), ("split_bf16", 1e-6, False)])
def test_seminaive_precision_forms(dtype, tol, copy_fed):
    """B = 128, batch 2, CN(0,1)/n: the FP32 and split-bf16 seminaive forms
    against the FP64 direct path (the bars of the direct forms); FP32 also with
    its Legendre slots (cosine-domain contraction length B) and forward radial
    slot on the copy-fed kernels."""
    B, batch = 128, 2
    c = synth.complex_normal_coeffs(B, batch, seed=SEED + 400, decay=1.0)
    c_dev = dev(c, torch.complex128)
    p64 = sgl.sgl_plan(B, batch, "f64")
    s64 = run(p64, c_dev, False)
    c64 = run(p64, s64, True)
    p = sgl.sgl_plan_ex([B] * batch, dtype, sgl.SGL_SEMINAIVE)
    if copy_fed:
        for slot in (3, 4, 6):
            p.set_launch_tile(slot, 2)
            assert p.launch_tiles()[slot] == (128, 128)
    cf = run(p, s64.to(torch.complex64), True)
    sf = run(p, c_dev.to(torch.complex64), False)
    nc, ns = D.num_coeffs(B), D.num_samples(B)
    ef = max(einf_dev(c64[b * nc:(b + 1) * nc], cf[b * nc:(b + 1) * nc]) for b in range(batch))
    ei = max(einf_dev(s64[b * ns:(b + 1) * ns], sf[b * ns:(b + 1) * ns]) for b in range(batch))
    print(f"seminaive {dtype} copy_fed={copy_fed}: forward e_inf {ef:.2e}, inverse e_inf {ei:.2e}", flush=True)
    assert ef <= tol and ei <= tol
    p.destroy()
    p64.destroy()


def test_seminaive_graph_replays_match_eager():
    B, batch = 32, 2
    eager = sgl.sgl_plan_ex([B] * batch, "split_bf16", sgl.SGL_SEMINAIVE)
    graph = sgl.sgl_plan_ex([B] * batch, "split_bf16", sgl.SGL_SEMINAIVE | sgl.SGL_GRAPHS | sgl.SGL_AUTOTUNE)
    ct = eager.complex_dtype
    s_in = dev(synth.complex_normal_samples(B, batch, seed=SEED + 600), ct)
    c_in = dev(synth.complex_normal_coeffs(B, batch, seed=SEED + 601), ct)
    ref_c, ref_s = run(eager, s_in, True), run(eager, c_in, False)
    for rep in range(3):
        _ = (torch.randn(1 << 20, device=DEV) * 2).sum()  # unrelated eager work
        assert torch.equal(run(graph, s_in, True), ref_c), rep
        assert torch.equal(run(graph, c_in, False), ref_s), rep
    eager.destroy()
    graph.destroy()
