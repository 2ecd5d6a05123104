"""Plan creation is all-or-nothing (the boundary's error convention): when a
device allocation fails part-way, sgl_plan_ex returns SGL_ERR_OOM, leaves the
output handle NULL and frees everything it had allocated.

The failure is injected from the host: SGL_TEST_FAIL_ALLOC=k makes the k-th
device allocation of one plan creation fail as hipMalloc does when memory runs
out (the library makes no device call for it), so no kernel sees a bad
pointer.  Every k from 1 up to the first creation that succeeds is tried, for
a plan that takes every allocating path (two bandlimits, shared tables,
seminaive constants, Bluestein constants, graph stream, autotuner scratch)."""

import ctypes
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1604_05140_amd import sgl  # noqa: E402

pytestmark = pytest.mark.gpu
SGL_ERR_OOM = 4


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _create(B_list, dtype, flags):
    lib = sgl._load()
    h = ctypes.c_void_p(12345)  # must be overwritten with NULL on failure
    arr = (ctypes.c_int * len(B_list))(*B_list)
    st = lib.sgl_plan_ex(ctypes.byref(h), arr, len(B_list), dtype, flags)
    return st, h


def _free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("B_list,dtype,flags", [
    ([16, 8, 8], sgl.SGL_F32, sgl.SGL_SEMINAIVE | sgl.SGL_AUTOTUNE | sgl.SGL_GRAPHS),
    ([12, 5], sgl.SGL_SPLIT_BF16, sgl.SGL_AUTOTUNE),
])
def test_failed_allocation_leaves_nothing(B_list, dtype, flags, monkeypatch):
    lib = sgl._load()
    print(f"all-or-nothing plan creation B={B_list} dtype={dtype} flags={flags}", flush=True)
    # first creation loads code objects and runtime pools; not part of the balance
    st, h = _create(B_list, dtype, flags)
    assert st == 0, sgl.status_name(st)
    lib.sgl_plan_destroy(h)
    base = _free_bytes()
    fails = 0
    for k in range(1, 400):
        monkeypatch.setenv("SGL_TEST_FAIL_ALLOC", str(k))
        st, h = _create(B_list, dtype, flags)
        monkeypatch.delenv("SGL_TEST_FAIL_ALLOC")
        if st == 0:
            lib.sgl_plan_destroy(h)
            break
        fails += 1
        assert st == SGL_ERR_OOM, (k, sgl.status_name(st), lib.sgl_last_error().decode())
        assert h.value is None, k
        assert _free_bytes() == base, k
    else:
        pytest.fail("plan creation never completed")
    assert fails >= 10, fails  # the plan makes many allocations; each failure point was tried
    assert _free_bytes() == base
    # the library is unharmed: a fresh plan recovers bandlimited coefficients
    p = sgl.sgl_plan_ex(B_list, dtype, 0)
    rng = np.random.default_rng(7)
    c = (rng.standard_normal(p.total_coeffs) + 1j * rng.standard_normal(p.total_coeffs)).astype(np.complex64)
    ct = torch.from_numpy(c).cuda()
    s = torch.empty(p.total_samples, dtype=p.complex_dtype, device="cuda")
    c2 = torch.empty_like(ct)
    sgl.sgl_inverse(p, ct, s)
    sgl.sgl_forward(p, s, c2)
    torch.cuda.synchronize()
    err = float((c2 - ct).abs().max() / ct.abs().max())
    p.destroy()
    assert err <= 1e-5, err
