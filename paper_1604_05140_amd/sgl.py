"""Thin ctypes binding of libsgl (include/sgl.h).

Argument marshalling only: every step of the transform runs in libsgl's HIP
kernels.  Device buffers are torch tensors (torch supplies device memory and
streams); each call passes tensor.data_ptr() and the current HIP stream.  If
libsgl.so is missing or fails to load, every entry point raises: there is no
fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgl.so")

SGL_F64, SGL_F32, SGL_SPLIT_BF16 = 0, 1, 2
SGL_SAMPLES_RAW = 1
SGL_GRAPHS = 2
SGL_AUTOTUNE = 4
SGL_SEMINAIVE = 8
SGL_MAX_B = 256
SGL_NUM_SLOTS = 10
DTYPES = {"f64": SGL_F64, "f32": SGL_F32, "split_bf16": SGL_SPLIT_BF16}

_lib = None


class SglError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {status_name(status)} ({msg})")
        self.status = status


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libsgl.so not built ({LIB_PATH} missing); run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64p = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "sgl_plan": ([ctypes.POINTER(P), ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "sgl_plan_ex": ([ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int,
                         ctypes.c_uint], ctypes.c_int),
        "sgl_plan_scaled": ([ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int,
                             ctypes.c_uint, ctypes.c_double], ctypes.c_int),
        "sgl_forward": ([P, P, P, P], ctypes.c_int),
        "sgl_inverse": ([P, P, P, P], ctypes.c_int),
        "sgl_forward_noalloc": ([P, P, P, P], ctypes.c_int),
        "sgl_naive_forward": ([P, P, P, P], ctypes.c_int),
        "sgl_naive_inverse": ([P, P, P, P], ctypes.c_int),
        "sgl_midpoint_forward": ([P, P, ctypes.c_int, ctypes.c_double, P, P], ctypes.c_int),
        "sgl_synthesize_points": ([P, P, ctypes.c_int, P, P, P], ctypes.c_int),
        "sgl_plan_destroy": ([P], ctypes.c_int),
        "sgl_num_samples": ([ctypes.c_int], ctypes.c_int64),
        "sgl_num_coeffs": ([ctypes.c_int], ctypes.c_int64),
        "sgl_coeff_index": ([ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int64),
        "sgl_plan_info": ([P, i64p, i64p, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "sgl_offsets": ([P, i64p, i64p], ctypes.c_int),
        "sgl_grid": ([P, ctypes.c_int, dp, dp, dp, dp, dp], ctypes.c_int),
        "sgl_table": ([P, ctypes.c_int, ctypes.c_int, dp], ctypes.c_int),
        "sgl_set_timing": ([P, ctypes.c_int], ctypes.c_int),
        "sgl_launch_grids": ([P, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "sgl_launch_tiles": ([P, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "sgl_set_launch_tile": ([P, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "sgl_stage_times": ([P, dp, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "sgl_debug_gemm": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P], ctypes.c_int),
        "sgl_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "sgl_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def exported_symbols():
    """Names declared in include/sgl.h that the loaded library resolves."""
    lib = _load()
    return [n for n in _HEADER_NAMES if hasattr(lib, n)]


_HEADER_NAMES = [
    "sgl_plan", "sgl_plan_ex", "sgl_forward", "sgl_inverse", "sgl_plan_destroy", "sgl_num_samples",
    "sgl_num_coeffs", "sgl_coeff_index", "sgl_plan_info", "sgl_offsets", "sgl_grid", "sgl_table",
    "sgl_set_timing", "sgl_stage_times", "sgl_debug_gemm", "sgl_status_string", "sgl_last_error",
    "sgl_launch_grids", "sgl_naive_forward", "sgl_naive_inverse", "sgl_plan_scaled",
    "sgl_midpoint_forward", "sgl_synthesize_points", "sgl_launch_tiles", "sgl_set_launch_tile",
    "sgl_forward_noalloc",
]


def status_name(st: int) -> str:
    try:
        return _load().sgl_status_string(st).decode()
    except Exception:  # pragma: no cover - library missing
        return str(st)


def _check(st: int, where: str):
    if st != 0:
        raise SglError(st, where, _load().sgl_last_error().decode())


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def sgl_num_samples(B: int) -> int:
    return int(_load().sgl_num_samples(B))


def sgl_num_coeffs(B: int) -> int:
    return int(_load().sgl_num_coeffs(B))


def sgl_coeff_index(n: int, l: int, m: int) -> int:
    return int(_load().sgl_coeff_index(n, l, m))


class Plan:
    """Owning wrapper of an sgl_plan_t."""

    def __init__(self, handle, dtype):
        self._h = handle
        self.dtype = dtype
        lib = _load()
        ts, tc, nf = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
        _check(lib.sgl_plan_info(self._h, ctypes.byref(ts), ctypes.byref(tc), ctypes.byref(nf)), "sgl_plan_info")
        self.total_samples, self.total_coeffs, self.nfunc = ts.value, tc.value, nf.value

    @property
    def handle(self):
        return self._h

    @property
    def complex_dtype(self):
        import torch
        return torch.complex128 if self.dtype == SGL_F64 else torch.complex64

    def offsets(self):
        so = (ctypes.c_int64 * self.nfunc)()
        co = (ctypes.c_int64 * self.nfunc)()
        _check(_load().sgl_offsets(self._h, so, co), "sgl_offsets")
        return np.array(so[:], dtype=np.int64), np.array(co[:], dtype=np.int64)

    def grid(self, B: int):
        L = 2 * B
        arrs = [np.zeros(L) for _ in range(5)]
        ptrs = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs]
        _check(_load().sgl_grid(self._h, B, *ptrs), "sgl_grid")
        return dict(zip(["r", "log_a", "log_sigma", "theta", "btilde"], arrs))

    def table(self, B: int, which: int) -> np.ndarray:
        out = np.zeros(B * B * (B + 1) // (2 if which == 2 else 1))
        _check(_load().sgl_table(self._h, B, which, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "sgl_table")
        return out

    def launch_grids(self):
        g = (ctypes.c_int * SGL_NUM_SLOTS)()
        _check(_load().sgl_launch_grids(self._h, g), "sgl_launch_grids")
        return list(g)

    def launch_tiles(self):
        """Per launch slot: (rows, complex columns) of a work item's tile ((0, 0) for FFT slots)."""
        t = (ctypes.c_int * (2 * SGL_NUM_SLOTS))()
        _check(_load().sgl_launch_tiles(self._h, t), "sgl_launch_tiles")
        return [(t[2 * q], t[2 * q + 1]) for q in range(SGL_NUM_SLOTS)]

    def set_launch_tile(self, slot: int, geometry: int):
        _check(_load().sgl_set_launch_tile(self._h, int(slot), int(geometry)), "sgl_set_launch_tile")

    def set_timing(self, enable: bool):
        _check(_load().sgl_set_timing(self._h, 1 if enable else 0), "sgl_set_timing")

    def stage_times(self):
        ms = (ctypes.c_double * 6)()
        cnt = (ctypes.c_int * 6)()
        _check(_load().sgl_stage_times(self._h, ms, cnt), "sgl_stage_times")
        return list(ms), list(cnt)

    def _check_tensor(self, t, n, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != self.complex_dtype or not t.is_contiguous() or t.numel() < n:
            raise ValueError(f"{name} must be a contiguous {self.complex_dtype} tensor of >= {n} elements")

    def forward(self, samples, coeffs, stream=None):
        sgl_forward(self, samples, coeffs, stream)

    def inverse(self, coeffs, samples, stream=None):
        sgl_inverse(self, coeffs, samples, stream)

    def destroy(self):
        if self._h:
            _load().sgl_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def sgl_plan(B: int, batch: int = 1, dtype=SGL_F64) -> Plan:
    lib = _load()
    dtype = DTYPES.get(dtype, dtype)
    h = ctypes.c_void_p()
    _check(lib.sgl_plan(ctypes.byref(h), int(B), int(batch), int(dtype)), "sgl_plan")
    return Plan(h, dtype)


def sgl_plan_ex(B_list, dtype=SGL_F64, flags: int = 0) -> Plan:
    lib = _load()
    dtype = DTYPES.get(dtype, dtype)
    arr = (ctypes.c_int * len(B_list))(*[int(b) for b in B_list])
    h = ctypes.c_void_p()
    _check(lib.sgl_plan_ex(ctypes.byref(h), arr, len(B_list), int(dtype), ctypes.c_uint(flags)), "sgl_plan_ex")
    return Plan(h, dtype)


def sgl_plan_scaled(B_list, dtype=SGL_F64, flags: int = 0, radial_scale: float = 1.0) -> Plan:
    """Plan for the radially scaled basis H^s_nlm(x) = s^(-3/2) H_nlm(x/s)."""
    lib = _load()
    dtype = DTYPES.get(dtype, dtype)
    arr = (ctypes.c_int * len(B_list))(*[int(b) for b in B_list])
    h = ctypes.c_void_p()
    _check(lib.sgl_plan_scaled(ctypes.byref(h), arr, len(B_list), int(dtype), ctypes.c_uint(flags),
                               ctypes.c_double(radial_scale)), "sgl_plan_scaled")
    return Plan(h, dtype)


def sgl_forward(plan: Plan, samples, coeffs, stream=None):
    plan._check_tensor(samples, plan.total_samples, "samples")
    plan._check_tensor(coeffs, plan.total_coeffs, "coeffs")
    _check(_load().sgl_forward(plan.handle, ctypes.c_void_p(samples.data_ptr()), ctypes.c_void_p(coeffs.data_ptr()),
                               _stream_handle(stream)), "sgl_forward")


def sgl_forward_noalloc(plan: Plan, samples, coeffs, stream=None):
    """sgl_forward on the library's static per-GPU workspace (allocates nothing)."""
    plan._check_tensor(samples, plan.total_samples, "samples")
    plan._check_tensor(coeffs, plan.total_coeffs, "coeffs")
    _check(_load().sgl_forward_noalloc(plan.handle, ctypes.c_void_p(samples.data_ptr()),
                                       ctypes.c_void_p(coeffs.data_ptr()), _stream_handle(stream)),
           "sgl_forward_noalloc")


def sgl_inverse(plan: Plan, coeffs, samples, stream=None):
    plan._check_tensor(coeffs, plan.total_coeffs, "coeffs")
    plan._check_tensor(samples, plan.total_samples, "samples")
    _check(_load().sgl_inverse(plan.handle, ctypes.c_void_p(coeffs.data_ptr()), ctypes.c_void_p(samples.data_ptr()),
                               _stream_handle(stream)), "sgl_inverse")


def sgl_naive_forward(plan: Plan, samples, coeffs, stream=None):
    """Alg. 1 (every coefficient as the full quadrature sum), SGL_F64 plans."""
    plan._check_tensor(samples, plan.total_samples, "samples")
    plan._check_tensor(coeffs, plan.total_coeffs, "coeffs")
    _check(_load().sgl_naive_forward(plan.handle, ctypes.c_void_p(samples.data_ptr()),
                                     ctypes.c_void_p(coeffs.data_ptr()), _stream_handle(stream)), "sgl_naive_forward")


def sgl_naive_inverse(plan: Plan, coeffs, samples, stream=None):
    """Alg. 2 (every sample as the full synthesis sum), SGL_F64 plans."""
    plan._check_tensor(coeffs, plan.total_coeffs, "coeffs")
    plan._check_tensor(samples, plan.total_samples, "samples")
    _check(_load().sgl_naive_inverse(plan.handle, ctypes.c_void_p(coeffs.data_ptr()),
                                     ctypes.c_void_p(samples.data_ptr()), _stream_handle(stream)), "sgl_naive_inverse")


def sgl_midpoint_forward(plan: Plan, values, nx: int, half_width: float, coeffs, stream=None):
    """Cartesian midpoint-rule projection of nx^3 cell values per function (SGL_F64 plans)."""
    plan._check_tensor(values, plan.nfunc * nx ** 3, "values")
    plan._check_tensor(coeffs, plan.total_coeffs, "coeffs")
    _check(_load().sgl_midpoint_forward(plan.handle, ctypes.c_void_p(values.data_ptr()), int(nx),
                                        ctypes.c_double(half_width), ctypes.c_void_p(coeffs.data_ptr()),
                                        _stream_handle(stream)), "sgl_midpoint_forward")


def sgl_synthesize_points(plan: Plan, coeffs, xyz, values, stream=None):
    """values[f, p] = sum fhat H(x_p) at arbitrary points xyz (npts x 3 float64 CUDA tensor)."""
    import torch
    if not isinstance(xyz, torch.Tensor) or not xyz.is_cuda or xyz.dtype != torch.float64 \
            or not xyz.is_contiguous() or xyz.dim() != 2 or xyz.shape[1] != 3:
        raise ValueError("xyz must be a contiguous float64 CUDA tensor of shape (npts, 3)")
    npts = int(xyz.shape[0])
    plan._check_tensor(coeffs, plan.total_coeffs, "coeffs")
    plan._check_tensor(values, plan.nfunc * npts, "values")
    _check(_load().sgl_synthesize_points(plan.handle, ctypes.c_void_p(coeffs.data_ptr()), npts,
                                         ctypes.c_void_p(xyz.data_ptr()), ctypes.c_void_p(values.data_ptr()),
                                         _stream_handle(stream)), "sgl_synthesize_points")


def sgl_plan_destroy(plan: Plan):
    plan.destroy()


def sgl_debug_gemm(dtype, A, X, C):
    """C = A @ X on the GPU through the stage GEMM core (A, X, C float64 CUDA tensors)."""
    dtype = DTYPES.get(dtype, dtype)
    M, K = A.shape
    K2, N = X.shape
    assert K == K2 and tuple(C.shape) == (M, N)
    _check(_load().sgl_debug_gemm(int(dtype), M, N, K, ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                                  ctypes.c_void_p(C.data_ptr())), "sgl_debug_gemm")
