"""Code-generation checks of the stage kernels (CPU: compiles the HIP sources for
gfx950 to device assembly with the library's flags and reads the result).

The kernels rely on properties the source can only request:
  * the spectrum F and the samples pass through HBM with streaming
    (non-temporal) stores, which keep the smaller stage (b)/(c) intermediates
    cached; a compiler that merges a streaming store with an ordinary one drops
    the hint silently (this happened once), so every store of the forward and
    inverse FFT kernels and of the inverse Legendre kernels must carry it;
  * the copy-fed inverse Legendre kernels (split and FP32) wait for their
    copies with a vector memory count that assumes exactly 16 epilogue stores
    per lane and item (the vector-memory counter of the CDNA ISA counts loads,
    stores and LDS copies of one wave and retires them in issue order), so
    their code must hold 16 stores;
  * the copy-fed Legendre kernels keep their copies in flight across items, so
    they must load nothing else through the vector-memory path: any register
    load (a class or work-list field read as a vector load) would make its
    first use wait for every outstanding copy.
"""

import os
import re
import subprocess
import concurrent.futures

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1604_05140_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "--cuda-device-only", "-S"]

_ASM = {}


def _asm(src, tmp):
    out = os.path.join(tmp, src + ".s")
    r = subprocess.run([HIPCC, *FLAGS, os.path.join(CSRC, src), "-o", out], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return open(out).read()


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    tmp = str(tmp_path_factory.mktemp("asm"))
    with concurrent.futures.ThreadPoolExecutor(2) as ex:
        gemm, fft = ex.map(lambda f: _asm(f, tmp), ["sgl_gemm.hip", "sgl_fft.hip"])
    return {"gemm": gemm, "fft": fft}


def kernels(text, pattern):
    """(mangled name, body) of every kernel whose name matches pattern."""
    out = []
    for m in re.finditer(r"^(_Z\S*" + pattern + r"\S*):", text, re.M):
        name = m.group(1)
        end = text.index(".Lfunc_end", m.end())
        out.append((name, text[m.end():end]))
    assert out, pattern
    return out


def stores(body):
    lines = [l for l in body.split("\n") if re.match(r"\s*global_store", l)]
    return len(lines), sum(1 for l in lines if re.search(r"\bnt\b", l))


def test_fft_kernels_stream_every_store(asm):
    for name, body in kernels(asm["fft"], r"k_fft_(?:forward|inverse)"):
        n, nt = stores(body)
        assert n > 0 and nt == n, (name, n, nt)


def test_inverse_legendre_kernels_stream_the_spectrum(asm):
    for name, body in kernels(asm["gemm"], r"k_legendre_(?:split|f32)ILi1E") + kernels(asm["gemm"], r"k_gemmILi\dELi1ELi\dE"):
        n, nt = stores(body)
        assert n > 0 and nt == n, (name, n, nt)


def test_copy_fed_inverse_legendre_has_sixteen_stores(asm):
    found = kernels(asm["gemm"], r"k_legendre_(?:split|f32)ILi1E")
    assert len(found) == 2
    for name, body in found:
        n, _ = stores(body)
        assert n == 16, (name, n)


def test_copy_fed_legendre_kernels_load_only_by_copies(asm):
    for name, body in kernels(asm["gemm"], r"k_legendre_(?:split|f32)"):
        loads = re.findall(r"^\s+((?:global|flat|buffer)_load\w*)", body, re.M)
        assert loads and all(l == "global_load_lds_dwordx4" for l in loads), (name, sorted(set(loads)))
