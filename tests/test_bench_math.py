"""The benchmark's roofline arithmetic (CPU): algorithmic bytes per stage launch
against the sizes of the buffers each stage must read and write (B = 128,
batch 4, complex64: samples 8B^3, spectrum (2B-1) 4B^2, intermediate 2B^3,
coefficients Omega per function; tables B^2 (B+1) entries of 6 bytes in the
split form), and the choice of the bound."""

import math
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

B, NF = 128, 4
C64 = 8
SAMPLES = 8 * B ** 3 * NF * C64              # 536870912
SPECTRUM = (2 * B - 1) * (2 * B) ** 2 * NF * C64  # 534773760
INTER = 2 * B ** 3 * NF * C64                # 134217728
COEFFS = 707264 * NF * C64                   # Omega(128) = 707264
TABLE = B * B * (B + 1) * 6


def test_stage_bytes_match_buffer_sizes():
    w = bench.stage_work(B, NF, "split_bf16")
    assert w["fwd_a_fft"][1] == w["inv_a_fft"][1] == SAMPLES + SPECTRUM == 1071644672
    assert w["fwd_b_legendre"][1] == w["inv_b_legendre"][1] == SPECTRUM + INTER + TABLE == 681672704
    assert w["fwd_c_radial"][1] == w["inv_c_radial"][1] == INTER + COEFFS + TABLE == 169531392


def test_legendre_flops_count_every_order():
    # sum over m in [1-B, B-1] of 2 (B-|m|) * 2B * 4B NF real flops = 16 B^4 NF; six products in the split form
    direct = sum(2 * (B - abs(m)) * (2 * B) * (2 * 2 * B * NF) for m in range(1 - B, B))
    assert bench.stage_work(B, NF, "f64")["fwd_b_legendre"][0] == direct
    assert bench.stage_work(B, NF, "split_bf16")["fwd_b_legendre"][0] == 6 * direct


@pytest.mark.parametrize("slow", ["fwd_a_fft", "inv_b_legendre"])
def test_roofline_takes_the_longest_stage(slow):
    ms = {k: 0.05 for k in bench.STAGES}
    ms[slow] = 0.25
    r = bench.roofline({"stage_ms": ms}, "split_bf16", B, NF)
    assert r["kernel"] == slow and r["bound"] == "hbm"
    nbytes = bench.stage_work(B, NF, "split_bf16")[slow][1]
    assert math.isclose(r["achieved"], nbytes / 0.25e-3 / 1e9)
    assert math.isclose(r["frac"], r["achieved"] / 8000.0)


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})])
def test_bench_refuses_more_than_one_gpu(argv, env):
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), *argv], capture_output=True, text=True,
                       env={**os.environ, **env}, timeout=120)
    assert r.returncode == 2
    assert "--gpus must be 1" in r.stderr
    assert r.stdout == ""
