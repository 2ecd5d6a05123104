"""Benchmark: SGL forward+inverse transforms/s at B = 128, batch 4 (libsgl on one MI355X).

One step = one forward (Alg. 3) and one inverse (Alg. 4) transform of the whole
batch: stage (a) azimuthal FFT, stage (b) Legendre projection, stage (c)
radial projection, and back.  Inputs are resident in HBM before timing:
complex-normal coefficients times 1/n (seeded), and the samples the plain FP64
GPU path synthesizes from them, rounded to complex64 for the reduced-precision
forms.  The headline form is the three-piece split-bf16 MFMA path; the plain
FP64 GPU path is timed beside it, and the split results are checked against it
(e_inf = max|delta| / max|ref| per function) before timing: a form over its
bar (split-bf16 1e-6, FP32 1e-5) is not timed, and the headline then prints a
null value with gate_failed and exits non-zero.  Every form is timed with the
headline's plan flags (SGL_AUTOTUNE | SGL_GRAPHS); the eager FP64 plan is
timed beside them.

Prints one JSON line.  Also reports per-stage kernel times (HIP events recorded
on the launch stream inside the timed region), the roofline position of the
dominant kernel, and the CPU oracle timed on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

STAGES = ["fwd_a_fft", "fwd_b_legendre", "fwd_c_radial", "inv_c_radial", "inv_b_legendre", "inv_a_fft"]
PEAK = {"hbm_GBs": 8000.0, "f64": 78.6, "f32": 157.3, "bf16": 2500.0}  # TFLOP/s, MI355X published dense


def num_coeffs(B):
    return B * (B + 1) * (2 * B + 1) // 6


def stage_work(B, nf, dtype):
    """Algorithmic flops and HBM bytes of one launch of each stage (per launch)."""
    es = 16 if dtype == "f64" else 8
    Om = num_coeffs(B)
    samples = 8 * B ** 3 * nf * es
    F = (2 * B - 1) * 4 * B * B * nf * es
    g = 2 * B ** 3 * nf * es
    coef = Om * nf * es
    tab = B * B * (B + 1) * {"f64": 8, "f32": 4, "split_bf16": 6}[dtype]
    mult = 6 if dtype == "split_bf16" else 1  # the split form issues six bf16 products per MAC
    fb = 16 * B ** 4 * nf * mult
    fc = 8 * B * Om * nf * mult
    fft_flops = 5 * 2 * B * math.log2(2 * B) * 4 * B * B * nf
    return {
        "fwd_a_fft": (fft_flops, samples + F),
        "fwd_b_legendre": (fb, F + g + tab),
        "fwd_c_radial": (fc, g + coef + tab),
        "inv_c_radial": (fc, coef + g + tab),
        "inv_b_legendre": (fb, g + F + tab),
        "inv_a_fft": (fft_flops, F + samples),
    }


def time_steps(torch, sgl, plan, c_in, s_in, cout, sout, steps):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        sgl.sgl_forward(plan, s_in, cout)
        sgl.sgl_inverse(plan, c_in, sout)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def run_form(sgl, torch, plan, c_in, s_in, steps, warmup):
    """Two timed regions of `steps` forward+inverse pairs each: the first with
    plain calls (graph replays when the plan was made with SGL_GRAPHS) gives
    ms_per_step; the second records HIP events around every stage launch on the
    launch stream (eager launches) and gives the per-stage kernel times."""
    dev = c_in.device
    cout = torch.empty(plan.total_coeffs, dtype=plan.complex_dtype, device=dev)
    sout = torch.empty(plan.total_samples, dtype=plan.complex_dtype, device=dev)
    for _ in range(warmup):
        sgl.sgl_forward(plan, s_in, cout)
        sgl.sgl_inverse(plan, c_in, sout)
    torch.cuda.synchronize()
    ms = time_steps(torch, sgl, plan, c_in, s_in, cout, sout, steps)
    plan.stage_times()  # reset
    plan.set_timing(True)
    ms_inst = time_steps(torch, sgl, plan, c_in, s_in, cout, sout, steps)
    st_ms, st_cnt = plan.stage_times()
    plan.set_timing(False)
    per_stage = {STAGES[q]: (st_ms[q] / st_cnt[q] if st_cnt[q] else None) for q in range(6)}
    return ms, ms_inst, per_stage, cout, sout


def measured_traffic(kernel_stage, dtype, B, nf):
    """HBM bytes per launch of a stage kernel from the committed rocprofv3 PMC
    summary (FETCH_SIZE and WRITE_SIZE, calibrated on a plain copy), or None
    when no summary covers this workload or the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{dtype}_b{B}_batch{nf}.txt")
    if not os.path.exists(path):
        return None
    rows, src_hash = {}, {}
    for line in open(path):
        line = line.strip()
        if line.startswith("source_sha256"):
            _, f, h = line.split()
            src_hash[f] = h
        elif line.startswith("stage="):
            kv = dict(x.split("=", 1) for x in line.split())
            rows[kv["stage"]] = kv
    r = rows.get(kernel_stage)
    if r is None:
        return None
    f = os.path.join(ROOT, "paper_1604_05140_amd", "csrc", r["source"])
    if not os.path.exists(f) or hashlib.sha256(open(f, "rb").read()).hexdigest() != src_hash.get(r["source"]):
        return None
    return float(r["traffic_bytes"])


def roofline(form, dtype, B, nf):
    """Roofline position of the dominant (longest) stage kernel of a form.  The
    bound is whichever of HBM (algorithmic bytes at 8 TB/s) or the matrix cores
    (issued flops at the dtype's dense peak; the split form issues six bf16
    products per multiply-add) gives the longer ideal time; `achieved` is the
    algorithmic bytes or flops of one launch over the measured launch time."""
    work = stage_work(B, nf, dtype)
    dom = max((k for k in STAGES if form["stage_ms"][k]), key=lambda k: form["stage_ms"][k])
    flops, nbytes = work[dom]
    t_s = form["stage_ms"][dom] / 1000.0
    pk = {"f64": PEAK["f64"], "f32": PEAK["f32"], "split_bf16": PEAK["bf16"]}[dtype]
    t_hbm = nbytes / (PEAK["hbm_GBs"] * 1e9)
    t_mfma = 0.0 if "fft" in dom else flops / (pk * 1e12)
    mult = 6 if dtype == "split_bf16" else 1
    if t_hbm >= t_mfma:
        roof = {"bound": "hbm", "achieved": nbytes / t_s / 1e9, "peak": PEAK["hbm_GBs"], "unit": "GB/s"}
    else:
        roof = {"bound": "mfma", "achieved": flops / mult / t_s / 1e12, "peak": pk / mult, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom, dtype, B, nf)
    roof["kernel"] = dom
    roof["avg_launch_ms"] = form["stage_ms"][dom]
    roof["algorithmic_bytes"] = nbytes
    roof["algorithmic_flops"] = flops if "fft" in dom else flops // mult
    return roof


def copy_reference(torch, dev, nbytes=1 << 30, reps=5):
    """Measured streaming rate of a plain device-to-device copy (torch's copy
    kernel, read + write bytes over time): a practical ceiling for kernels that
    read and write HBM once, for context beside the published 8 TB/s."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / ms / 1e6


def stage_rooflines(form, dtype, B, nf):
    """Every stage of a form against HBM (algorithmic bytes) and against its
    dtype's dense MFMA peak (issued flops; stage (a) runs on the vector ALUs)."""
    work = stage_work(B, nf, dtype)
    pk = {"f64": PEAK["f64"], "f32": PEAK["f32"], "split_bf16": PEAK["bf16"]}[dtype]
    out = {}
    for st in STAGES:
        t = form["stage_ms"][st]
        if not t:
            continue
        flops, nbytes = work[st]
        row = {"ms": t, "hbm_GBps": nbytes / t / 1e6, "hbm_frac": nbytes / t / 1e6 / PEAK["hbm_GBs"]}
        if "fft" not in st:
            row["mfma_TFLOPs_issued"] = flops / t / 1e9
            row["mfma_frac"] = flops / t / 1e9 / pk
        out[st] = row
    return out


def host_cpu():
    """CPU model, logical CPUs and the CPUs this process may use (its worker bound:
    at most 16, the host share of one GPU)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable, "workers": max(1, min(16, usable))}


_ORACLE_JOB = {}


def _oracle_forward_part(oms):
    from oracle import direct as D
    j = _ORACLE_JOB
    return D.forward(j["s"], j["B"], omegas=oms)


def _oracle_inverse_part(pts):
    from oracle import direct as D
    j = _ORACLE_JOB
    return D.inverse(j["c"], j["B"], points=pts)


def _oracle_sample(B, n_coef, n_pts, seed, workers):
    """Time the oracle's forward sums at n_coef seeded coefficients and its
    synthesis sums at n_pts seeded grid points, on `workers` processes (1 = this
    process); returns (forward s, inverse s)."""
    import multiprocessing as mp

    import numpy as np

    from oracle import direct as D
    from paper_1604_05140_amd import synth

    D.get_basis(B)  # nodes, weights and basis tables (set-up, not timed)
    _ORACLE_JOB.update(B=B, s=synth.complex_normal_samples(B, 1, seed=seed)[0],
                       c=synth.complex_normal_coeffs(B, 1, seed=seed + 1, decay=1.0)[0])
    oms = synth.subset(n_coef, D.num_coeffs(B), seed=seed + 2)
    pts = synth.grid_points(n_pts, B, seed=seed + 3)
    if workers == 1:
        t0 = time.perf_counter()
        _oracle_forward_part(oms)
        t1 = time.perf_counter()
        _oracle_inverse_part(pts)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1
    with mp.get_context("fork").Pool(workers) as pool:
        pool.map(_oracle_forward_part, [oms[:1]] * workers)  # workers started and warm
        t0 = time.perf_counter()
        pool.map(_oracle_forward_part, np.array_split(oms, workers))
        t1 = time.perf_counter()
        pool.map(_oracle_inverse_part, np.array_split(pts, workers))
        t2 = time.perf_counter()
    return t1 - t0, t2 - t1


def cpu_baseline(B, n_coef, n_pts, seed):
    """The oracle (plain direct quadrature sums, numpy, one process per worker) on a
    bounded sample, scaled to one full forward+inverse pair: one worker, then every
    usable host CPU (up to 16) on a sample as many times larger."""
    from oracle import direct as D

    cpu = host_cpu()
    W = cpu["workers"]
    f1, i1 = _oracle_sample(B, n_coef, n_pts, seed, 1)
    fW, iW = _oracle_sample(B, n_coef * W, n_pts * W, seed, W) if W > 1 else (f1, i1)
    per_pair = lambda tf, ti, k: tf / (n_coef * k) * D.num_coeffs(B) + ti / (n_pts * k) * D.num_samples(B)
    t1, tW = per_pair(f1, i1, 1), per_pair(fW, iW, W)
    return {
        "value": 1.0 / tW,
        "unit": "transforms/s",
        "cores": W,
        "kind": "oracle",
        "host_cpu": cpu["model"],
        "host_logical_cpus": cpu["logical_cpus"],
        "host_usable_cpus": cpu["usable_cpus"],
        "single_core_value": 1.0 / t1,
        "sample": (f"B={B}: the oracle's forward quadrature sums at seeded coefficients and inverse synthesis "
                   f"sums at seeded grid points, scaled to all {D.num_coeffs(B)} coefficients and "
                   f"{D.num_samples(B)} points of one forward+inverse pair (extrapolated); {W} worker processes: "
                   f"{n_coef * W} coefficients ({fW:.1f} s) + {n_pts * W} points ({iW:.1f} s) -> {tW:.3g} s per "
                   f"pair; 1 process: {n_coef} coefficients ({f1:.1f} s) + {n_pts} points ({i1:.1f} s) -> "
                   f"{t1:.3g} s per pair; host {cpu['model']}, {cpu['usable_cpus']} usable of "
                   f"{cpu['logical_cpus']} logical CPUs"),
    }


def bench_oracle(args):
    """The oracle's full direct transforms (Alg. 1 forward over every coefficient,
    Alg. 2 synthesis at every grid point) at B = 2..max, on one process and on
    every usable host CPU (up to 16), as in the paper's Table 2 protocol (one
    inverse and one forward transform of coefficients with Re, Im uniform on
    (-1, 1)); CPU only."""
    import multiprocessing as mp

    import numpy as np

    from oracle import direct as D
    from paper_1604_05140_amd import synth

    cpu = host_cpu()
    W = cpu["workers"]
    rows = []
    for B in [b for b in (2, 4, 8, 16, 32) if b <= args.oracle_max_b]:
        c = synth.uniform_coeffs(B, 1, seed=synth.BASE_SEED + 60 + B)[0]
        D.get_basis(B)
        row = {"B": B}
        for w in sorted({1, W}):
            t0 = time.perf_counter()
            if w == 1:
                s = D.inverse(c, B)
                t1 = time.perf_counter()
                f = D.forward(s, B)
            else:
                pts = np.stack(np.meshgrid(*(np.arange(2 * B),) * 3, indexing="ij"), -1).reshape(-1, 3)
                _ORACLE_JOB.update(B=B, c=c)
                with mp.get_context("fork").Pool(w) as pool:
                    s = np.concatenate(pool.map(_oracle_inverse_part, np.array_split(pts, w)))
                t1 = time.perf_counter()
                _ORACLE_JOB["s"] = s  # the forward's workers are forked with the synthesized samples
                with mp.get_context("fork").Pool(w) as pool:
                    f = np.concatenate(pool.map(_oracle_forward_part, np.array_split(np.arange(D.num_coeffs(B)), w)))
            t2 = time.perf_counter()
            row[f"workers_{w}"] = {"inverse_s": t1 - t0, "forward_s": t2 - t1, "pair_s": t2 - t0,
                                   "max_abs_err": float(np.abs(f - c).max())}
            print(f"[bench] oracle B={B} workers={w}: inverse {t1 - t0:.3g} s, forward {t2 - t1:.3g} s",
                  file=sys.stderr, flush=True)
        rows.append(row)
    print(json.dumps({
        "metric": "CPU oracle: full direct SGL forward+inverse transform (Alg. 1/2), seconds per pair",
        "unit": "s", "dtype": "f64", "data": "synthetic", "host_cpu": cpu,
        "config": {"workload": "one inverse then one forward direct transform, coefficients with Re, Im "
                               "uniform on (-1, 1)"},
        "rows": rows}), flush=True)


def bench_batched(args, torch, sgl, synth, dev):
    """256 functions with bandlimits uniform in {16..96}, one persistent launch per
    stage over the (order, bandlimit) work list, autotuned grids, graph replay."""
    dtype = "f32" if args.dtype == "split_bf16" and "--dtype" not in sys.argv else args.dtype
    Bs = [int(b) for b in synth.batched_bandlimits(256, 16, 96, seed=synth.BASE_SEED + 4)]
    print(f"[bench] batched: 256 functions, form {dtype}", file=sys.stderr, flush=True)
    plan = sgl.sgl_plan_ex(Bs, dtype, sgl.SGL_AUTOTUNE | sgl.SGL_GRAPHS)
    ct = plan.complex_dtype
    cs = [synth.complex_normal_coeffs(B, 1, seed=synth.BASE_SEED + 4000 + q, decay=1.0)[0] for q, B in enumerate(Bs)]
    import numpy as np
    c_in = torch.from_numpy(np.concatenate(cs)).to(dev, ct)
    s_in = torch.empty(plan.total_samples, dtype=ct, device=dev)
    sgl.sgl_inverse(plan, c_in, s_in)
    ms, ms_inst, per_stage, _, _ = run_form(sgl, torch, plan, c_in, s_in, args.steps, args.warmup)
    out = {
        "metric": "SGL fwd+inv transforms/s, 256 functions with B uniform in {16..96} (batched form)",
        "value": 256 * 1000.0 / ms,
        "unit": "transforms/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"split_bf16": "bf16x3 (fp32 accumulate)", "f32": "f32", "f64": "f64"}[dtype],
        "data": "synthetic",
        "config": {"workload": "SGL forward+inverse, 256 functions, B uniform in {16..96}, complex-normal/n "
                               "coefficients", "form": dtype, "total_coeffs": plan.total_coeffs,
                   "total_samples": plan.total_samples},
        "stage_ms": per_stage, "ms_per_step_with_stage_events": ms_inst, "launch_grids": plan.launch_grids(),
        "launch_tiles": plan.launch_tiles(),
    }
    print(json.dumps(out), flush=True)


def seminaive_stage_work(B, nf, dtype):
    """Algorithmic flops and HBM bytes of the seminaive Legendre stage (Sect. 3.3.1)
    per direction: the DCT pass over the spectrum (read F, write the B cosine rows;
    inverse: read them, write F) plus the contraction over k < B (read the cosine
    rows and the table, write g; inverse the reverse).  Flops: the 4B-point FFT of
    every spectrum column and 8 B^4 per function for the contraction (half of the
    direct 16 B^4; times six issued bf16 products in the split form)."""
    es = 16 if dtype == "f64" else 8
    cols = (2 * B - 1) * 2 * B * nf
    F = cols * 2 * B * es
    T = cols * B * es
    g = 2 * B ** 3 * nf * es
    tab = B * B * (B + 1) // 2 * {"f64": 8, "f32": 4, "split_bf16": 6}[dtype]
    mult = 6 if dtype == "split_bf16" else 1
    dct_flops = 5 * 4 * B * math.log2(4 * B) * cols
    return dct_flops + 8 * B ** 4 * nf * mult, (F + T) + (T + g + tab)


def bench_seminaive(args, torch, sgl, synth, dev):
    """The seminaive Legendre step (SGL_SEMINAIVE) beside the direct sums, B = 128
    batch 4, in the headline split-bf16 form and in plain FP64: ms per step, the
    per-stage kernel times, the errors against the FP64 direct path, and the
    Legendre stages against HBM and the matrix-core peak."""
    B, nf = args.B, args.batch
    ns, nc = 8 * B ** 3, num_coeffs(B)
    c = synth.complex_normal_coeffs(B, nf, seed=synth.BASE_SEED + 3, decay=1.0).reshape(-1)
    c128 = torch.from_numpy(c).to(dev)
    p64 = sgl.sgl_plan(B, nf, "f64")
    s128 = torch.empty(p64.total_samples, dtype=torch.complex128, device=dev)
    sgl.sgl_inverse(p64, c128, s128)
    c_ref = torch.empty_like(c128)
    sgl.sgl_forward(p64, s128, c_ref)
    torch.cuda.synchronize()

    def einf(ref, got, n):
        ref = ref.reshape(-1, n).to(torch.complex128)
        got = got.reshape(-1, n).to(torch.complex128)
        return float(((got - ref).abs().amax(dim=1) / ref.abs().amax(dim=1)).max())

    forms = {}
    for dtype in ([args.dtype] + [d for d in ("f64",) if d != args.dtype]):
        for semi in (True, False):
            flags = sgl.SGL_AUTOTUNE | sgl.SGL_GRAPHS | (sgl.SGL_SEMINAIVE if semi else 0)
            plan = sgl.sgl_plan_ex([B] * nf, dtype, flags)
            s_in = s128 if dtype == "f64" else s128.to(torch.complex64)
            c_in = c128 if dtype == "f64" else c128.to(torch.complex64)
            print(f"[bench] seminaive={semi} {dtype}: timing", file=sys.stderr, flush=True)
            ms, ms_inst, per_stage, cout, sout = run_form(sgl, torch, plan, c_in, s_in, args.steps, args.warmup)
            key = f"{dtype}_{'seminaive' if semi else 'direct'}"
            forms[key] = {"ms_per_step": ms, "transforms_per_s": nf * 1000.0 / ms, "stage_ms": per_stage,
                          "e_inf_forward_vs_f64": einf(c_ref, cout, nc),
                          "e_inf_inverse_vs_f64": einf(s128, sout, ns)}
            if semi:
                fl, nb = seminaive_stage_work(B, nf, dtype)
                pk = {"f64": PEAK["f64"], "f32": PEAK["f32"], "split_bf16": PEAK["bf16"]}[dtype]
                forms[key]["legendre_roofline"] = {
                    st: {"ms": per_stage[st], "hbm_GBps": nb / per_stage[st] / 1e6,
                         "hbm_frac": nb / per_stage[st] / 1e6 / PEAK["hbm_GBs"],
                         "issued_TFLOPs": fl / per_stage[st] / 1e9, "mfma_frac": fl / per_stage[st] / 1e9 / pk}
                    for st in ("fwd_b_legendre", "inv_b_legendre")}
                forms[key]["algorithmic_bytes_per_legendre_launch"] = nb
            print(f"[bench] {key}: {ms:.3f} ms/step", file=sys.stderr, flush=True)
            del cout, sout
            plan.destroy()
    head = forms[f"{args.dtype}_seminaive"]
    out = {
        "metric": f"SGL fwd+inv transforms/s at B={B} batch {nf}, seminaive Legendre step (Sect. 3.3.1)",
        "value": head["transforms_per_s"], "unit": "transforms/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"split_bf16": "bf16x3 (fp32 accumulate)", "f32": "f32", "f64": "f64"}[args.dtype],
        "data": "synthetic",
        "config": {"workload": f"SGL forward+inverse, B={B}, batch {nf}, complex-normal/n coefficients, "
                               "seminaive vs direct Legendre step", "form": args.dtype},
        "forms": forms,
        "seminaive_over_direct_time": {d: forms[f"{d}_seminaive"]["ms_per_step"] / forms[f"{d}_direct"]["ms_per_step"]
                                       for d in {args.dtype, "f64"}},
    }
    print(json.dumps(out), flush=True)


def bench_naive(args, torch, sgl, synth, dev):
    """The paper's Sect. 4 protocol on the GPU, naive (Alg. 1/2) beside fast
    (Alg. 3/4), both plain FP64: coefficients with real and imaginary parts
    uniform on (-1, 1), one inverse then one forward transform, errors of the
    recovered coefficients (maximum absolute and maximum relative, averaged over
    10 functions), and transforms/s of each."""
    import numpy as np
    rows = []
    for B in [b for b in (2, 4, 8, 16, 32, 64) if b <= args.naive_max_b]:
        nf = 10
        c = synth.uniform_coeffs(B, nf, seed=synth.BASE_SEED + 60 + B)
        plan = sgl.sgl_plan(B, nf, "f64")
        c_in = torch.from_numpy(c.reshape(-1)).to(dev)
        s = torch.empty(plan.total_samples, dtype=torch.complex128, device=dev)
        c_out = torch.empty_like(c_in)
        row = {"B": B, "functions": nf}
        for name, inv, fwd in (("naive", sgl.sgl_naive_inverse, sgl.sgl_naive_forward),
                               ("fast", sgl.sgl_inverse, sgl.sgl_forward)):
            inv(plan, c_in, s)
            fwd(plan, s, c_out)
            torch.cuda.synchronize()
            reps = 1 if name == "naive" and B >= 32 else 3
            t0 = time.perf_counter()
            for _ in range(reps):
                inv(plan, c_in, s)
                fwd(plan, s, c_out)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            got = c_out.cpu().numpy().reshape(nf, -1)
            d = np.abs(got - c)
            row[name] = {"ms_per_pair_of_all": dt * 1e3, "transforms_per_s": nf / dt,
                         "avg_max_abs_err": float(d.max(axis=1).mean()),
                         "avg_max_rel_err": float((d / np.abs(c)).max(axis=1).mean())}
        print(f"[bench] naive B={B}: naive {row['naive']['ms_per_pair_of_all']:.2f} ms, "
              f"fast {row['fast']['ms_per_pair_of_all']:.3f} ms for {nf} pairs", file=sys.stderr, flush=True)
        rows.append(row)
        plan.destroy()
    print(json.dumps({
        "metric": "naive (Alg. 1/2) vs fast (Alg. 3/4) FP64 SGL transforms on the GPU, Sect. 4 protocol",
        "unit": "transforms/s", "n_gpus": 1, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "inverse then forward transform of 10 functions per bandlimit, coefficients "
                               "with Re, Im uniform on (-1, 1)"},
        "rows": rows}), flush=True)


def bench_midpoint(args, torch, sgl, synth, dev):
    """Sect. 5's foil: the Cartesian midpoint-rule projection (the field's
    practice) against the sampling-theorem transform, FP64 on the GPU.  A
    bandlimited function with CN(0,1)/n coefficients is synthesized on the cells
    of a regular grid on [-h, h]^3 (GPU), projected by the midpoint rule, and
    compared with its true coefficients, for several cell sizes; the
    sampling-theorem forward transform of its samples on the SGL grid is timed
    and checked beside it."""
    import numpy as np
    rows = []
    h = 10.0
    for B in (8, 16):
        c = synth.complex_normal_coeffs(B, 1, seed=synth.BASE_SEED + 80 + B, decay=1.0)[0]
        c_in = torch.from_numpy(c).to(dev)
        plan = sgl.sgl_plan(B, 1, "f64")
        s = torch.empty(plan.total_samples, dtype=torch.complex128, device=dev)
        out = torch.empty(plan.total_coeffs, dtype=torch.complex128, device=dev)
        sgl.sgl_inverse(plan, c_in, s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sgl.sgl_forward(plan, s, out)
        torch.cuda.synchronize()
        t_sgl = time.perf_counter() - t0
        e_sgl = float((out - c_in).abs().max() / c_in.abs().max())
        for cell in (1.0, 0.75, 0.5, 0.35, 0.25):
            nx = int(round(2 * h / cell))
            ax = -h + (torch.arange(nx, dtype=torch.float64, device=dev) + 0.5) * (2 * h / nx)
            gx, gy, gz = torch.meshgrid(ax, ax, ax, indexing="ij")
            xyz = torch.stack([gx.reshape(-1), gy.reshape(-1), gz.reshape(-1)], dim=1).contiguous()
            vals = torch.empty(nx ** 3, dtype=torch.complex128, device=dev)
            sgl.sgl_synthesize_points(plan, c_in, xyz, vals)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sgl.sgl_midpoint_forward(plan, vals, nx, h, out)
            torch.cuda.synchronize()
            t_mid = time.perf_counter() - t0
            e_mid = float((out - c_in).abs().max() / c_in.abs().max())
            rows.append({"B": B, "cell": 2 * h / nx, "nx": nx, "cells": nx ** 3, "midpoint_e_inf": e_mid,
                         "midpoint_ms": t_mid * 1e3, "sgl_grid_points": 8 * B ** 3, "sgl_e_inf": e_sgl,
                         "sgl_forward_ms": t_sgl * 1e3})
            print(f"[bench] midpoint B={B} cell={2 * h / nx:.3f}: e_inf {e_mid:.2e} ({t_mid * 1e3:.2f} ms); "
                  f"SGL grid e_inf {e_sgl:.2e} ({t_sgl * 1e3:.3f} ms)", file=sys.stderr, flush=True)
        plan.destroy()
    print(json.dumps({
        "metric": "midpoint-rule Cartesian projection vs SGL sampling-theorem transform, FP64 (Sect. 5 foil)",
        "n_gpus": 1, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"bandlimited functions, CN(0,1)/n coefficients, cells on [-{h}, {h}]^3"},
        "rows": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--B", type=int, default=128)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--dtype", default="split_bf16", choices=["split_bf16", "f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 and FP32 side runs")
    ap.add_argument("--workload", default="b128", choices=["b128", "batched", "naive", "midpoint", "seminaive", "oracle"],
                    help="b128: B=128 batch 4 (headline); batched: 256 functions, B uniform in {16..96}; "
                         "naive: naive vs fast FP64 transforms at B = 2..32 (the paper's Sect. 4 protocol); "
                         "midpoint: Cartesian midpoint-rule projection vs the sampling-theorem transform; "
                         "seminaive: the seminaive (cosine-domain) Legendre step beside the direct sums; "
                         "oracle: the CPU oracle's full direct transforms at B = 2..32 (no GPU)")
    ap.add_argument("--naive-max-b", type=int, default=32, help="largest bandlimit of the naive workload")
    ap.add_argument("--oracle-max-b", type=int, default=32, help="largest bandlimit of the oracle workload")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one MI355X: the SGL transforms are not sharded across GPUs here "
              "(--gpus must be 1).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "oracle":
        return bench_oracle(args)
    import torch

    from paper_1604_05140_amd import sgl, synth

    dev = torch.device("cuda:0")
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20)
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        dst.copy_(src)
        e0.record()
        for _ in range(3):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        print(json.dumps({"copy_probe_bytes": n, "launches": 4, "ms_per_copy": ms,
                          "copy_GBps": 2 * n / ms / 1e6}), flush=True)
        return
    if args.workload == "batched":
        return bench_batched(args, torch, sgl, synth, dev)
    if args.workload == "naive":
        return bench_naive(args, torch, sgl, synth, dev)
    if args.workload == "midpoint":
        return bench_midpoint(args, torch, sgl, synth, dev)
    if args.workload == "seminaive":
        return bench_seminaive(args, torch, sgl, synth, dev)
    B, nf = args.B, args.batch
    ns, nc = 8 * B ** 3, num_coeffs(B)
    cpu_base = None
    if not args.no_cpu_baseline:
        # the oracle's worker processes are forked before this process touches the GPU
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cpu_base = cpu_baseline(B, 24, 300, synth.BASE_SEED + 7)
    print(f"[bench] B={B} batch={nf} form={args.dtype}: building inputs", file=sys.stderr, flush=True)
    # coefficient decay n^-p: p = 1 up to B = 128, 1.5 for the B = 256 configuration
    decay = 1.5 if B >= 256 else 1.0
    c = synth.complex_normal_coeffs(B, nf, seed=synth.BASE_SEED + 3, decay=decay).reshape(-1)
    c128 = torch.from_numpy(c).to(dev)
    p64 = sgl.sgl_plan(B, nf, "f64")
    s128 = torch.empty(p64.total_samples, dtype=torch.complex128, device=dev)
    sgl.sgl_inverse(p64, c128, s128)
    c_ref = torch.empty_like(c128)
    sgl.sgl_forward(p64, s128, c_ref)
    torch.cuda.synchronize()

    def einf(ref, got, n):
        ref = ref.reshape(-1, n).to(torch.complex128)
        got = got.reshape(-1, n).to(torch.complex128)
        return float(((got - ref).abs().amax(dim=1) / ref.abs().amax(dim=1)).max())

    rt64 = einf(c128, c_ref, nc)
    # the error bar of each form against the plain FP64 GPU path (FP64: its round
    # trip); a form over its bar is reported without a throughput
    bar = {"split_bf16": 1e-6, "f32": 1e-5, "f64": 1e-12}
    forms = {}
    # every form is timed as the headline form is built (SGL_AUTOTUNE | SGL_GRAPHS);
    # the plain eager FP64 plan of the reference inputs is timed beside it
    order = [args.dtype] + ([] if args.no_compare else [d for d in ("f64", "f32") if d != args.dtype] + ["f64_eager"])
    for key in order:
        head_form = key == args.dtype
        dtype = "f64" if key == "f64_eager" else key
        eager = key == "f64_eager"
        plan = p64 if eager else sgl.sgl_plan_ex([B] * nf, dtype, sgl.SGL_AUTOTUNE | sgl.SGL_GRAPHS)
        s_in = s128 if dtype == "f64" else s128.to(torch.complex64)
        c_in = c128 if dtype == "f64" else c128.to(torch.complex64)
        # precision gate, before any timing: one forward and one inverse of the
        # timed plan on the timed inputs against the FP64 GPU results
        cout = torch.empty(plan.total_coeffs, dtype=plan.complex_dtype, device=dev)
        sout = torch.empty(plan.total_samples, dtype=plan.complex_dtype, device=dev)
        sgl.sgl_forward(plan, s_in, cout)
        sgl.sgl_inverse(plan, c_in, sout)
        torch.cuda.synchronize()
        # (an FP64 plan's forward is held to the seeded coefficients themselves)
        ef, ei = einf(c128 if dtype == "f64" else c_ref, cout, nc), einf(s128, sout, ns)
        del cout, sout
        gate_ok = max(ef, ei) <= bar[dtype]
        print(f"[bench] gate {key}: forward e_inf {ef:.2e}, inverse e_inf {ei:.2e} (bar {bar[dtype]:g}) "
              f"{'ok' if gate_ok else 'FAILED'}", file=sys.stderr, flush=True)
        if head_form and not gate_ok:
            print(json.dumps({"metric": "SGL fwd+inv transforms/s at B=128 (MFMA split vs FP64), rel err <=1e-6",
                              "value": None, "unit": "transforms/s", "n_gpus": 1, "gate_failed": True,
                              "e_inf_forward_vs_f64": ef, "e_inf_inverse_vs_f64": ei, "bar": bar[dtype]}),
                  flush=True)
            sys.exit(1)
        steps = args.steps if head_form else max(3, args.steps // 4)
        warm = args.warmup if head_form else 2
        print(f"[bench] timing {key}: {warm} warmup + {steps} steps", file=sys.stderr, flush=True)
        ms, ms_inst, per_stage, cout, sout = run_form(sgl, torch, plan, c_in, s_in, steps, warm)
        forms[key] = {
            "ms_per_step": ms,
            "transforms_per_s": nf * 1000.0 / ms,
            "plan_flags": "none (eager launches, default grids)" if eager else "SGL_AUTOTUNE|SGL_GRAPHS",
            "ms_per_step_with_stage_events": ms_inst,
            "stage_ms": per_stage,
            "steps": steps,
            "e_inf_forward_vs_f64": ef,
            "e_inf_inverse_vs_f64": ei,
            "within_bar": gate_ok,
            "launch_grids": plan.launch_grids(),
            "launch_tiles": plan.launch_tiles(),
        }
        # every stage of this form against HBM and against its own dtype's MFMA peak
        forms[key]["stage_roofline"] = stage_rooflines(forms[key], key.replace("_eager", ""), B, nf)
        print(f"[bench] {key}: {ms:.3f} ms/step, {nf * 1000.0 / ms:.1f} transforms/s "
              f"(stage-timed pass {ms_inst:.3f} ms/step)", file=sys.stderr, flush=True)
        del cout, sout
        if plan is not p64:
            plan.destroy()

    head = forms[args.dtype]
    roof = roofline(head, args.dtype, B, nf)
    if roof["bound"] == "hbm":
        roof["copy_GBps"] = copy_reference(torch, dev)
        roof["frac_of_copy"] = roof["achieved"] / roof["copy_GBps"]

    out = {
        "metric": "SGL fwd+inv transforms/s at B=128 (MFMA split vs FP64), rel err <=1e-6",
        "value": head["transforms_per_s"],
        "unit": "transforms/s",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"split_bf16": "bf16x3 (fp32 accumulate)", "f32": "f32", "f64": "f64"}[args.dtype],
        "data": "synthetic",
        "config": {
            "workload": f"SGL forward+inverse, B={B}, batch {nf}, complex-normal/n^{decay:g} coefficients, "
                        f"{'complex128' if args.dtype == 'f64' else 'complex64'} scaled samples on the "
                        f"sampling-theorem grid",
            "B": B, "batch": nf, "form": args.dtype,
        },
        "e_inf_vs_f64": max(head["e_inf_forward_vs_f64"], head["e_inf_inverse_vs_f64"]),
        "f64_round_trip_e_inf": rt64,
        "forms": forms,
        "roofline": roof,
        "stage_roofline": stage_rooflines(head, args.dtype, B, nf),
        "coefficients_per_s": head["transforms_per_s"] * nc,
    }
    if "f64" in forms and args.dtype != "f64":
        # like for like: both plans built with SGL_AUTOTUNE | SGL_GRAPHS
        out["speedup_vs_f64"] = head["transforms_per_s"] / forms["f64"]["transforms_per_s"]
        out["speedup_vs_f64_eager"] = head["transforms_per_s"] / forms["f64_eager"]["transforms_per_s"]
    if cpu_base is not None:
        out["cpu_baseline"] = cpu_base
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
