#!/usr/bin/env python3
"""Benchmark of the 3D FFT pair and the Navier-Stokes step on one MI355X.

Headline: one forward r2c + inverse c2r pair of a 512^3 FP32 field of i.i.d. N(0,1)
values (seed 0), inputs resident in HBM, timed with HIP events over K pairs after W
warm-ups.  value = pair traffic of the three-pass plan (2 R + 10 C bytes, R = 4 N^3,
C = 8 N^2 (N/2+1)) divided by the pair time, in GB/s.  Also reported: the 1024^3 pair,
the per-pass kernel durations (HIP events on the launch stream), the roofline of the
dominant pass, the Navier-Stokes RK2 steps/s at 512^3 and the FP64 CPU oracle timed on
the host cores on one 512^3 pair.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-ns]
"""
import argparse
import json
import os
import sys
import time

HBM_PEAK_GBPS = 8000.0


def field_bytes(n):
    R = 4 * n ** 3
    C = 8 * n * n * (n // 2 + 1)
    return R, C


def pass_bytes(n):
    """Algorithmic bytes per launch of each pass (read + write of its logical arrays)."""
    R, C = field_bytes(n)
    return {"z_r2c": R + C, "y_fwd": 2 * C, "x_fwd": 2 * C, "x_inv": 2 * C, "y_inv": 2 * C, "z_c2r": C + R}


def pair_flops(n):
    """Nominal flops of a forward+inverse pair, 2 * 5 N^3 log2 N^3 (the paper's FLOP
    convention for its effective GFLOP/s tables)."""
    import math
    return 2 * 5 * n ** 3 * math.log2(n ** 3)


def time_pairs(tk, torch, n, steps, warmup, seed=0):
    import numpy as np
    import synth
    f = synth.gaussian_field((n, n, n), seed)
    x = torch.from_numpy(f).cuda()
    del f
    plan = tk.FFT3D(n, dtype=torch.float32, flags=tk.TK_FFT_TIMING)
    X = plan.empty_cplx()
    y = plan.empty_real()
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.r2c(x, X)
        plan.c2r(X, y)
    torch.cuda.synchronize()
    plan.pass_times()  # reset the event averages
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(steps):
        plan.r2c(x, X)
        plan.c2r(X, y)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    pt = plan.pass_times()
    names = ["z_r2c", "y_fwd", "x_fwd", "x_inv", "y_inv", "z_c2r"]
    passes = dict(zip(names, pt))
    desc = {p: plan.describe(p) for p in range(3)}
    err = (torch.linalg.vector_norm((y - x).double()) / torch.linalg.vector_norm(x.double())).item()
    plan.close()
    del x, X, y
    torch.cuda.empty_cache()
    return ms, passes, desc, err


def roofline(n, passes):
    pb = pass_bytes(n)
    dom = max(passes, key=lambda k: passes[k])
    achieved = pb[dom] / (passes[dom] * 1e-3) / 1e9
    return dom, {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBPS, 4),
        "traffic": None,
        "kernel": dom,
        "kernel_ms": round(passes[dom], 4),
        "bytes_per_launch": pb[dom],
    }


def cpu_baseline(n=512):
    """The FP64 oracle (C, OpenMP over lines) on one forward+inverse pair of the same
    512^3 input, on the host cores."""
    import numpy as np
    import synth
    from oracle import fft as offt
    f = synth.gaussian_field((n, n, n), 0).astype(np.float64)
    t = time.perf_counter()
    F = offt.rfft3(f)
    g = offt.irfft3(F)
    dt = time.perf_counter() - t
    R, C = field_bytes(n)
    return {
        "value": round((2 * R + 10 * C) / dt / 1e9, 3),
        "unit": "GB/s",
        "cores": offt.num_threads(),
        "kind": "oracle",
        "sample": "one forward+inverse pair of the 512^3 N(0,1) seed-0 field in FP64 (%.1f s)" % dt,
        "pair_s": round(dt, 3),
    }


def ns_steps_per_s(tk, torch, n, steps, warmup):
    """RK2 steps/s of the 512^3 decaying-turbulence configuration (CFL 0.5, nu 1e-3)."""
    import synth
    ns = tk.NS(n, dtype=torch.float32, nu=1e-3, cfl=0.5)
    noise = torch.from_numpy(synth.gaussian_field((3, n, n, n), 1)).cuda()
    u = ns.init_random(noise)
    del noise
    ns.step(u, 0.0, warmup)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ns.step(u, 0.0, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    e = ns.diagnostics(u)["energy"]
    ns.close()
    return steps / dt, e


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ns", action="store_true")
    ap.add_argument("--no-1024", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the multi-GPU (slab all-to-all) path is design-only "
              "in this library, so --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1805_07801_amd as tk
    tk.load()
    n = 512
    R, C = field_bytes(n)
    # the library's autotuner picks the tile shapes of each pass (untimed)
    for nn in ((512,) if args.no_1024 else (512, 1024)):
        tk.autotune(nn, iters=3)
    ms, passes, desc, err = time_pairs(tk, torch, n, args.steps, args.warmup)
    value = (2 * R + 10 * C) / (ms * 1e-3) / 1e9
    dom, roof = roofline(n, passes)
    pb = pass_bytes(n)
    out = {
        "metric": "3D FFT pair GB/s & %HBM peak at 512^3/1024^3 FP32; NS RK2 steps/sec",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fft3d_pair_512", "n": n, "batch": 1, "input": "N(0,1) seed 0",
                   "step": "forward r2c + inverse c2r"},
        "pct_hbm_peak": round(100 * value / HBM_PEAK_GBPS, 2),
        "compulsory_GBps": round(2 * (R + C) / (ms * 1e-3) / 1e9, 1),
        "gflops_paper_convention": round(pair_flops(n) / (ms * 1e-3) / 1e9, 1),
        "roundtrip_rel_l2": err,
        "passes_ms": {k: round(v, 4) for k, v in passes.items()},
        "passes_GBps": {k: round(pb[k] / (passes[k] * 1e-3) / 1e9, 1) for k in passes if passes[k] > 0},
        "tiles": desc,
        "roofline": roof,
    }
    if not args.no_1024:
        n2 = 1024
        R2, C2 = field_bytes(n2)
        k2 = max(5, args.steps // 5)
        ms2, passes2, desc2, err2 = time_pairs(tk, torch, n2, k2, max(2, args.warmup // 5))
        pb2 = pass_bytes(n2)
        out["fft1024"] = {
            "ms_per_pair": round(ms2, 3),
            "GBps": round((2 * R2 + 10 * C2) / (ms2 * 1e-3) / 1e9, 1),
            "pct_hbm_peak": round(100 * (2 * R2 + 10 * C2) / (ms2 * 1e-3) / 1e9 / HBM_PEAK_GBPS, 2),
            "gflops_paper_convention": round(pair_flops(n2) / (ms2 * 1e-3) / 1e9, 1),
            "passes_GBps": {k: round(pb2[k] / (passes2[k] * 1e-3) / 1e9, 1) for k in passes2 if passes2[k] > 0},
            "roundtrip_rel_l2": err2,
        }
    if not args.no_ns and hasattr(tk, "NS"):
        sps, e = ns_steps_per_s(tk, torch, 512, max(10, args.steps // 5), 2)
        out["ns512_rk2_steps_per_s"] = round(sps, 2)
        out["ns512_energy_after"] = e
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(512)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
