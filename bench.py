#!/usr/bin/env python3
"""Benchmark of the 3D FFT pair and the Navier-Stokes step on one MI355X.

Headline: one forward r2c + inverse c2r pair of a 512^3 FP32 field of i.i.d. N(0,1)
values (seed 0), inputs resident in HBM, timed with HIP events over K pairs after W
warm-ups.  value = pair traffic of the three-pass plan (2 R + 10 C bytes, R = 4 N^3,
C = 8 N^2 (N/2+1)) divided by the pair time, in GB/s.  Also reported: the 1024^3 pair,
the per-pass kernel durations (HIP events on the launch stream), the roofline of the
dominant pass, the Navier-Stokes RK2 steps/s at 512^3 and the FP64 CPU oracle timed on
the host cores on one 512^3 pair.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-cpu-legs] [--no-ns]
                      [--no-1024] [--no-extra]
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


def ensemble_rate(tk, torch, steps=50):
    """The 48-member ensemble (16 x 64^3, 16 x 96^3, 16 x 128^3, CFL 0.5): member-steps/s,
    grid-point-steps/s and the achieved HBM rate over the members' algorithmic bytes per
    step (two stages of P2, P3, P4 and the fused P5+P1 each), one HIP-graph launch per
    ensemble step, HIP events on the launch stream."""
    import synth
    sizes = synth.ensemble_sizes()
    ens = tk.Ensemble(sizes, synth.ensemble_viscosities(), cfl=0.5)
    st = [ens.init_random(i, torch.from_numpy(synth.gaussian_field((3, m, m, m), synth.ensemble_seed(i))).cuda())
          for i, m in enumerate(sizes)]
    ens.step(st, 0.0, 2)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    ens.step(st, 0.0, steps)
    e1.record()
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3 / steps
    pts = sum(m ** 3 for m in sizes)
    step_bytes = 0
    for m in sizes:
        pb = ns_pass_bytes(m)
        step_bytes += 2 * sum(sum(pb[k]) for k in ("P2", "P3", "P4", "P5+P1"))
    ens.close()
    gbps = step_bytes / dt / 1e9
    return {"ensemble_steps_per_s": round(1 / dt, 2), "member_steps_per_s": round(len(sizes) / dt, 1),
            "point_steps_per_s": round(pts / dt, 1), "ensemble_alg_GB_per_step": round(step_bytes / 1e9, 3),
            "ensemble_GBps": round(gbps, 1), "ensemble_frac_hbm_peak": round(gbps / HBM_PEAK_GBPS, 3)}


MLP_FLOP_PER_POINT = 2 * (9 * 64 + 64 * 64 + 64 * 6)  # forward multiply-adds x 2
MFMA_F32_PEAK_TFLOPS = 157.3


def les_rate(tk, torch, steps=50):
    """64^3 LES steps/s with a closure network (random weights: the cost does not depend
    on them) and without; the network's forward kernel and its fused loss + backward at
    M = 64^3 points, in the definition's FP32 flops per second against the FP32 matrix
    peak.  The forward runs its products as exact three-term BF16 splits on the BF16
    matrix instruction (FP32 sums) and is bound by its GELUs' vector work; the backward
    runs on the FP32 matrix instruction."""
    import numpy as np
    import synth
    Ws, bs = synth.mlp_init(seed=7)
    theta = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in zip(Ws, bs)])
    net = tk.Closure(theta, in_scale=2.0, out_scale=1e-3)
    ns = tk.NS(64, dtype=torch.float32, nu=1e-3)
    u = ns.init_random(torch.from_numpy(synth.gaussian_field((3, 64, 64, 64), 3)).cuda())
    out = {}
    for name, model in (("les64_closure_steps_per_s", net), ("les64_plain_steps_per_s", None)):
        tk.les_step(ns, model, u, 1e-3, 2)
        ms = event_time(torch, lambda: tk.les_step(ns, model, u, 1e-3, steps), 1)
        out[name] = round(1e3 * steps / ms, 1)
    ns.close()
    M = 64 ** 3
    g = torch.Generator(device="cuda").manual_seed(5)
    x9 = torch.randn((9, M), generator=g, device="cuda")
    t6 = torch.randn((6, M), generator=g, device="cuda")
    y6 = torch.empty((6, M), device="cuda")
    net.forward(x9, y6)
    from paper_1805_07801_amd import les_train
    ms_f = event_time(torch, lambda: net.forward(x9, y6), 50)
    ms_b = event_time(torch, lambda: les_train._loss_grad_async(net, x9, t6), 20)
    for name, ms, flop, bound, instr in (
            ("mlp_forward", ms_f, MLP_FLOP_PER_POINT * M, "alu (GELU vector work)",
             "v_mfma_f32_16x16x32_bf16 on three-term BF16 splits of the activations"),
            ("mlp_loss_backward", ms_b, 3 * MLP_FLOP_PER_POINT * M, "mfma", "v_mfma_f32_16x16x4_f32")):
        tf = flop / (ms * 1e-3) / 1e12
        out[name + "_64cubed"] = {"ms": round(ms, 4), "GFLOP": round(flop / 1e9, 3), "TFLOPs": round(tf, 2),
                                  "bound": bound, "matrix_instruction": instr,
                                  "peak_TFLOPs": MFMA_F32_PEAK_TFLOPS, "frac": round(tf / MFMA_F32_PEAK_TFLOPS, 3)}
    return out


def time_pairs(tk, torch, n, steps, warmup, seed=0, repeats=False, overwrite=True):
    import numpy as np
    import synth
    f = synth.gaussian_field((n, n, n), seed)
    x = torch.from_numpy(f).cuda()
    del f
    # with overwrite, c2r may use its input as workspace (as FFTW's c2r does): every pass
    # stays in place; else c2r preserves its input (the X inverse writes a workspace)
    flags = tk.TK_FFT_TIMING | (tk.TK_FFT_C2R_OVERWRITE if overwrite else 0)
    plan = tk.FFT3D(n, dtype=torch.float32, flags=flags)
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
    # four more timed runs of the same K pairs, for the spread (the first run is `value`)
    reps = [ms]
    for _ in range(4 if repeats else 0):
        t0.record(stream)
        for _ in range(steps):
            plan.r2c(x, X)
            plan.c2r(X, y)
        t1.record(stream)
        torch.cuda.synchronize()
        reps.append(t0.elapsed_time(t1) / steps)
    names = ["z_r2c", "y_fwd", "x_fwd", "x_inv", "y_inv", "z_c2r"]
    passes = dict(zip(names, pt))
    desc = {p: plan.describe(p) for p in range(3)}
    err = (torch.linalg.vector_norm((y - x).double()) / torch.linalg.vector_norm(x.double())).item()
    plan.close()
    del x, X, y
    torch.cuda.empty_cache()
    return ms, passes, desc, err, reps


def kernel_names(desc, n):
    """Template names of the six pass kernels from the plan's tile descriptions."""
    import re
    z = re.search(r"LPW=(\d+) E=(\d+)", desc[0])
    names = {}
    if z:
        names["z_r2c"] = "k_z_r2c<float, %d, %s, %s>" % (n // 2, z.group(2), z.group(1))
        names["z_c2r"] = "k_z_c2r<float, %d, %s, %s>" % (n // 2, z.group(2), z.group(1))
    for p, keys in ((1, ("y_fwd", "y_inv")), (2, ("x_fwd", "x_inv"))):
        m = re.search(r"W=(\d+) E=(\d+) v=(\d+)", desc[p])
        if m:
            v = m.group(3)
            if v in ("1", "2", "3", "7", "8", "9"):  # persistent: <T, L, E, W, MASK, WPE>
                nt = int(m.group(1)) * n // int(m.group(2))
                wpe = 1 if v in ("1", "2", "3") else 2 * nt // 256
                name = "k_strided_pp<float, %d, %s, %s, false, %d>" % (n, m.group(2), m.group(1), wpe)
            else:  # one tile per workgroup: <T, L, E, W, MASK, SPLIT>
                name = "k_strided<float, %d, %s, %s, false, %s>" % (n, m.group(2), m.group(1),
                                                                     "true" if v in ("5", "6") else "false")
            names[keys[0]] = names[keys[1]] = name
    return names


def roofline(n, passes, names):
    """Roofline of the dominant kernel: the one with the largest time per pair (a kernel
    may run two passes, e.g. the X forward and inverse); achieved = algorithmic bytes per
    launch / its mean launch duration (HIP events on the launch stream)."""
    pb = pass_bytes(n)
    groups = {}
    for p, t in passes.items():
        groups.setdefault(names.get(p, p), []).append(p)
    dom = max(groups, key=lambda k: sum(passes[p] for p in groups[k]))
    ps = groups[dom]
    mean_ms = sum(passes[p] for p in ps) / len(ps)
    bytes_per_launch = pb[ps[0]]
    achieved = bytes_per_launch / (mean_ms * 1e-3) / 1e9
    return dom, {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBPS, 4),
        "traffic": None,
        "kernel_name": dom,
        "passes": ps,
        "launches_per_pair": len(ps),
        "kernel_ms_mean": round(mean_ms, 4),
        "bytes_per_launch": bytes_per_launch,
    }


def copy_bandwidth(torch, nbytes=1 << 29, reps=20):
    """Measured device copy bandwidth (read + write bytes / time) of a plain copy kernel on
    a 512 MiB buffer: the practical ceiling the passes are compared with."""
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        y.copy_(x)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del x, y
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def profile_record(summary, sources, key, kernel_name):
    """A per-launch figure of the named kernel from a committed rocprofv3 counter summary
    (lines `key <kernel name without spaces> <value>`), or None if the summary does not
    cover this kernel or the kernel sources changed since the counters were taken (the
    summary's `source_digest` line: sha256 of the listed sources, first 16 hex digits)."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", summary)
    if not os.path.exists(path):
        return None
    src = b""
    for f in sources:
        with open(os.path.join(here, "paper_1805_07801_amd", "csrc", f), "rb") as fh:
            src += fh.read()
    digest = hashlib.sha256(src).hexdigest()[:16]
    rec = {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) >= 3 and parts[0] == "source_digest":
                rec["digest"] = parts[1]
            if len(parts) >= 3 and parts[0] == key:
                rec[parts[1]] = float(parts[2])
    if rec.get("digest") != digest:
        return None
    return rec.get(kernel_name.replace(" ", ""))


def traffic_from_profile(kernel_name):
    """HBM bytes per launch of the named pair kernel (FETCH_SIZE + WRITE_SIZE, each scaled
    by the copy-kernel calibration)."""
    return profile_record("fft3d_pair_512_pmc.txt", ("fft_core.hpp", "fft_kernels.hpp"),
                          "traffic_bytes_per_launch", kernel_name)


# wave64 VALU instructions per second the chip can issue: 256 CUs x 4 SIMDs x 2.4 GHz, one
# wave64 instruction per SIMD every 4 cycles (= 39.3 T lane operations/s)
VALU_PEAK_GIPS = 256 * 4 * 2.4 / 4


def p3_kernel_name(n=512):
    """Template name of the solver's fused Z pass at n^3 FP32 under the committed tile cache
    (tile-table pass 4: a = lines per workgroup, E = points per thread; default 8 and 8)."""
    from paper_1805_07801_amd import tune
    a, E = 8, 8
    if os.path.exists(tune.DEFAULT_CACHE):
        with open(tune.DEFAULT_CACHE) as fh:
            for line in fh:
                if line.strip():
                    e = json.loads(line)
                    if e["L"] == n and e["dtype"] == 0 and e["pass"] == 4:
                        a, E = e["a"], e["E"]
    return "k_ns_p3<float, %d, %d, %d, false>" % (n // 2, E, a)


def p3_alu_roofline(ms):
    """ALU roofline of the fused Z pass of the 512^3 solver (six inverse and three forward
    line transforms with the products between them, bound by vector ALU issue): VALU
    instructions per launch from the committed counter summary / the live mean launch time."""
    name = p3_kernel_name(512)
    n_inst = profile_record("ns512_counters.txt", ("fft_core.hpp", "ns_kernels.hpp"),
                            "valu_instructions_per_launch", name)
    if n_inst is None:
        return None
    achieved = n_inst / (ms * 1e-3) / 1e9
    return {"bound": "alu", "achieved": round(achieved, 1), "peak": VALU_PEAK_GIPS,
            "unit": "G wave64 VALU instructions/s", "frac": round(achieved / VALU_PEAK_GIPS, 4),
            "instructions_per_launch": n_inst, "kernel_name": name}


def host_cores():
    """(physical cores, logical CPUs) of this host from lscpu (sockets x cores per socket)."""
    import subprocess
    logical = os.cpu_count() or 0
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        kv = {}
        for line in txt.splitlines():
            if ":" in line:
                a, b = line.split(":", 1)
                kv[a.strip()] = b.strip()
        return int(kv["Socket(s)"]) * int(kv["Core(s) per socket"]), int(kv.get("CPU(s)", logical))
    except Exception:
        return None, logical


def cpu_baseline(n=512, min_s=10.0, max_pairs=8):
    """The FP64 oracle (C, OpenMP over lines) on forward+inverse pairs of the same 512^3
    input, on the host cores: pairs are repeated until about min_s seconds of CPU work
    (at most max_pairs), and the mean pair time gives the rate."""
    import numpy as np
    import synth
    from oracle import fft as offt
    f = synth.gaussian_field((n, n, n), 0).astype(np.float64)
    times = []
    while len(times) < max_pairs and sum(times) < min_s:
        t = time.perf_counter()
        F = offt.rfft3(f)
        g = offt.irfft3(F)
        times.append(time.perf_counter() - t)
        del F, g
    dt = sum(times) / len(times)
    R, C = field_bytes(n)
    phys, logical = host_cores()
    return {
        "value": round((2 * R + 10 * C) / dt / 1e9, 3),
        "unit": "GB/s",
        "cores": offt.num_threads(),
        "kind": "oracle",
        "sample": "%d forward+inverse pairs of the 512^3 N(0,1) seed-0 field in FP64 (%.1f s in all)" % (
            len(times), sum(times)),
        "pair_s": round(dt, 3),
        "host_physical_cores": phys,
        "host_logical_cpus": logical,
    }


_CPU_LEG = r"""
import sys, time, json
sys.path.insert(0, %(root)r)
import numpy as np
import synth
from oracle import fft as offt, init as oinit, ns as ons
leg = %(leg)r
out = {"threads": offt.num_threads()}
if leg.startswith("pair"):
    n = int(leg[4:])
    f = synth.gaussian_field((n, n, n), 0).astype(np.float64)
    t = time.perf_counter()
    g = offt.irfft3(offt.rfft3(f))
    out["s"] = time.perf_counter() - t
elif leg == "scipy512":
    # library context, not the oracle: scipy's pocketfft on all logical CPUs, FP64 and FP32
    import os
    import scipy.fft as sf
    w = os.cpu_count() or 1
    out["threads"] = w
    f = synth.gaussian_field((512, 512, 512), 0)
    for key, dt in (("s", np.float64), ("s_fp32", np.float32)):
        x = f.astype(dt)
        t = time.perf_counter()
        g = sf.irfftn(sf.rfftn(x, workers=w), s=x.shape, workers=w)
        out[key] = time.perf_counter() - t
        del x, g
elif leg == "ns32":
    u = offt.rfft3(synth.taylor_green(32))
    t = time.perf_counter()
    k = 0
    while time.perf_counter() - t < 2.0:
        u = ons.ifrk2_step(u, 0.01, 0.01)[0]
        k += 1
    out["s"] = (time.perf_counter() - t) / k
else:
    n = 512
    u = oinit.random_solenoidal(synth.gaussian_field((3, n, n, n), 1))
    h = ons.cfl_dt(u, 0.5)
    t = time.perf_counter()
    ons.ifrk2_step(u, 1e-3, h)
    out["s"] = time.perf_counter() - t
print(json.dumps(out))
"""


def cpu_legs():
    """The oracle on the rest of the workloads, each in a child process: one 512^3 pair on
    one thread, one 1024^3 pair, and one IF-RK2 step of the 32^3 FP64 Taylor-Green case
    (repeated for 2 s) and of the 512^3 decaying-turbulence field, on all threads; and, as
    library context only, scipy.fft's 512^3 pair in FP64 and FP32."""
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    R, C = field_bytes(512)
    R2, C2 = field_bytes(1024)
    legs = {}
    for name, leg, env in (("pair512_1thread", "pair512", {"OMP_NUM_THREADS": "1"}), ("pair1024", "pair1024", {}),
                           ("ns32_fp64_step", "ns32", {}), ("ns512_step", "ns512", {}),
                           ("scipy_pair512_library_context", "scipy512", {})):
        e = dict(os.environ)
        e.update(env)
        try:
            r = subprocess.run([sys.executable, "-c", _CPU_LEG % {"root": here, "leg": leg}], capture_output=True,
                               text=True, env=e, timeout=600)
            d = json.loads(r.stdout.strip().splitlines()[-1])
        except Exception as ex:  # a leg that cannot run here is reported, not fatal
            legs[name] = {"error": str(ex)[:200]}
            continue
        rec = {"s": round(d["s"], 4), "threads": d["threads"]}
        if leg == "pair512":
            rec["GBps"] = round((2 * R + 10 * C) / d["s"] / 1e9, 3)
        elif leg == "scipy512":
            rec["kind"] = "library (scipy.fft), not the oracle"
            rec["s_fp32"] = round(d["s_fp32"], 4)
        elif leg == "pair1024":
            rec["GBps"] = round((2 * R2 + 10 * C2) / d["s"] / 1e9, 3)
        else:
            rec["steps_per_s"] = round(1.0 / d["s"], 4)
        legs[name] = rec
    return legs


def ns_pass_bytes(n):
    """Algorithmic HBM bytes (read, write) of each solver pass at n^3 FP32: kept modes of
    the 2/3 rule (K = (n-1)//3), transit rows of KZP complex values."""
    K = (n - 1) // 3
    KZP = min((K + 1 + 15) // 16 * 16, n // 2 + 1)
    kk = 2 * K + 1
    c = 8
    return {
        "P1": (3 * kk * kk * KZP * c, 6 * n * kk * KZP * c),
        "P2": (6 * n * KZP * kk * c, 6 * n * KZP * n * c),
        "P3": (6 * n * n * (K + 1) * c, 3 * n * n * KZP * c),
        "P4": (3 * n * KZP * n * c, 3 * n * KZP * kk * c),
        "P5": (3 * n * kk * KZP * c, 3 * kk * kk * KZP * c),
        "P5+P1": (3 * n * kk * KZP * c + 3 * kk * kk * KZP * c, 3 * kk * kk * KZP * c + 6 * n * kk * KZP * c),
    }


def event_time(torch, fn, reps):
    """Mean ms of fn() over reps calls, HIP events on the current stream."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def pass_entry(ms, rw, peak=HBM_PEAK_GBPS):
    """Per-kernel record: mean launch ms, algorithmic bytes, achieved GB/s and fraction of peak."""
    r, w = rw
    gbps = (r + w) / (ms * 1e-3) / 1e9
    return {"ms": round(ms, 4), "alg_MB": round((r + w) / 1e6, 1), "GBps": round(gbps, 1),
            "frac_hbm_peak": round(gbps / peak, 3)}


def ns_steps_per_s(tk, torch, n, steps, warmup):
    """RK2 steps/s of the 512^3 decaying-turbulence configuration (CFL 0.5, nu 1e-3), timed
    with HIP events on the launch stream over `steps` steps, and the achieved HBM rate of
    each solver pass (HIP events around each pass)."""
    import synth
    ns = tk.NS(n, dtype=torch.float32, nu=1e-3, cfl=0.5)
    noise = torch.from_numpy(synth.gaussian_field((3, n, n, n), 1)).cuda()
    u = ns.init_random(noise)
    del noise
    ns.step(u, 0.0, warmup)
    ms = event_time(torch, lambda: ns.step(u, 0.0, steps), 1)
    e = ns.diagnostics(u)["energy"]
    pt = ns.pass_times(u, iters=5)
    ns.close()
    passes = {}
    for k, rw in ns_pass_bytes(n).items():
        if pt.get(k, 0.0) > 0:
            passes[k] = pass_entry(pt[k], rw)
    if n == 512 and "P3" in passes:
        alu = p3_alu_roofline(pt["P3"])
        if alu:
            passes["P3"]["alu_roofline"] = alu
    return steps / (ms * 1e-3), e, passes


def rbc_pass_bytes(n):
    """Algorithmic HBM bytes (read, write) of each pass of the convection right-hand side at
    n^3 FP32 (kept modes, transit rows of KZP), as for the solver passes: P1 4 -> 7 fields,
    P2 7 fields, P3 7 -> 6, P4 6 fields, P5 6 transit fields plus theta and u_z of the input
    state -> 4 output fields."""
    K = (n - 1) // 3
    KZC = K + 1
    KZP = min((K + 1 + 15) // 16 * 16, n // 2 + 1)
    kk = 2 * K + 1
    c = 8
    return {
        "P1": (4 * kk * kk * KZP * c, 7 * n * kk * KZP * c),
        "P2": (7 * n * KZP * kk * c, 7 * n * KZP * n * c),
        "P3": (7 * n * n * KZC * c, 6 * n * n * KZP * c),
        "P4": (6 * n * KZP * n * c, 6 * n * KZP * kk * c),
        "P5": (6 * n * kk * KZC * c + 2 * kk * kk * KZC * c, 4 * kk * kk * KZC * c),
    }


def extension_rates(tk, torch, n=512):
    """The rows built beyond the hot path, each at 512^3 FP32: IF-RK4 steps/s of the
    decaying-turbulence field (CFL 0.5), the energy-transfer diagnostics, Rayleigh-Benard
    (FFF) IF-RK2 steps/s with the GB/s of each of its passes, and the sine-basis (SFF) and
    all-sine/cosine (SSS) transform pairs with the GB/s of each pass; and the IF-RK2 solver
    at 1024^3, HIP events throughout."""
    import synth
    out = {}
    R, C = field_bytes(n)
    noise = torch.from_numpy(synth.gaussian_field((3, n, n, n), 1)).cuda()
    ns = tk.NS(n, dtype=torch.float32, nu=1e-3, cfl=0.5, scheme="rk4")
    u = ns.init_random(noise)
    del noise
    ns.step(u, 0.0, 2)
    k = 20
    out["ns512_rk4_steps_per_s"] = round(1e3 * k / event_time(torch, lambda: ns.step(u, 0.0, k), 1), 2)
    # energy transfer T(s) (one right-hand side plus a shell reduction of u^* . N) and a
    # 4-band shell-to-shell matrix of the same state
    nsh = tk.num_shells(n)
    ns.energy_transfer(u)
    ms = event_time(torch, lambda: ns.energy_transfer(u), 3)
    pb = ns_pass_bytes(n)
    K = (n - 1) // 3
    kk = 2 * K + 1
    rw = (sum(pb[p][0] for p in ("P1", "P2", "P3", "P4", "P5")) + 6 * kk * kk * (K + 1) * 8,
          sum(pb[p][1] for p in ("P1", "P2", "P3", "P4", "P5")))
    out["transfer512"] = pass_entry(ms, rw)
    bands = [min(3, s // 8) for s in range(nsh)]
    t = time.perf_counter()
    ns.shell_to_shell(u, bands, 4)
    torch.cuda.synchronize()
    out["shell_to_shell512_4bands_ms"] = round((time.perf_counter() - t) * 1e3, 2)
    ns.close()
    del u
    # convection: random small state (u, theta), Ra 1e6, Pr 1
    rbc = tk.RBC(n, Ra=1e6, Pr=1.0)
    g = torch.Generator(device="cuda").manual_seed(3)
    s4 = (torch.randn((4, n, n, n // 2 + 1), generator=g, device="cuda", dtype=torch.complex64) * 1e-6).contiguous()
    rbc.step(s4, 1e-4, 2)
    k = 20
    out["rbc512_rk2_steps_per_s"] = round(1e3 * k / event_time(torch, lambda: rbc.step(s4, 1e-4, k), 1), 2)
    pt = rbc.pass_times(s4, iters=5)
    out["rbc512_passes"] = {p: pass_entry(pt[p], rw) for p, rw in rbc_pass_bytes(n).items()}
    del s4, rbc
    torch.cuda.empty_cache()
    # sine basis along x (SFF), and cos / cos / sin on every axis (SSS): r2c + c2r pairs
    x = torch.randn((1, n, n, n), generator=g, device="cuda", dtype=torch.float32)
    for name, kw, pbytes in (("sff512", {"basis_x": 1}, pass_bytes(n)),
                             ("sss512", {"basis_x": 2, "basis_y": 2, "basis_z": 1},
                              {p: 2 * R for p in ("z_r2c", "y_fwd", "x_fwd", "x_inv", "y_inv", "z_c2r")})):
        plan = tk.FFT3D(n, dtype=torch.float32, flags=tk.TK_FFT_TIMING, **kw)
        X = plan.empty_cplx()
        y = plan.empty_real()

        def pair():
            plan.r2c(x, X)
            plan.c2r(X, y)

        for _ in range(3):
            pair()
        torch.cuda.synchronize()
        plan.pass_times()
        ms = event_time(torch, pair, 10)
        pt = plan.pass_times()
        names = ["z_r2c", "y_fwd", "x_fwd", "x_inv", "y_inv", "z_c2r"]
        out[name + "_pair_ms"] = round(ms, 4)
        out[name + "_pair_GBps"] = round(sum(pbytes.values()) / (ms * 1e-3) / 1e9, 1)
        out[name + "_passes"] = {p: pass_entry(t, (pbytes[p] / 2, pbytes[p] / 2)) for p, t in zip(names, pt)}
        plan.close()
        del X, y
    del x
    torch.cuda.empty_cache()
    # the solver at its largest grid: 1024^3 IF-RK2 (CFL 0.5) of a random solenoidal field
    # (noise drawn on the device; the 15 fields of the solver take 65 GB of the 288 GB)
    m = 1024
    noise = torch.randn((3, m, m, m), generator=g, device="cuda", dtype=torch.float32)
    ns = tk.NS(m, dtype=torch.float32, nu=5e-4, cfl=0.5)
    u = ns.init_random(noise)
    del noise
    ns.step(u, 0.0, 2)
    k = 10
    ms = event_time(torch, lambda: ns.step(u, 0.0, k), 1) / k
    pb = ns_pass_bytes(m)
    step_bytes = 2 * sum(sum(pb[p]) for p in ("P2", "P3", "P4", "P5+P1"))
    out["ns1024_rk2"] = {"steps_per_s": round(1e3 / ms, 2), "ms_per_step": round(ms, 3),
                         "alg_GB_per_step": round(step_bytes / 1e9, 2),
                         "GBps": round(step_bytes / (ms * 1e-3) / 1e9, 1),
                         "frac_hbm_peak": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3)}
    ns.close()
    del u
    torch.cuda.empty_cache()
    return out


def tg32_steps_per_s(tk, torch, steps=200):
    """Steps/s of the 32^3 FP64 Taylor-Green configuration (nu 0.01, fixed dt 0.01, IF-RK2):
    launch/latency-bound, one graph launch per step."""
    import synth
    from paper_1805_07801_amd import FFT3D
    n = 32
    plan = FFT3D(n, batch=3, dtype=torch.float64)
    u = plan.r2c(torch.from_numpy(synth.taylor_green(n)).cuda())
    plan.close()
    ns = tk.NS(n, dtype=torch.float64, nu=0.01)
    ns.step(u, 0.01, 10)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ns.step(u, 0.01, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ns.close()
    return steps / dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-cpu-legs", action="store_true", help="time only the 512^3 oracle pair on the host")
    ap.add_argument("--no-ns", action="store_true")
    ap.add_argument("--no-1024", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the ensemble and LES measurements")
    ap.add_argument("--retune", action="store_true", help="autotune instead of using the committed cache")
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
    # tile shapes: the committed autotuner cache for this GPU, else a fresh autotune (untimed)
    from paper_1805_07801_amd import tune
    if args.retune or tune.load_default() == 0:
        for nn in ((512,) if args.no_1024 else (512, 1024)):
            tk.autotune(nn, iters=3)
    copy_gbps = copy_bandwidth(torch)
    ms, passes, desc, err, reps = time_pairs(tk, torch, n, args.steps, args.warmup, repeats=True)
    value = (2 * R + 10 * C) / (ms * 1e-3) / 1e9
    kname, roof = roofline(n, passes, kernel_names(desc, n))
    roof["traffic"] = traffic_from_profile(kname)
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
                   "step": "forward r2c + inverse c2r", "c2r_input": "used as workspace (TK_FFT_C2R_OVERWRITE)"},
        "pct_hbm_peak": round(100 * value / HBM_PEAK_GBPS, 2),
        "copy_GBps_measured": round(copy_gbps, 1),
        "pct_of_measured_copy": round(100 * value / copy_gbps, 2),
        "compulsory_GBps": round(2 * (R + C) / (ms * 1e-3) / 1e9, 1),
        "gflops_paper_convention": round(pair_flops(n) / (ms * 1e-3) / 1e9, 1),
        "roundtrip_rel_l2": err,
        "pair_ms_repeats": [round(r, 4) for r in reps],
        "pair_ms_median_of_5": round(sorted(reps)[len(reps) // 2], 4),
        "passes_ms": {k: round(v, 4) for k, v in passes.items()},
        "passes_GBps": {k: round(pb[k] / (passes[k] * 1e-3) / 1e9, 1) for k in passes if passes[k] > 0},
        "tiles": desc,
        "roofline": roof,
    }
    # the same pair with a c2r that preserves its input (the ABI default)
    ms_p, passes_p, _, err_p, _ = time_pairs(tk, torch, n, max(10, args.steps // 2), 2, overwrite=False)
    out["pair_input_preserving"] = {
        "ms_per_pair": round(ms_p, 4),
        "GBps": round((2 * R + 10 * C) / (ms_p * 1e-3) / 1e9, 1),
        "passes_GBps": {k: round(pb[k] / (passes_p[k] * 1e-3) / 1e9, 1) for k in passes_p if passes_p[k] > 0},
        "roundtrip_rel_l2": err_p,
    }
    if not args.no_1024:
        n2 = 1024
        R2, C2 = field_bytes(n2)
        k2 = max(5, args.steps // 5)
        ms2, passes2, desc2, err2, _ = time_pairs(tk, torch, n2, k2, max(2, args.warmup // 5))
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
        nsteps = max(50, args.steps // 2)
        sps, e, nsp = ns_steps_per_s(tk, torch, 512, nsteps, 2)
        out["ns512_timed_steps"] = nsteps
        out["ns512_rk2_steps_per_s"] = round(sps, 2)
        out["ns512_energy_after"] = e
        out["ns512_passes"] = nsp
        out["tg32_fp64_rk2_steps_per_s"] = round(tg32_steps_per_s(tk, torch), 1)
    if not args.no_extra:
        out.update(extension_rates(tk, torch))
        out.update(ensemble_rate(tk, torch))
        out.update(les_rate(tk, torch))
        if "ns512_rk2_steps_per_s" in out:
            out["les64_over_dns512_speed"] = round(out["les64_closure_steps_per_s"] / out["ns512_rk2_steps_per_s"], 1)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(512)
        if not args.no_cpu_legs:
            out["cpu_baseline"]["legs"] = cpu_legs()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
