"""Autotune the 3D FFT tile shapes on this GPU and save / load them as JSON lines.

    python -m paper_1805_07801_amd.tune --sizes 512 1024 64 96 128 --ns-sizes 512 256 128 64 \
        --batch-sizes 128 96 64 --out FILE

Every candidate is checked against the default tile before it may be chosen (see
fft3d_autotune and ns_autotune in include/tk.h); the file records the choice per
(length, dtype, pass), passes 3-7 being the solver's P1, P3, P5, Y passes and fused P5 + P1,
pass 8 the ensemble kernels' thread count and persistent grid.
"""
import argparse
import os
import re

import paper_1805_07801_amd as tk

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_gfx950.json")


def run(sizes, iters=5, dtype=None, ns_sizes=(), batch_sizes=()):
    import torch
    dtype = dtype or torch.float32
    entries = []
    reports = []
    jobs = [(n, "fft") for n in sizes] + [(n, "ns") for n in ns_sizes] + [(n, "batch") for n in batch_sizes]
    for n, kind in jobs:
        if kind == "ns":
            rep = tk.ns_autotune(n, iters=iters, dtype=dtype)
        elif kind == "batch":
            rep = tk.ns_batch_autotune(n, members=16, iters=iters)
        else:
            rep = tk.autotune(n, iters=iters, dtype=dtype)
        reports.append(rep)
        for line in rep.splitlines():
            m = re.match(r"chosen pass (\d) L=(\d+): a=(\d+) E=(\d+) v=(\d+)", line)
            if m and int(m.group(3)) > 0:
                p, L, a, E, v = (int(x) for x in m.groups())
                entries.append((L, tk._dtype_code(dtype), p, a, E, v))
    return entries, "\n".join(reports)


def load_default():
    """Apply the committed cache if present; returns the number of entries applied."""
    if os.path.exists(DEFAULT_CACHE):
        return tk.tune_load(DEFAULT_CACHE)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="*", default=[512, 1024, 64, 96, 128, 32])
    ap.add_argument("--ns-sizes", type=int, nargs="*", default=[512, 256, 128, 64])
    ap.add_argument("--batch-sizes", type=int, nargs="*", default=[128, 96, 64])
    ap.add_argument("--iters", type=int, default=7)
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--report", default=None)
    ap.add_argument("--merge", action="store_true", help="keep the file's other entries, replace the re-tuned ones")
    args = ap.parse_args()
    tk.load()
    entries, report = run(args.sizes, args.iters, ns_sizes=args.ns_sizes, batch_sizes=args.batch_sizes)
    if args.merge and os.path.exists(args.out):
        import json
        keep = []
        tuned = {(L, dt, p) for (L, dt, p, _, _, _) in entries}
        with open(args.out) as f:
            for line in f:
                if line.strip():
                    e = json.loads(line)
                    if (e["L"], e["dtype"], e["pass"]) not in tuned:
                        keep.append((e["L"], e["dtype"], e["pass"], e["a"], e["E"], e.get("v", 0)))
        entries = keep + entries
    tk.tune_save(args.out, entries)
    if args.report:
        with open(args.report, "w") as f:
            f.write(report)
    print("wrote %d tile choices to %s" % (len(entries), args.out))


if __name__ == "__main__":
    main()
