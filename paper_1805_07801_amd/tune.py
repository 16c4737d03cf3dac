"""Autotune the 3D FFT tile shapes on this GPU and save / load them as JSON lines.

    python -m paper_1805_07801_amd.tune --sizes 512 1024 64 96 128 --ns-sizes 512 256 128 64 --out FILE

Every candidate is checked against the default tile before it may be chosen (see
fft3d_autotune and ns_autotune in include/tk.h); the file records the choice per
(length, dtype, pass), passes 3-7 being the solver's P1, P3, P5, Y passes and fused P5 + P1.
"""
import argparse
import os
import re

import paper_1805_07801_amd as tk

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_gfx950.json")


def run(sizes, iters=5, dtype=None, ns_sizes=()):
    import torch
    dtype = dtype or torch.float32
    entries = []
    reports = []
    for n, solver in [(n, False) for n in sizes] + [(n, True) for n in ns_sizes]:
        rep = tk.ns_autotune(n, iters=iters, dtype=dtype) if solver else tk.autotune(n, iters=iters, dtype=dtype)
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
    ap.add_argument("--sizes", type=int, nargs="+", default=[512, 1024, 64, 96, 128, 32])
    ap.add_argument("--ns-sizes", type=int, nargs="*", default=[512, 256, 128, 64])
    ap.add_argument("--iters", type=int, default=7)
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    tk.load()
    entries, report = run(args.sizes, args.iters, ns_sizes=args.ns_sizes)
    tk.tune_save(args.out, entries)
    if args.report:
        with open(args.report, "w") as f:
            f.write(report)
    print("wrote %d tile choices to %s" % (len(entries), args.out))


if __name__ == "__main__":
    main()
