"""Training and a-posteriori evaluation of the learned sub-grid closure.

Orchestration only: every operation on field data runs in libtk's kernels (DNS steps,
box filtering, network forward / backward / Adam, LES steps, spectra).

Workflow (the LES configuration: 64^3 LES of the 512^3 decaying-turbulence DNS):
  1. dns_snapshots: run the DNS with the solver and filter snapshots with the box
     |k_i| <= kc onto the LES grid (gradients and sub-grid stress per point).
  2. train: Adam on the mean-square stress error in normalised units; the input and
     output scales are the RMS of the training gradients and stresses.
  3. a_posteriori: from the filtered DNS at an intermediate time, run the LES with and
     without the closure to the final DNS time and compare shell spectra with the
     filtered DNS spectrum.
"""
import math

import paper_1805_07801_amd as tk


def filtered_spectrum(ens_ns, ubar_hat):
    return ens_ns.diagnostics(ubar_hat)["spectrum"]


def dns_snapshots(n=512, seed=1, nu=1e-3, cfl=0.5, nsteps=200, snap_steps=(), n_les=64, kc=21, keep_ubar=(),
                  noise_fn=None):
    """Run the DNS; at each step in snap_steps return (step, t, grad9, tau6); for steps in
    keep_ubar also the filtered state.  Returns (snapshots, filtered states, final time,
    DNS steps/s)."""
    import time
    import torch
    ns = tk.NS(n, dtype=torch.float32, nu=nu, cfl=cfl)
    noise = noise_fn(seed)
    u = ns.init_random(noise)
    del noise
    torch.cuda.empty_cache()
    snaps, ubars = [], {}
    t = 0.0
    done = 0
    marks = sorted(set(list(snap_steps) + list(keep_ubar) + [nsteps]))
    elapsed = 0.0
    for m in marks:
        if m > done:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t = ns.step(u, 0.0, m - done, t)
            elapsed += time.perf_counter() - t0
            done = m
        if m in snap_steps or m in keep_ubar:
            g, tau, ub = tk.les_filter_dns(u, n_les, kc, with_ubar=True)
            if m in snap_steps:
                snaps.append((m, t, g, tau))
            if m in keep_ubar:
                ubars[m] = (t, ub)
    ns.close()
    del u
    torch.cuda.empty_cache()
    return snaps, ubars, t, nsteps / elapsed if elapsed > 0 else float("nan")


def scales(snaps):
    g2 = sum(tk.sum_squares(g) for (_, _, g, _) in snaps)
    t2 = sum(tk.sum_squares(tau) for (_, _, _, tau) in snaps)
    ng = sum(g.numel() for (_, _, g, _) in snaps)
    nt = sum(tau.numel() for (_, _, _, tau) in snaps)
    return math.sqrt(g2 / ng), math.sqrt(t2 / nt)


def train(snaps, theta0, steps=1500, lr=2e-3, lr_final=2e-4, log_every=250):
    """Adam over full snapshots taken in turn, with a geometric learning-rate decay.
    Returns (closure, log) with log = [(step, mean loss over all snapshots)]."""
    s_in, s_out = scales(snaps)
    net = tk.Closure(theta0, in_scale=s_in, out_scale=s_out, lr=lr)
    log = [(0, mean_loss(net, snaps))]
    decay = (lr_final / lr) ** (1.0 / max(1, steps - 1))
    for k in range(steps):
        _, _, g, tau = snaps[k % len(snaps)]
        _loss_grad_async(net, g, tau)
        net.adam_step()
        net.opt.lr = lr * decay ** (k + 1)
        if (k + 1) % log_every == 0 or k + 1 == steps:
            log.append((k + 1, mean_loss(net, snaps)))
    return net, log


def mean_loss(net, snaps):
    """Mean normalised loss over snapshots (the gradient buffer is overwritten)."""
    return sum(net.loss_grad(g, tau) for (_, _, g, tau) in snaps) / len(snaps)


def snapshot_losses(net, snaps):
    return [(m, net.loss_grad(g, tau)) for (m, _, g, tau) in snaps]


def _loss_grad_async(net, g, tau):
    import ctypes
    d = net.desc()
    tk.check(tk.lib().sgs_mlp_loss_grad(ctypes.byref(d), tk._ptr(g), tk._ptr(tau), g.shape[-1], tk._ptr(net.grad),
                                        None, tk._stream()))
    return None


def spectrum_error(E, Eref, s_lo=1, s_hi=21):
    """Mean and max over shells s_lo..s_hi of |E - Eref| / Eref."""
    errs = [abs(E[s] - Eref[s]) / Eref[s] for s in range(s_lo, s_hi + 1) if Eref[s] > 0]
    return sum(errs) / len(errs), max(errs)


def les_run(net, ubar_hat0, t0, t1, nu, n_les=64, nsteps=None, cfl=0.5):
    """LES from ubar_hat0 at t0 to t1 with a fixed step that keeps the CFL number below
    `cfl` at t0; returns (final state, steps, steps/s, fallback)."""
    import time
    import torch
    ns = tk.NS(n_les, dtype=torch.float32, nu=nu, cfl=cfl)
    u = ubar_hat0.clone()
    # CFL step of the initial field, then a whole number of equal steps to t1
    ns_probe = tk.NS(n_les, dtype=torch.float32, nu=nu, cfl=cfl)
    up = u.clone()
    ns_probe.step(up, 0.0, 1)
    h_cfl = ns_probe.last_dt()
    ns_probe.close()
    if nsteps is None:
        nsteps = max(1, int(math.ceil((t1 - t0) / h_cfl)))
    dt = (t1 - t0) / nsteps
    ns_fixed = tk.NS(n_les, dtype=torch.float32, nu=nu)
    tk.les_step(ns_fixed, net, u, dt, 1, t0)  # warm-up on a copy is not needed; measure from here
    u = ubar_hat0.clone()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    t, fb = tk.les_step(ns_fixed, net, u, dt, nsteps, t0)
    torch.cuda.synchronize()
    rate = nsteps / (time.perf_counter() - t_start)
    spec = ns_fixed.diagnostics(u)["spectrum"]
    ns_fixed.close()
    ns.close()
    return u, spec, nsteps, rate, fb
