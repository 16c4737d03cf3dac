"""Pseudo-spectral incompressible Navier-Stokes in a periodic (2 pi)^3 box (oracle; FP64).

TEST INFRASTRUCTURE.  Follows the paper's Section "Spectral Solver": the Fourier-space
momentum equation (eq:NSk) with the incompressibility constraint (eq:continuity2),
the nonlinear term evaluated pseudo-spectrally (transform to real space, multiply,
transform back) and dealiased by the 2/3 rule.  Written step by step, each step a
plain array expression; no fusion.

Readings taken where the paper is silent (each is listed in the design notes):
  * nonlinear term in rotational form u x omega; identical after projection to the
    paper's -i k_l (u_l u_j)^ form, which is also implemented (``rhs_conservative``);
  * 2/3 rule as a cube: keep a mode only if 3|kx| < N, 3|ky| < N and 3 kz < N;
  * odd derivatives of the Nyquist wavenumber are taken as zero;
  * the pressure term is the projection P = I - k k^T / |k|^2, with N(0) = 0;
  * time stepping: integrating-factor Heun (RK2) on v = exp(nu |k|^2 t) u^, so the
    viscous term is exact; plain explicit Heun and classical RK4 variants are given.
"""
import numpy as np

from . import fft


def deriv_wavenumbers(n):
    """Wavenumbers for odd (first) derivatives: as ``fft.wavenumbers`` but with the
    Nyquist entry (index n/2, on every axis) set to zero."""
    kx, ky, kz = fft.wavenumbers(n)
    kx = np.where(np.abs(kx) == n // 2, 0, kx)
    ky = np.where(np.abs(ky) == n // 2, 0, ky)
    kz = np.where(kz == n // 2, 0, kz)
    return kx, ky, kz


def dealias_mask(n):
    """2/3 rule (paper, Section "Spectral Solver"): True where the mode is kept."""
    kx, ky, kz = fft.wavenumbers(n)
    return (3 * np.abs(kx) < n) & (3 * np.abs(ky) < n) & (3 * kz < n)


def k_squared(n):
    kx, ky, kz = fft.wavenumbers(n)
    return (kx * kx + ky * ky + kz * kz).astype(np.float64)


def curl(uhat):
    """omega^ = i k x u^ for a [3][n][n][n/2+1] spectral field."""
    n = uhat.shape[-3]
    kx, ky, kz = deriv_wavenumbers(n)
    ux, uy, uz = uhat
    return np.stack([
        1j * (ky * uz - kz * uy),
        1j * (kz * ux - kx * uz),
        1j * (kx * uy - ky * ux),
    ])


def project(chat):
    """Leray projection c^ - k (k . c^) / |k|^2; the k = 0 mode is set to zero."""
    n = chat.shape[-3]
    kx, ky, kz = fft.wavenumbers(n)
    k2 = k_squared(n)
    kdotc = kx * chat[0] + ky * chat[1] + kz * chat[2]
    inv = np.zeros_like(k2)
    np.divide(1.0, k2, out=inv, where=k2 > 0)
    out = np.stack([chat[0] - kx * kdotc * inv, chat[1] - ky * kdotc * inv, chat[2] - kz * kdotc * inv])
    out[:, 0, 0, 0] = 0.0
    return out


def rhs(uhat):
    """Nonlinear term N(u^) = P M F[u x omega] (no viscous term).

    1. omega^ = i k x u^       2. u = F^-1 u^, omega = F^-1 omega^
    3. c = u x omega (pointwise)  4. c^ = F c
    5. M: 2/3 mask              6. P: projection, N(0) = 0
    """
    n = uhat.shape[-3]
    what = curl(uhat)
    u = fft.irfft3(uhat)
    w = fft.irfft3(what)
    c = np.stack([
        u[1] * w[2] - u[2] * w[1],
        u[2] * w[0] - u[0] * w[2],
        u[0] * w[1] - u[1] * w[0],
    ])
    chat = fft.rfft3(c)
    chat = chat * dealias_mask(n)
    return project(chat)


def rhs_conservative(uhat):
    """The paper's eq:NSk form: N_j = -P M [ i k_l F(u_l u_j) ]."""
    n = uhat.shape[-3]
    kx, ky, kz = deriv_wavenumbers(n)
    u = fft.irfft3(uhat)
    k = (kx, ky, kz)
    out = []
    for j in range(3):
        acc = 0
        for l in range(3):
            acc = acc + 1j * k[l] * fft.rfft3(u[l] * u[j])
        out.append(-acc)
    chat = np.stack(out) * dealias_mask(n)
    return project(chat)


def cfl_dt(uhat, cfl):
    """h = cfl * dx / max_x(|u_x| + |u_y| + |u_z|), dx = 2 pi / N."""
    n = uhat.shape[-3]
    u = fft.irfft3(uhat)
    umax = np.max(np.abs(u[0]) + np.abs(u[1]) + np.abs(u[2]))
    return cfl * (2.0 * np.pi / n) / umax


def ifrk2_step(uhat, nu, h, rhs_fn=rhs):
    """One integrating-factor Heun step, E = exp(-nu |k|^2 h):
         u* = E (u + h N(u)),   u+ = E u + (h/2) (E N(u) + N(u*)).
    Returns (u+, N(u), u*)."""
    n = uhat.shape[-3]
    E = np.exp(-nu * k_squared(n) * h)
    N0 = rhs_fn(uhat)
    ustar = E * (uhat + h * N0)
    N1 = rhs_fn(ustar)
    unew = E * uhat + 0.5 * h * (E * N0 + N1)
    return unew, N0, ustar


def heun_step(uhat, nu, h, rhs_fn=rhs):
    """Explicit Heun on du/dt = N(u) - nu |k|^2 u (alternative reading of RK2)."""
    n = uhat.shape[-3]
    k2 = k_squared(n)

    def f(v):
        return rhs_fn(v) - nu * k2 * v

    k1 = f(uhat)
    k2v = f(uhat + h * k1)
    return uhat + 0.5 * h * (k1 + k2v)


def ifrk4_step(uhat, nu, h, rhs_fn=rhs):
    """Classical RK4 on v = exp(nu |k|^2 t) u^ (integrating factor), the paper's
    fourth-order Runge-Kutta time stepping (Section "Scaling of Fluid spectral solver")."""
    n = uhat.shape[-3]
    k2 = k_squared(n)
    Eh = np.exp(-nu * k2 * h)
    Eh2 = np.exp(-nu * k2 * 0.5 * h)
    a1 = rhs_fn(uhat)
    a2 = rhs_fn(Eh2 * (uhat + 0.5 * h * a1))
    a3 = rhs_fn(Eh2 * uhat + 0.5 * h * a2)
    a4 = rhs_fn(Eh * uhat + h * Eh2 * a3)
    return Eh * uhat + (h / 6.0) * (Eh * a1 + 2.0 * Eh2 * (a2 + a3) + a4)


def run(uhat, nu, h, nsteps, stepper=ifrk2_step, cfl=None):
    """Advance nsteps; with cfl set, h is recomputed from u at the start of each step."""
    t = 0.0
    for _ in range(nsteps):
        hh = cfl_dt(uhat, cfl) if cfl else h
        res = stepper(uhat, nu, hh)
        uhat = res[0] if isinstance(res, tuple) else res
        t += hh
    return uhat, t
