"""Rayleigh-Benard (Boussinesq) convection in the periodic FFF basis, FP64 (oracle; test
infrastructure).

Paper, Section "Spectral Solver": the nondimensional equations eq:u_Usmall_Plarge and
eq:T_Usmall_Plarge,
    d_t u + (u . grad) u = -grad sigma + theta z + sqrt(Pr/Ra) lap u,
    d_t theta + (u . grad) theta = u_z + lap theta / sqrt(Ra Pr),
with div u = 0, in the Fourier basis along all three axes (the paper's FFF runs).  The box
is periodic of side Lbox (wavenumbers scaled by a = 2 pi / Lbox; the paper's unit cube is
Lbox = 1).  Nonlinear terms pseudo-spectral and 2/3-dealiased: u x omega for momentum and
the conservative -i k . F(u theta) for temperature (div u = 0), so one right-hand side takes
7 inverse (u, omega, theta) and 6 forward (u x omega, u theta) transforms: 13, as the paper
counts for its RBC solver.  Time stepping: integrating-factor Heun with exp(-nu a^2 |k|^2 h)
for u and exp(-kappa a^2 |k|^2 h) for theta.
"""
import numpy as np

from . import fft, ns


def viscosities(Ra, Pr):
    return np.sqrt(Pr / Ra), 1.0 / np.sqrt(Ra * Pr)


def rhs(uhat, that, a=1.0):
    """(N_u, N_theta): N_u = P M [F(u x omega) + theta z], N_theta = M [-i a k . F(u theta) + u_z]
    (diffusion excluded)."""
    n = uhat.shape[-3]
    kx, ky, kz = ns.deriv_wavenumbers(n)
    k = (a * kx, a * ky, a * kz)
    ux, uy, uz = uhat
    what = np.stack([1j * (k[1] * uz - k[2] * uy), 1j * (k[2] * ux - k[0] * uz), 1j * (k[0] * uy - k[1] * ux)])
    u = fft.irfft3(uhat)
    w = fft.irfft3(what)
    th = fft.irfft3(that)
    c = np.stack([u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]])
    q = fft.rfft3(u * th[None])
    mask = ns.dealias_mask(n)
    chat = fft.rfft3(c)
    chat[2] = chat[2] + that
    Nu = ns.project(chat * mask)
    Nt = (-1j * (k[0] * q[0] + k[1] * q[1] + k[2] * q[2]) + uhat[2]) * mask
    return Nu, Nt


def ifrk2_step(uhat, that, nu, kappa, h, a=1.0):
    n = uhat.shape[-3]
    k2 = ns.k_squared(n) * a * a
    Eu = np.exp(-nu * k2 * h)
    Et = np.exp(-kappa * k2 * h)
    N0u, N0t = rhs(uhat, that, a)
    us = Eu * (uhat + h * N0u)
    ts = Et * (that + h * N0t)
    N1u, N1t = rhs(us, ts, a)
    return Eu * uhat + 0.5 * h * (Eu * N0u + N1u), Et * that + 0.5 * h * (Et * N0t + N1t)
