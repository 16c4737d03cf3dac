"""Pins for the oracle's Boussinesq (RBC, FFF basis) right-hand side and step (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import diag, fft, init, ns, rbc


def grid3(n):
    x = synth.grid(n)
    return x[:, None, None], x[None, :, None], x[None, None, :]


def rand_fields(n, seed):
    u = init.random_solenoidal(synth.gaussian_field((3, n, n, n), seed))
    t = fft.rfft3(synth.gaussian_field((n, n, n), seed + 1).astype(np.float64)) * ns.dealias_mask(n)
    t[0, 0, 0] = 0
    return u, t


def test_zero_temperature_reduces_to_navier_stokes():
    u, _ = rand_fields(16, 1)
    Nu, Nt = rbc.rhs(u, np.zeros_like(u[0]))
    assert np.max(np.abs(Nu - ns.rhs(u))) <= 1e-17
    assert np.max(np.abs(Nt - u[2] * ns.dealias_mask(16))) == 0


@pytest.mark.parametrize("a", [1.0, 2 * np.pi])
def test_single_temperature_mode_buoyancy(a):
    """u = 0, theta = cos(k0 . x): N_theta = 0 and N_u = P (theta z): the z component is
    theta^ (1 - kz^2/|k|^2), the others -k_i kz theta^/|k|^2."""
    n = 16
    X, Y, Z = grid3(n)
    t = fft.rfft3(np.cos(2 * X + 1 * Y + 3 * Z))
    Nu, Nt = rbc.rhs(np.zeros((3,) + t.shape, complex), t, a)
    assert np.max(np.abs(Nt)) == 0
    k = np.array([2.0, 1.0, 3.0])
    k2 = np.sum(k * k)
    c = t[2, 1, 3]
    assert abs(Nu[2, 2, 1, 3] - c * (1 - 9 / k2)) <= 1e-16
    assert abs(Nu[0, 2, 1, 3] + c * 2 * 3 / k2) <= 1e-16
    assert abs(Nu[1, 2, 1, 3] + c * 1 * 3 / k2) <= 1e-16


def test_advection_conserves_temperature_variance_and_buoyancy_exchange():
    n = 16
    u, t = rand_fields(n, 3)
    Nu, Nt = rbc.rhs(u, t)
    w = fft.hermitian_weight(n)
    # sum w Re(theta^* N_theta) = sum w Re(theta^* u_z): advection moves no variance
    adv = np.sum(w * np.real(np.conj(t) * (Nt - u[2] * ns.dealias_mask(n))))
    scale = np.sqrt(np.sum(w * np.abs(Nt) ** 2) * np.sum(w * np.abs(t) ** 2))
    assert abs(adv) <= 1e-14 * scale
    # kinetic energy changes only through buoyancy: sum w Re(u^* N_u) = sum w Re(u_z^* theta^)
    ke = np.sum(w * np.real(np.conj(u) * Nu))
    buoy = np.sum(w * np.real(np.conj(u[2]) * t))
    assert abs(ke - buoy) <= 1e-14 * scale


def test_linear_mode_second_order():
    """Small-amplitude single mode (nonlinear terms negligible): u_z, theta follow the 2x2
    linear system d/dt [u_z, theta] = [[-nu k^2, 1 - kz^2/k^2], [1, -kappa k^2]] [u_z, theta];
    IF-RK2 converges to its exact solution at second order."""
    n = 16
    X, Y, Z = grid3(n)
    eps = 1e-8
    t0 = fft.rfft3(eps * np.cos(1 * X + 0 * Y + 1 * Z))
    u0 = np.zeros((3,) + t0.shape, complex)
    nu, kappa = 0.05, 0.02
    k2 = 2.0
    A = np.array([[-nu * k2, 1 - 1 / k2], [1.0, -kappa * k2]])
    T = 0.8
    lam, V = np.linalg.eig(A)
    x0 = np.array([0.0, t0[1, 0, 1]])
    xT = V @ (np.exp(lam * T) * np.linalg.solve(V, x0))
    errs = []
    for steps in (8, 16, 32):
        u, t = u0.copy(), t0.copy()
        for _ in range(steps):
            u, t = rbc.ifrk2_step(u, t, nu, kappa, T / steps)
        errs.append(abs(t[1, 0, 1] - xT[1]) + abs(u[2, 1, 0, 1] - xT[0]))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def test_viscosities_from_rayleigh_prandtl():
    nu, kappa = rbc.viscosities(1.0e6, 1.0)
    assert abs(nu - 1e-3) <= 1e-18 and abs(kappa - 1e-3) <= 1e-18
