"""Pins for the oracle's Navier-Stokes right-hand side, time steppers, diagnostics and
initial fields (CPU only): closed forms, invariants and brute force."""
import itertools

import numpy as np
import pytest

import synth
from oracle import diag, fft, init, ns


def tg_state(n):
    return fft.rfft3(synth.taylor_green(n))


def grid3(n):
    x = synth.grid(n)
    return x[:, None, None], x[None, :, None], x[None, None, :]


@pytest.mark.parametrize("n", [8, 16, 32])
def test_taylor_green_vorticity_energy(n):
    """omega = (-cos x sin y sin z, -sin x cos y sin z, 2 sin x sin y cos z); E = 1/8; Omega = 3/8."""
    X, Y, Z = grid3(n)
    uh = tg_state(n)
    w = fft.irfft3(ns.curl(uh))
    ex = np.stack([-np.cos(X) * np.sin(Y) * np.sin(Z),
                   -np.sin(X) * np.cos(Y) * np.sin(Z),
                   2 * np.sin(X) * np.sin(Y) * np.cos(Z)])
    assert np.max(np.abs(w - ex)) <= 1e-14
    assert abs(diag.energy(uh) - 0.125) <= 1e-15
    assert abs(diag.enstrophy(uh) - 0.375) <= 1e-15
    assert abs(diag.dissipation(uh, 0.01) - 2 * 0.01 * 0.375) <= 1e-16


@pytest.mark.parametrize("n", [8, 16, 32])
def test_taylor_green_rhs_closed_form(n):
    """At t = 0 the TG nonlinear term is -u.grad u - grad p with the classical TG pressure
    p = (cos 2x + cos 2y)(cos 2z + 2)/16, i.e.
    ( -sin2x cos2z / 8, -sin2y cos2z / 8, (cos2x + cos2y) sin2z / 8 )."""
    X, Y, Z = grid3(n)
    ex = np.stack([-np.sin(2 * X) * np.cos(2 * Z) / 8 + 0 * Y,
                   -np.sin(2 * Y) * np.cos(2 * Z) / 8 + 0 * X,
                   (np.cos(2 * X) + np.cos(2 * Y)) * np.sin(2 * Z) / 8])
    got = ns.rhs(tg_state(n))
    assert np.max(np.abs(got - fft.rfft3(ex))) <= 1e-15


def random_masked_state(n, seed=0):
    noise = synth.gaussian_field((3, n, n, n), seed)
    return init.random_solenoidal(noise)


@pytest.mark.parametrize("n", [12, 16, 24])
def test_rhs_invariants(n):
    uh = random_masked_state(n, seed=n)
    N = ns.rhs(uh)
    kx, ky, kz = fft.wavenumbers(n)
    w = fft.hermitian_weight(n)
    # inviscid energy neutrality: sum w Re(u^* . N) = 0 (u . (u x omega) = 0 pointwise, exact under 2/3)
    p = np.sum(w * np.real(np.conj(uh) * N))
    assert abs(p) <= 1e-14 * np.sqrt(np.sum(w * np.abs(N) ** 2) * np.sum(w * np.abs(uh) ** 2))
    # divergence free, masked
    assert np.max(np.abs(kx * N[0] + ky * N[1] + kz * N[2])) <= 1e-13
    assert np.max(np.abs(N * ~ns.dealias_mask(n))) == 0.0
    assert np.max(np.abs(N[:, 0, 0, 0])) == 0.0
    # rotational form == conservative form (paper's eq:NSk)
    Nc = ns.rhs_conservative(uh)
    assert np.max(np.abs(N - Nc)) <= 1e-13 * np.max(np.abs(N))


def test_shear_wave_has_no_nonlinear_term():
    n = 16
    X, Y, Z = grid3(n)
    u = np.stack([np.cos(3 * Y + 0 * X + 0 * Z), np.zeros((n, n, n)), np.zeros((n, n, n))])
    assert np.max(np.abs(ns.rhs(fft.rfft3(u)))) <= 1e-16


def full_spectrum(Fh, n):
    """Hermitian extension of a half spectrum to the full [n][n][n] array of coefficients."""
    F = np.zeros((n, n, n), complex)
    F[:, :, : n // 2 + 1] = Fh
    for kz in range(n // 2 + 1, n):
        F[:, :, kz] = np.conj(Fh[(-np.arange(n)) % n][:, (-np.arange(n)) % n][:, :, n - kz])
    return F


@pytest.mark.parametrize("n", [10, 12])
def test_dealiased_product_equals_truncated_convolution(n):
    """With the 2/3 mask the pseudo-spectral product equals the exact convolution
    sum_{p+q=k} u^(p) x omega^(q) restricted to kept modes (brute-force O(M^2) sum)."""
    uh = random_masked_state(n, seed=3)
    wh = ns.curl(uh)
    u = fft.irfft3(uh)
    w = fft.irfft3(wh)
    c = np.stack([u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]])
    ch = fft.rfft3(c) * ns.dealias_mask(n)
    U = np.stack([full_spectrum(uh[i], n) for i in range(3)])
    W = np.stack([full_spectrum(wh[i], n) for i in range(3)])
    kmax = (n - 1) // 3
    kept = np.arange(-kmax, kmax + 1)
    P = np.array(list(itertools.product(kept, kept, kept)))
    Up = U[:, P[:, 0] % n, P[:, 1] % n, P[:, 2] % n]
    ref = np.zeros_like(ch)
    for (a, b, cz) in P:
        if cz < 0:
            continue
        Q = np.array([a, b, cz])[None, :] - P
        ok = np.max(np.abs(Q), axis=1) <= kmax
        Wq = W[:, Q[ok, 0] % n, Q[ok, 1] % n, Q[ok, 2] % n]
        acc = np.sum(np.cross(Up[:, ok].T, Wq.T), axis=0)
        ref[:, a % n, b % n, cz] = acc
    assert np.max(np.abs(ch - ref)) <= 1e-14


def test_single_mode_viscous_decay_exact():
    """A single shear wave has N = 0, so IF-RK2 reproduces u(t) = u(0) exp(-nu k^2 t) to round-off."""
    n = 16
    X, Y, Z = grid3(n)
    u = np.stack([np.sin(2 * Z + 0 * X + 0 * Y), np.zeros((n, n, n)), np.zeros((n, n, n))])
    uh0 = fft.rfft3(u)
    nu, h, steps = 0.05, 0.1, 20
    uh = uh0
    for _ in range(steps):
        uh = ns.ifrk2_step(uh, nu, h)[0]
    assert np.max(np.abs(uh - uh0 * np.exp(-nu * 4 * h * steps))) <= 1e-15


def test_ifrk2_second_order_on_taylor_green():
    n, nu, T = 16, 0.01, 0.4
    uh0 = tg_state(n)
    ref, _ = ns.run(uh0, nu, T / 64, 64, stepper=ns.ifrk4_step)
    errs = []
    for steps in (4, 8, 16):
        u, _ = ns.run(uh0, nu, T / steps, steps)
        errs.append(np.sqrt(np.sum(np.abs(u - ref) ** 2)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.6 and 3.5 < r2 < 4.6, errs


def test_ifrk4_fourth_order_on_taylor_green():
    n, nu, T = 16, 0.01, 0.8
    uh0 = tg_state(n)
    ref, _ = ns.run(uh0, nu, T / 128, 128, stepper=ns.ifrk4_step)
    errs = []
    for steps in (4, 8):
        u, _ = ns.run(uh0, nu, T / steps, steps, stepper=ns.ifrk4_step)
        errs.append(np.sqrt(np.sum(np.abs(u - ref) ** 2)))
    assert 12.0 < errs[0] / errs[1] < 20.0, errs


def test_inviscid_energy_drift_third_order():
    """nu = 0: the exact flow conserves energy, so a second-order step changes it by
    O(h^3) or less per step (ratio >= ~8 when h halves; the measured ratio is ~16)."""
    n = 16
    uh = random_masked_state(n, seed=11)
    e0 = diag.energy(uh)
    d = []
    for h in (0.02, 0.01):
        d.append(abs(diag.energy(ns.ifrk2_step(uh, 0.0, h)[0]) - e0))
    assert 6.0 < d[0] / d[1] < 20.0, d


def test_energy_budget_and_divergence():
    n, nu, h = 16, 0.02, 0.005
    uh = random_masked_state(n, seed=12)
    un = ns.ifrk2_step(uh, nu, h)[0]
    dE = diag.energy(un) - diag.energy(uh)
    pred = -h * 0.5 * (diag.dissipation(uh, nu) + diag.dissipation(un, nu))
    assert abs(dE - pred) <= 1e-3 * abs(pred)
    assert diag.max_divergence(un) <= 1e-13


def test_explicit_heun_matches_if_for_zero_viscosity():
    uh = random_masked_state(12, seed=4)
    a = ns.ifrk2_step(uh, 0.0, 0.01)[0]
    b = ns.heun_step(uh, 0.0, 0.01)
    assert np.max(np.abs(a - b)) <= 1e-15


@pytest.mark.parametrize("n", [16, 24])
def test_spectrum_sums_to_real_space_energy(n):
    uh = random_masked_state(n, seed=n + 1)
    u = fft.irfft3(uh)
    e_real = 0.5 * np.mean(np.sum(u ** 2, axis=0))
    assert abs(np.sum(diag.spectrum(uh)) - e_real) <= 1e-14
    assert abs(diag.energy(uh) - e_real) <= 1e-14


def test_shell_index_integer_rule():
    n = 32
    s = diag.shell_index(n)
    kx, ky, kz = fft.wavenumbers(n)
    k2 = np.broadcast_to(kx * kx + ky * ky + kz * kz, s.shape)
    assert np.all(((2 * s - 1) ** 2 <= 4 * k2) | (s == 0))
    assert np.all((s == 0) == (k2 == 0))
    assert np.all(4 * k2 < (2 * s + 1) ** 2)
    assert s.max() < diag.num_shells(n)


@pytest.mark.parametrize("n", [16, 24, 32])
def test_random_init_properties(n):
    uh = random_masked_state(n, seed=1)
    assert abs(diag.energy(uh) - 1.0) <= 1e-13
    assert diag.max_divergence(uh) <= 1e-13
    assert np.max(np.abs(uh * ~ns.dealias_mask(n))) == 0
    assert np.max(np.abs(uh[:, 0, 0, 0])) == 0
    E = diag.spectrum(uh)
    s = np.arange(len(E))
    ok = E > 0
    ratio = E[ok] / init.target_spectrum(s[ok])
    assert np.max(ratio) / np.min(ratio) <= 1 + 1e-12


def test_cfl_dt_taylor_green():
    """max(|u|+|v|+|w|) of TG sampled on a grid containing x = pi/4 points is 2 * (1/sqrt2)^2 ... exact:
    |sin x cos y cos z| + |cos x sin y cos z| peaks at 1 (x = y = pi/4, z = 0)."""
    n = 32
    h = ns.cfl_dt(tg_state(n), 0.5)
    assert abs(h - 0.5 * (2 * np.pi / n) / 1.0) <= 1e-14


def test_max_divergence_closed_forms():
    """u = (sin x, 0, 0) is a pure compression mode: |k.u^|/|k| = |u^| at k = (+-1,0,0), so
    the relative divergence is 1; Taylor-Green is solenoidal (0 to round-off)."""
    n = 16
    X, Y, Z = grid3(n)
    u = np.stack([np.sin(X + 0 * Y + 0 * Z), np.zeros((n, n, n)), np.zeros((n, n, n))])
    assert abs(diag.max_divergence(fft.rfft3(u)) - 1.0) <= 1e-14
    assert diag.max_divergence(tg_state(n)) <= 1e-15
    assert diag.max_divergence(np.zeros((3, n, n, n // 2 + 1), complex)) == 0.0
