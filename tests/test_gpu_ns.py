"""Parity of the HIP Navier-Stokes path with the FP64 oracle (GPU).

Tolerances (relative L2, Hermitian-weighted): right-hand side 1e-5 (FP32) / 1e-12 (FP64);
one step from a shared state 1e-4 (FP32) / 1e-12 (FP64).
"""
import numpy as np
import pytest

import synth
from oracle import diag, fft as offt, init as oinit, ns as ons

pytestmark = pytest.mark.gpu


def tdt(name):
    import torch
    return {"f32": torch.float32, "f64": torch.float64}[name]


def to_gpu(a, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64 if dt == "f32" else np.complex128))).cuda()


def rand_state(n, seed):
    return oinit.random_solenoidal(synth.gaussian_field((3, n, n, n), seed))


def band_state(n, seed):
    """Every kept mode O(1): parity measured on this field sees the whole 2/3 band (the
    decaying-turbulence field holds almost no energy beyond shell 20)."""
    return oinit.band_filling(synth.gaussian_field((3, n, n, n), seed))


def assert_shells(got, ref, n, tol):
    """Relative L2 error of every shell 1..K (K = (n-1)//3, the 2/3 cutoff) within tol."""
    K = (n - 1) // 3
    e = diag.shell_rel_l2(got, ref, n, range(1, K + 1))
    assert np.max(e) <= tol, (int(np.argmax(e)) + 1, float(np.max(e)))


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("n", [8, 12, 16, 24, 32, 48, 64, 96, 128])
def test_rhs_vs_oracle(tk, n, dt):
    u = rand_state(n, seed=n)
    ref = ons.rhs(u)
    s = tk.NS(n, dtype=tdt(dt), nu=0.0)
    got = s.rhs(to_gpu(u, dt)).cpu().numpy()
    tol = 1e-5 if dt == "f32" else 1e-12
    assert diag.rel_l2(got, ref, n) <= tol
    # masked modes exactly zero
    assert np.max(np.abs(got * ~ons.dealias_mask(n))) == 0


@pytest.mark.parametrize("n", [128, 192, 256])
def test_rhs_every_solver_variant_vs_oracle(tk, n):
    """Every compiled tile variant of P1, P3, P5 and of the solver's Y passes (the
    autotuner's choices) reproduces the oracle's right-hand side; the masked modes stay
    exactly zero."""
    import torch
    u = band_state(n, seed=n + 1)
    ref = ons.rhs(u)
    ud = to_gpu(u, "f32")
    try:
        for p in (3, 4, 5, 6):
            cands = tk.tile_candidates(n, torch.float32, p)
            assert cands, (n, p)
            for (a, E, v) in cands:
                tk.tune_set(n, torch.float32, p, a, E, v)
                s = tk.NS(n, dtype=torch.float32, nu=0.0)
                got = s.rhs(ud).cpu().numpy()
                s.close()
                assert diag.rel_l2(got, ref, n) <= 1e-5, (p, a, E)
                assert_shells(got, ref, n, 1e-4)
                assert np.max(np.abs(got * ~ons.dealias_mask(n))) == 0, (p, a, E)
            tk.tune_set(n, torch.float32, p, 0, 0)
    finally:
        tk.tune_clear()


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_taylor_green_32_ten_steps(tk, dt):
    """32^3 Taylor-Green, nu = 0.01, dt = 0.01, IF-RK2, 10 steps."""
    n = 32
    u0 = offt.rfft3(synth.taylor_green(n))
    ref, tref = ons.run(u0, 0.01, 0.01, 10)
    s = tk.NS(n, dtype=tdt(dt), nu=0.01)
    ud = to_gpu(u0, dt)
    t = s.step(ud, 0.01, 10)
    assert abs(t - tref) <= 1e-12
    err = diag.rel_l2(ud.cpu().numpy(), ref, n)
    assert err <= (1e-12 if dt == "f64" else 1e-4), err
    d = s.diagnostics(ud)
    assert abs(d["energy"] - diag.energy(ref)) <= (1e-13 if dt == "f64" else 1e-6)
    assert d["max_div"] <= (1e-13 if dt == "f64" else 1e-5)


@pytest.mark.parametrize("scheme", ["rk2", "rk4"])
@pytest.mark.parametrize("n,dt", [(24, "f64"), (48, "f32"), (96, "f32"), (128, "f32"), (64, "f64")])
def test_one_step_vs_oracle(tk, n, dt, scheme):
    u = band_state(n, seed=100 + n)
    nu, h = 2e-3, 0.004
    stepper = ons.ifrk2_step if scheme == "rk2" else ons.ifrk4_step
    res = stepper(u, nu, h)
    ref = res[0] if isinstance(res, tuple) else res
    s = tk.NS(n, dtype=tdt(dt), nu=nu, scheme=scheme)
    ud = to_gpu(u, dt)
    s.step(ud, h, 1)
    got = ud.cpu().numpy()
    err = diag.rel_l2(got, ref, n)
    assert err <= (1e-12 if dt == "f64" else 1e-4), err
    assert_shells(got, ref, n, 1e-11 if dt == "f64" else 1e-4)


@pytest.mark.parametrize("scheme", ["rk2", "rk4"])
def test_fused_stepper_every_variant_and_state_change(tk, scheme):
    """Inside a run of steps every P5 runs fused with the next right-hand side's P1 (the
    stage input never goes through memory).  Every compiled fused variant must reproduce
    the oracle over several steps, and a state changed between two calls must be picked
    up (each call transforms its state afresh before the first step)."""
    import torch
    n = 128
    u = rand_state(n, seed=7)
    nu, h = 2e-3, 0.004
    stepper = ons.ifrk2_step if scheme == "rk2" else ons.ifrk4_step

    def ref_steps(v, k):
        for _ in range(k):
            r = stepper(v, nu, h)
            v = r[0] if isinstance(r, tuple) else r
        return v

    ref = ref_steps(u, 2)
    ref2 = ref_steps(0.5 * ref, 1)
    cands = tk.tile_candidates(n, torch.float32, 7)
    assert cands
    try:
        for (a, E, v) in cands:
            tk.tune_set(n, torch.float32, 7, a, E, v)
            s = tk.NS(n, dtype=torch.float32, nu=nu, scheme=scheme)
            ud = to_gpu(u, "f32")
            s.step(ud, h, 2)
            assert diag.rel_l2(ud.cpu().numpy(), ref, n) <= 1e-4, (a, E, v)
            ud.mul_(0.5)
            s.step(ud, h, 1)
            assert diag.rel_l2(ud.cpu().numpy(), ref2, n) <= 1e-4, (a, E, v)
            s.close()
    finally:
        tk.tune_clear()


def test_cfl_step_vs_oracle(tk):
    n = 64
    u = rand_state(n, seed=1)
    s = tk.NS(n, dtype=tdt("f32"), nu=1e-3, cfl=0.5)
    ud = to_gpu(u, "f32")
    t = s.step(ud, 0.0, 1)
    h_ref = ons.cfl_dt(u, 0.5)
    assert abs(s.last_dt() - h_ref) <= 1e-5 * h_ref
    assert abs(t - s.last_dt()) <= 1e-15
    ref = ons.ifrk2_step(u, 1e-3, h_ref)[0]
    assert diag.rel_l2(ud.cpu().numpy(), ref, n) <= 1e-4


@pytest.mark.parametrize("n", [16, 48, 96])
def test_diagnostics_vs_oracle(tk, n):
    u = rand_state(n, seed=5)
    u[:, 3, 2, 1] += 0.01  # a little divergence
    s = tk.NS(n, dtype=tdt("f64"), nu=0.01)
    d = s.diagnostics(to_gpu(u, "f64"))
    assert abs(d["energy"] - diag.energy(u)) <= 1e-13 * diag.energy(u)
    assert abs(d["dissipation"] - diag.dissipation(u, 0.01)) <= 1e-13 * diag.dissipation(u, 0.01)
    assert abs(d["max_div"] - diag.max_divergence(u)) <= 1e-12
    assert np.max(np.abs(np.array(d["spectrum"]) - diag.spectrum(u))) <= 1e-13


@pytest.mark.parametrize("n,dt", [(32, "f64"), (64, "f32"), (96, "f32")])
def test_init_random_vs_oracle(tk, n, dt):
    import torch
    noise = synth.gaussian_field((3, n, n, n), 1)
    ref = oinit.random_solenoidal(noise)
    s = tk.NS(n, dtype=tdt(dt), nu=1e-3)
    nz = torch.from_numpy(noise.astype(np.float32 if dt == "f32" else np.float64)).cuda()
    got = s.init_random(nz).cpu().numpy()
    assert diag.rel_l2(got, ref, n) <= (1e-12 if dt == "f64" else 1e-5)


def test_single_mode_decay_exact(tk):
    n = 16
    x = synth.grid(n)
    u = np.zeros((3, n, n, n))
    u[0] = np.sin(2 * x)[None, None, :]
    uh = offt.rfft3(u)
    s = tk.NS(n, dtype=tdt("f64"), nu=0.05)
    ud = to_gpu(uh, "f64")
    s.step(ud, 0.1, 20)
    assert np.max(np.abs(ud.cpu().numpy() - uh * np.exp(-0.05 * 4 * 2.0))) <= 1e-15


def test_inviscid_energy_and_divergence(tk):
    n = 64
    u = rand_state(n, seed=9)
    s = tk.NS(n, dtype=tdt("f32"), nu=0.0)
    ud = to_gpu(u, "f32")
    N = s.rhs(ud).cpu().numpy().astype(np.complex128)
    w = offt.hermitian_weight(n)
    p = np.sum(w * np.real(np.conj(u) * N))
    assert abs(p) <= 1e-6 * np.sqrt(np.sum(w * np.abs(N) ** 2) * np.sum(w * np.abs(u) ** 2))
    e0 = s.diagnostics(ud)["energy"]
    s.step(ud, 0.002, 10)
    d = s.diagnostics(ud)
    assert abs(d["energy"] - e0) <= 1e-5
    assert d["max_div"] <= 1e-5


def test_rhs_512_vs_oracle(tk, band512):
    """512^3 FP32: the decaying-turbulence initial field against the oracle's, then one
    right-hand side of a band-filling field (every kept mode O(1)), globally and shell by
    shell up to the cutoff K = 170."""
    import torch
    n = 512
    noise = synth.gaussian_field((3, n, n, n), 1)
    s = tk.NS(n, dtype=torch.float32, nu=1e-3, cfl=0.5)
    ud = s.init_random(torch.from_numpy(noise).cuda())
    u = oinit.random_solenoidal(noise)
    del noise
    assert diag.rel_l2(ud.cpu().numpy(), u, n) <= 1e-5
    del u, ud
    got = s.rhs(to_gpu(band512, "f32")).cpu().numpy()
    ref = ons.rhs(band512)
    assert diag.rel_l2(got, ref, n) <= 1e-5
    assert_shells(got, ref, n, 1e-4)
    assert np.max(np.abs(got * ~ons.dealias_mask(n))) == 0


def test_pass_times_leave_the_state_alone(tk):
    """ns_pass_times times every solver pass (and the fused one) without writing the
    state; a step afterwards still matches the oracle (it transforms the state afresh)."""
    import torch
    n = 64
    u = rand_state(n, seed=21)
    s = tk.NS(n, dtype=torch.float32, nu=2e-3)
    ud = to_gpu(u, "f32")
    before = ud.clone()
    t = s.pass_times(ud, iters=3)
    assert set(t) == {"P1", "P2", "P3", "P4", "P5", "P5+P1"}
    assert all(v > 0 for v in t.values()), t
    assert torch.equal(ud, before)
    s.step(ud, 0.004, 1)
    ref = ons.ifrk2_step(u, 2e-3, 0.004)[0]
    assert diag.rel_l2(ud.cpu().numpy(), ref, n) <= 1e-4
    s.close()
