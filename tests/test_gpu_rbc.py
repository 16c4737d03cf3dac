"""Boussinesq convection (FFF basis) on the GPU against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import diag, fft as offt, init as oinit, ns as ons, rbc as orbc

pytestmark = pytest.mark.gpu


def fields(n, seed, amp_t=0.5):
    u = oinit.random_solenoidal(synth.gaussian_field((3, n, n, n), seed))
    t = offt.rfft3(synth.gaussian_field((n, n, n), seed + 1).astype(np.float64)) * ons.dealias_mask(n)
    t[0, 0, 0] = 0
    t *= amp_t / np.sqrt(diag.energy(np.stack([t, 0 * t, 0 * t])))
    return u, t


def gpu_state(u, t, dt):
    import torch
    s = np.concatenate([u, t[None]]).astype(np.complex64 if dt == "f32" else np.complex128)
    return torch.from_numpy(np.ascontiguousarray(s)).cuda()


def tdt(name):
    import torch
    return {"f32": torch.float32, "f64": torch.float64}[name]


@pytest.mark.parametrize("n,dt,box", [(16, "f64", 1.0), (32, "f32", 1.0), (48, "f32", 2 * np.pi), (24, "f64", 2.0)])
def test_rbc_rhs_vs_oracle(tk, n, dt, box):
    u, t = fields(n, n)
    a = 2 * np.pi / box
    Nu, Nt = orbc.rhs(u, t, a)
    ref = np.concatenate([Nu, Nt[None]])
    s = tk.RBC(n, Ra=1e6, Pr=1.0, box=box, dtype=tdt(dt))
    got = s.rhs(gpu_state(u, t, dt)).cpu().numpy()
    assert diag.rel_l2(got, ref, n) <= (1e-12 if dt == "f64" else 1e-5)


@pytest.mark.parametrize("n,dt", [(24, "f64"), (64, "f32")])
def test_rbc_step_vs_oracle(tk, n, dt):
    u, t = fields(n, 3 * n)
    Ra, Pr, box, h = 1e6, 1.0, 1.0, 2e-3
    nu, kappa = orbc.viscosities(Ra, Pr)
    uu, tt = orbc.ifrk2_step(u, t, nu, kappa, h, a=2 * np.pi / box)
    ref = np.concatenate([uu, tt[None]])
    s = tk.RBC(n, Ra=Ra, Pr=Pr, box=box, dtype=tdt(dt))
    st = gpu_state(u, t, dt)
    s.step(st, h, 1)
    assert diag.rel_l2(st.cpu().numpy(), ref, n) <= (1e-12 if dt == "f64" else 1e-4)
    d = s.diagnostics(st)
    w = offt.hermitian_weight(n)
    assert abs(d["kinetic"] - diag.energy(uu)) <= (1e-12 if dt == "f64" else 1e-6)
    assert abs(d["thermal"] - float(np.sum(w * 0.5 * np.abs(tt) ** 2))) <= (1e-12 if dt == "f64" else 1e-6)
    fl = float(np.sum(w * np.real(np.conj(uu[2]) * tt)))
    assert abs(d["uz_theta"] - fl) <= (1e-12 if dt == "f64" else 1e-6)
    assert abs(d["nusselt"] - (1 + np.sqrt(Ra * Pr) * d["uz_theta"])) <= 1e-9 * abs(d["nusselt"])


def test_rbc_cfl_steps_stay_solenoidal(tk):
    import torch
    n = 64
    u, t = fields(n, 5)
    s = tk.RBC(n, Ra=1e7, Pr=1.0, box=1.0, dtype=torch.float32, cfl=0.5)
    st = gpu_state(u, t, "f32")
    s.step(st, 0.0, 20)
    out = st.cpu().numpy().astype(np.complex128)
    assert diag.max_divergence(out[:3]) <= 1e-5
    assert np.max(np.abs(out * ~ons.dealias_mask(n))) == 0
    assert np.isfinite(s.diagnostics(st)["kinetic"])
