"""Energy transfer diagnostics on the GPU against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import diag, init as oinit, transfer as otr

pytestmark = pytest.mark.gpu


def tdt(name):
    import torch
    return {"f32": torch.float32, "f64": torch.float64}[name]


def to_gpu(a, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64 if dt == "f32" else np.complex128))).cuda()


@pytest.mark.parametrize("n,dt", [(16, "f64"), (32, "f32"), (64, "f32"), (48, "f64")])
def test_shell_transfer_vs_oracle(tk, n, dt):
    u = oinit.random_solenoidal(synth.gaussian_field((3, n, n, n), 21))
    ref = otr.shell_transfer(u)
    s = tk.NS(n, dtype=tdt(dt), nu=0.0)
    got = np.array(s.energy_transfer(to_gpu(u, dt)))
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= (1e-12 if dt == "f64" else 1e-5) * scale
    assert abs(np.sum(got)) <= (1e-12 if dt == "f64" else 1e-5) * scale * len(got)


@pytest.mark.parametrize("n,dt", [(16, "f64"), (24, "f32")])
def test_shell_to_shell_vs_oracle(tk, n, dt):
    u = oinit.random_solenoidal(synth.gaussian_field((3, n, n, n), 22))
    nsh = diag.num_shells(n)
    bands = np.full(nsh, -1)
    edges = [1, 2, 3, 4, 6, 9, nsh]
    for b in range(len(edges) - 1):
        bands[edges[b]:edges[b + 1]] = b
    nb = len(edges) - 1
    ref = otr.shell_to_shell(u, bands, nb)
    s = tk.NS(n, dtype=tdt(dt), nu=0.0)
    got = np.array(s.shell_to_shell(to_gpu(u, dt), bands, nb))
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= (1e-11 if dt == "f64" else 1e-4) * scale
    assert np.max(np.abs(got + got.T)) <= (1e-11 if dt == "f64" else 1e-4) * scale
