"""Ensembles of mixed grid sizes (persistent kernels, one HIP graph per step) against the
single solver and the FP64 oracle (GPU)."""
import numpy as np
import pytest

import synth
from oracle import diag, init as oinit, ns as ons

pytestmark = pytest.mark.gpu


def test_members_match_standalone_and_oracle(tk):
    import torch
    sizes = [16, 24, 32, 48, 64, 96, 128, 24, 16]
    nus = [2e-3 * (1 + i) for i in range(len(sizes))]
    ens = tk.Ensemble(sizes, nus)
    states, refs = [], []
    for i, n in enumerate(sizes):
        u0 = oinit.random_solenoidal(synth.gaussian_field((3, n, n, n), 200 + i))
        states.append(torch.from_numpy(u0.astype(np.complex64)).cuda())
        refs.append(u0)
    singles = [s.clone() for s in states]
    h, k = 0.003, 3
    t = ens.step(states, h, k)
    assert all(abs(v - k * h) < 1e-12 for v in t)
    for i, n in enumerate(sizes):
        s = tk.NS(n, dtype=torch.float32, nu=nus[i])
        s.step(singles[i], h, k)
        a = states[i].cpu().numpy()
        b = singles[i].cpu().numpy()
        assert diag.rel_l2(a, b, n) <= 1e-6, (i, n)
        ref = refs[i]
        for _ in range(k):
            ref = ons.ifrk2_step(ref, nus[i], h)[0]
        assert diag.rel_l2(a, ref, n) <= 1e-4, (i, n)


def test_ensemble_48_cfl(tk):
    """The 48-member configuration: 16 x 64^3, 16 x 96^3, 16 x 128^3, viscosities uniform in
    [5e-4, 5e-3], random solenoidal fields (seeds 100 + i), CFL 0.5."""
    import torch
    sizes = synth.ensemble_sizes()
    nus = synth.ensemble_viscosities()
    ens = tk.Ensemble(sizes, nus, cfl=0.5)
    states = []
    for i, n in enumerate(sizes):
        noise = torch.from_numpy(synth.gaussian_field((3, n, n, n), synth.ensemble_seed(i))).cuda()
        states.append(ens.init_random(i, noise))
    e0 = [ens.diagnostics(i, u)["energy"] for i, u in enumerate(states)]
    assert max(abs(e - 1.0) for e in e0) <= 1e-5
    ens.step(states, 0.0, 5)
    dts = ens.last_dt()
    for i, u in enumerate(states):
        d = ens.diagnostics(i, u)
        assert np.isfinite(d["energy"]) and d["energy"] < e0[i]
        assert d["max_div"] <= 1e-5
        assert 0 < dts[i] < 1.0
    # member 0 against the oracle for one CFL step from its state
    n0 = sizes[0]
    u = states[0].cpu().numpy().astype(np.complex128)
    h = ons.cfl_dt(u, 0.5)
    ref = ons.ifrk2_step(u, nus[0], h)[0]
    ens.step(states, 0.0, 1)
    assert diag.rel_l2(states[0].cpu().numpy(), ref, n0) <= 1e-4
