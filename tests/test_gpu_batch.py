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
    # one member of each size class (64^3, 96^3, 128^3) against the oracle for one CFL step
    # from its state after the five steps
    picks = [0, 16, 32, 47]
    us = [states[i].cpu().numpy().astype(np.complex128) for i in picks]
    ens.step(states, 0.0, 1)
    dts = ens.last_dt()
    for i, u in zip(picks, us):
        n = sizes[i]
        h = ons.cfl_dt(u, 0.5)
        assert abs(dts[i] - h) <= 1e-5 * h, (i, n)
        ref = ons.ifrk2_step(u, nus[i], h)[0]
        assert diag.rel_l2(states[i].cpu().numpy(), ref, n) <= 1e-4, (i, n)


def test_every_ensemble_tile_matches(tk):
    """Every compiled ensemble shape (threads per workgroup x persistent grid, the
    autotuner's candidates, tile table pass 8) reproduces the standalone solver's steps and
    the oracle, for a mixed ensemble of every supported grid size."""
    import torch
    sizes = [128, 96, 64, 48, 32, 24, 16]
    nus = [1e-3 * (1 + i) for i in range(len(sizes))]
    u0 = [oinit.random_solenoidal(synth.gaussian_field((3, n, n, n), 300 + i)) for i, n in enumerate(sizes)]
    h, k = 0.002, 2
    refs = []
    for i, n in enumerate(sizes):
        r = u0[i]
        for _ in range(k):
            r = ons.ifrk2_step(r, nus[i], h)[0]
        refs.append(r)
    shapes = sorted({(a, v) for n in sizes for (a, E, v) in tk.tile_candidates(n, torch.float32, 8)})
    assert len(shapes) >= 10
    try:
        for (nt, gv) in shapes:
            for n in sizes:
                cands = tk.tile_candidates(n, torch.float32, 8)
                E = cands[0][1]
                if (nt, E, gv) in cands:
                    tk.tune_set(n, torch.float32, 8, nt, E, gv)
                else:  # this thread count is not compiled for n: the default shape
                    tk.tune_set(n, torch.float32, 8, 0, 0)
            ens = tk.Ensemble(sizes, nus)
            states = [torch.from_numpy(u.astype(np.complex64)).cuda() for u in u0]
            ens.step(states, h, k)
            for i, n in enumerate(sizes):
                assert diag.rel_l2(states[i].cpu().numpy(), refs[i], n) <= 1e-4, (nt, gv, n)
            ens.close()
    finally:
        tk.tune_clear()
