"""Pins for the oracle's energy transfer diagnostics (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import diag, fft, init, ns, transfer


def state(n, seed):
    return init.random_solenoidal(synth.gaussian_field((3, n, n, n), seed))


@pytest.mark.parametrize("n", [16, 24])
def test_transfer_conserves_energy(n):
    """The nonlinear term moves energy between shells without creating any: sum_s T(s) = 0,
    so the flux out of the largest sphere vanishes."""
    u = state(n, 3)
    T = transfer.shell_transfer(u)
    scale = np.max(np.abs(T))
    assert scale > 0
    assert abs(np.sum(T)) <= 1e-14 * max(1.0, scale) * len(T)
    assert abs(transfer.flux(T)[-1]) <= 1e-13 * max(1.0, scale) * len(T)


def test_shell_to_shell_antisymmetric_and_sums_to_shell_transfer():
    n = 16
    u = state(n, 4)
    nsh = diag.num_shells(n)
    bands = np.full(nsh, -1)
    edges = [0, 2, 3, 4, 6, 9, nsh]
    for b in range(len(edges) - 1):
        bands[edges[b]:edges[b + 1]] = b
    nb = len(edges) - 1
    Tnm = transfer.shell_to_shell(u, bands, nb)
    scale = np.max(np.abs(Tnm))
    assert scale > 0
    # giver / receiver antisymmetry
    assert np.max(np.abs(Tnm + Tnm.T)) <= 1e-13 * scale
    # what band n receives from all bands is its total transfer rate
    T = transfer.shell_transfer(u)
    Tb = np.array([np.sum(T[bands == b]) for b in range(nb)])
    assert np.max(np.abs(Tnm.sum(axis=1) - Tb)) <= 1e-13 * scale


def test_taylor_green_initial_transfer_vanishes():
    """At t = 0 the TG field has modes only at |k|^2 = 3 and its nonlinear term only at
    |k|^2 = 8: no shell exchanges energy yet."""
    n = 16
    u = fft.rfft3(synth.taylor_green(n))
    assert np.max(np.abs(transfer.shell_transfer(u))) <= 1e-17
