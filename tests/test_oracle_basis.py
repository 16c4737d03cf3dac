"""Pins for the oracle's sine / cosine bases (CPU only): scipy's independent DCT-II / DST-II,
closed forms and round trips."""
import numpy as np
import pytest
import scipy.fft as sf

from oracle import fft


@pytest.mark.parametrize("n", [8, 12, 16])
def test_r2r_rows_match_scipy(n):
    rng = np.random.default_rng(n)
    g = rng.standard_normal(n)
    C = fft._r2r_matrix(n, fft.COSINE, False) @ g
    S = fft._r2r_matrix(n, fft.SINE, False) @ g
    # scipy: dct-II y_k = 2 sum x_j cos(pi k (2j+1) / 2N); dst-II y_k = 2 sum x_j sin(pi (k+1)(2j+1) / 2N)
    assert np.max(np.abs(C - sf.dct(g, type=2) / (2 * n))) <= 1e-15
    assert np.max(np.abs(S - sf.dst(g, type=2) / (2 * n))) <= 1e-15
    for b in (fft.SINE, fft.COSINE):
        Mi = fft._r2r_matrix(n, b, True)
        Mf = fft._r2r_matrix(n, b, False)
        assert np.max(np.abs(Mi @ Mf - np.eye(n))) <= 1e-13


@pytest.mark.parametrize("bx,by", [(1, 0), (2, 0), (0, 1), (1, 2), (2, 2)])
def test_basis_round_trip_and_fourier_limit(bx, by):
    rng = np.random.default_rng(3)
    f = rng.standard_normal((8, 12, 10))
    F = fft.rfft3_basis(f, bx, by)
    assert F.shape == (8, 12, 6)
    assert np.max(np.abs(fft.irfft3_basis(F, 10, bx, by) - f)) <= 1e-12
    assert np.max(np.abs(fft.rfft3_basis(f, 0, 0) - fft.rfft3(f))) == 0


def test_single_modes():
    """f = cos(3 x) cos(2 y') on the cosine/Fourier grid gives F = 1/2 at (kx=3, ky=+-2) ...
    and f = sin(2 x) gives the sine coefficient 1/2 at k = 2 (stored at index 1)."""
    nx, ny, nz = 8, 8, 4
    x = np.pi * (np.arange(nx) + 0.5) / nx
    y = 2 * np.pi * np.arange(ny) / ny
    f = np.cos(3 * x)[:, None, None] * np.cos(2 * y)[None, :, None] * np.ones(nz)
    F = fft.rfft3_basis(f, fft.COSINE, fft.FOURIER)
    exp = np.zeros_like(F)
    exp[3, 2, 0] = 0.25
    exp[3, ny - 2, 0] = 0.25
    assert np.max(np.abs(F - exp)) <= 1e-15
    g = np.sin(2 * x)[:, None, None] * np.ones((1, ny, nz))
    G = fft.rfft3_basis(g, fft.SINE, fft.FOURIER)
    exp = np.zeros_like(G)
    exp[1, 0, 0] = 0.5
    assert np.max(np.abs(G - exp)) <= 1e-15


@pytest.mark.parametrize("b", [(2, 2, 1), (1, 2, 2), (1, 1, 1), (2, 2, 2), (2, 1, 1)])
def test_sss_matches_scipy_and_round_trips(b):
    """SSS family (a sine or cosine basis on every axis): scipy's independent multi-axis
    DCT-II / DST-II (each axis its own type), the round trip, and a single mode: the
    u_z basis function 8 cos(kx x) cos(ky y) sin(kz z) of the paper's Section "Fast Fourier
    Transform" has the one coefficient 1 (sin 0 is the zero function, so a sine k starts
    at 1, stored at index k - 1)."""
    bx, by, bz = b
    rng = np.random.default_rng(sum(b))
    f = rng.standard_normal((8, 12, 10))
    F = fft.rfft3_sss(f, bx, by, bz)
    ref = f.copy()
    for ax, bb in zip(range(3), b):
        n = f.shape[ax]
        ref = (sf.dct(ref, type=2, axis=ax) if bb == fft.COSINE else sf.dst(ref, type=2, axis=ax)) / (2 * n)
    assert np.max(np.abs(F - ref)) <= 1e-15
    assert np.max(np.abs(fft.irfft3_sss(F, bx, by, bz) - f)) <= 1e-13
    nx, ny, nz = 8, 12, 10
    grid = [np.pi * (np.arange(n) + 0.5) / n for n in (nx, ny, nz)]
    kx, ky, kz = 3, 2, 4
    g = 8 * np.cos(kx * grid[0])[:, None, None] * np.cos(ky * grid[1])[None, :, None] * np.sin(kz * grid[2])[None, None, :]
    G = fft.rfft3_sss(g, fft.COSINE, fft.COSINE, fft.SINE)
    exp = np.zeros_like(G)
    exp[kx, ky, kz - 1] = 1.0
    assert np.max(np.abs(G - exp)) <= 1e-14
    with pytest.raises(ValueError):
        fft.rfft3_sss(f, fft.FOURIER, 1, 1)


def test_sss_line_evaluator_matches_full_transform():
    rng = np.random.default_rng(5)
    f = rng.standard_normal((8, 12, 10))
    for b in ((2, 2, 1), (1, 2, 2)):
        F = fft.rfft3_sss(f, *b)
        g = fft.irfft3_sss(F, *b)
        Lz = fft.sss_lines(f, *b, axis=2, pts=[(0, 0), (3, 7), (7, 11)])
        Lx = fft.sss_lines(f, *b, axis=0, pts=[(0, 0), (5, 9), (11, 3)])
        Iz = fft.sss_lines(F, *b, axis=2, pts=[(2, 4)], inverse=True)
        for i, (p, q) in enumerate([(0, 0), (3, 7), (7, 11)]):
            assert np.max(np.abs(Lz[i] - F[p, q, :])) <= 1e-15
        for i, (p, q) in enumerate([(0, 0), (5, 9), (11, 3)]):
            assert np.max(np.abs(Lx[i] - F[:, p, q])) <= 1e-15
        assert np.max(np.abs(Iz[0] - g[2, 4, :])) <= 1e-13
        assert np.max(np.abs(Iz[0] - f[2, 4, :])) <= 1e-13
