"""Pins for the oracle's 3D transform (CPU only).

Each check ties the oracle to something other than itself: the transform's
definition evaluated as a brute-force triple sum, closed forms, invariants and an
independent library routine (numpy's pocketfft).
"""
import numpy as np
import pytest

from oracle import diag, fft


def brute_forward(f):
    """F(k) = N^-3 sum_x f(x) exp(-i k.x), written out as matrices of exponentials."""
    nx, ny, nz = f.shape
    ex = np.exp(-2j * np.pi * np.outer(np.arange(nx), np.arange(nx)) / nx)
    ey = np.exp(-2j * np.pi * np.outer(np.arange(ny), np.arange(ny)) / ny)
    ez = np.exp(-2j * np.pi * np.outer(np.arange(nz // 2 + 1), np.arange(nz)) / nz)
    out = np.zeros((nx, ny, nz // 2 + 1), complex)
    for kx in range(nx):
        for ky in range(ny):
            for kz in range(nz // 2 + 1):
                out[kx, ky, kz] = np.sum(f * ex[kx][:, None, None] * ey[ky][None, :, None] * ez[kz][None, None, :])
    return out / (nx * ny * nz)


def brute_inverse(F, nz):
    """f(x) = sum_{kz=0}^{nz/2} w(kz) Re[sum_{kx,ky} F(k) exp(+i k.x)], brute force."""
    nx, ny, nzh = F.shape
    f = np.zeros((nx, ny, nz))
    X = np.arange(nx)[:, None, None]
    Y = np.arange(ny)[None, :, None]
    Z = np.arange(nz)[None, None, :]
    for kx in range(nx):
        for ky in range(ny):
            for kz in range(nzh):
                w = 1.0 if kz in (0, nz // 2) else 2.0
                ph = np.exp(2j * np.pi * (kx * X / nx + ky * Y / ny + kz * Z / nz))
                f += w * np.real(F[kx, ky, kz] * ph)
    return f


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 9, 12, 16, 18, 25, 27, 32])
def test_fft1d_brute(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for sign in (-1, 1):
        ref = np.array([np.sum(x * np.exp(sign * 2j * np.pi * k * np.arange(n) / n)) for k in range(n)])
        got = fft.fft1d(x, sign)
        assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 6, 6), (8, 8, 8), (9, 12, 8), (4, 6, 12), (12, 9, 16), (16, 4, 6)])
def test_rfft3_brute(shape):
    f = np.random.default_rng(sum(shape)).standard_normal(shape)
    got = fft.rfft3(f)
    ref = brute_forward(f)
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-13


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 9, 8), (8, 6, 12)])
def test_irfft3_brute_nonhermitian(shape):
    """The inverse follows the w(kz) Re[...] definition even for non-Hermitian input
    (kz = 0 and nz/2 planes with arbitrary values)."""
    nx, ny, nz = shape
    rng = np.random.default_rng(7)
    F = rng.standard_normal((nx, ny, nz // 2 + 1)) + 1j * rng.standard_normal((nx, ny, nz // 2 + 1))
    got = fft.irfft3(F, nz)
    ref = brute_inverse(F, nz)
    assert np.max(np.abs(got - ref)) <= 1e-12


@pytest.mark.parametrize("n", [32, 64, 96, 128])
def test_rfft3_vs_numpy(n):
    f = np.random.default_rng(0).standard_normal((n, n, n), dtype=np.float32).astype(np.float64)
    got = fft.rfft3(f)
    ref = np.fft.rfftn(f) / n ** 3
    assert diag.rel_l2(got, ref, n) <= 1e-14
    back = fft.irfft3(got)
    assert np.max(np.abs(back - f)) <= 1e-12


@pytest.mark.parametrize("n", [12, 16, 24])
def test_single_mode_closed_form(n):
    """f = cos(k0.x + phi) has F = 1/2 e^{+i phi} at k0 and 1/2 e^{-i phi} at -k0."""
    k0 = (2, -3, 1)
    phi = 0.7
    x = 2 * np.pi * np.arange(n) / n
    f = np.cos(k0[0] * x[:, None, None] + k0[1] * x[None, :, None] + k0[2] * x[None, None, :] + phi)
    F = fft.rfft3(f)
    exp = np.zeros_like(F)
    exp[k0[0] % n, k0[1] % n, k0[2]] = 0.5 * np.exp(1j * phi)
    assert np.max(np.abs(F - exp)) <= 1e-14
    # kz = 0 mode with both +-k0 stored on the kz = 0 plane
    g = np.cos(3 * x[:, None, None] + 1 * x[None, :, None] + 0 * x[None, None, :] + phi)
    G = fft.rfft3(g)
    exp = np.zeros_like(G)
    exp[3, 1, 0] = 0.5 * np.exp(1j * phi)
    exp[-3 % n, -1 % n, 0] = 0.5 * np.exp(-1j * phi)
    assert np.max(np.abs(G - exp)) <= 1e-14


def test_delta_and_constant():
    n = 16
    f = np.zeros((n, n, n))
    f[0, 0, 0] = 1.0
    F = fft.rfft3(f)
    assert np.max(np.abs(F - 1.0 / n ** 3)) <= 1e-17
    g = fft.irfft3(F)
    assert np.max(np.abs(g - f)) <= 1e-14
    c = np.full((n, n, n), 2.5)
    C = fft.rfft3(c)
    assert abs(C[0, 0, 0] - 2.5) <= 1e-14
    C[0, 0, 0] = 0
    assert np.max(np.abs(C)) <= 1e-14


def test_shift_theorem_and_linearity():
    n = 12
    rng = np.random.default_rng(3)
    f = rng.standard_normal((n, n, n))
    g = rng.standard_normal((n, n, n))
    F, G = fft.rfft3(f), fft.rfft3(g)
    assert np.max(np.abs(fft.rfft3(2 * f - 3 * g) - (2 * F - 3 * G))) <= 1e-14
    s = (1, 2, 3)
    fs = np.roll(f, s, axis=(0, 1, 2))
    kx, ky, kz = fft.wavenumbers(n)
    phase = np.exp(-2j * np.pi * (kx * s[0] + ky * s[1] + kz * s[2]) / n)
    assert np.max(np.abs(fft.rfft3(fs) - F * phase)) <= 1e-13


def test_hermitian_planes_and_parseval():
    n = 16
    f = np.random.default_rng(5).standard_normal((n, n, n))
    F = fft.rfft3(f)
    for kz in (0, n // 2):
        P = F[:, :, kz]
        Pc = np.conj(P[(-np.arange(n)) % n][:, (-np.arange(n)) % n])
        assert np.max(np.abs(P - Pc)) <= 1e-15
    a, b = diag.parseval(f, F)
    assert abs(a - b) <= 1e-13 * a


def test_sampled_definitions_match_full_transform():
    """dft_at / idft_at evaluate the definitions directly; they agree with the full transform."""
    n = 24
    rng = np.random.default_rng(9)
    f = rng.standard_normal((n, 12, 16))
    F = fft.rfft3(f)
    ks = [(0, 0, 0), (3, 5, 2), (23, 11, 8), (12, 6, 7)]
    got = fft.dft_at(f, ks)
    assert np.max(np.abs(got - np.array([F[k] for k in ks]))) <= 1e-15
    xs = [(0, 0, 0), (5, 7, 3), (23, 11, 15)]
    assert np.max(np.abs(fft.idft_at(F, 16, xs) - np.array([f[x] for x in xs]))) <= 1e-13


def test_plane_and_line_evaluators_match_the_full_transform():
    """The large-grid evaluators (complete kz-planes; complete x-lines in a Fourier, sine
    or cosine x basis, forward and inverse) agree with the full 3D oracle transforms."""
    from oracle import fft as offt
    rng = np.random.default_rng(17)
    f = rng.standard_normal((24, 12, 16))
    F = offt.rfft3(f)
    P = offt.dft_planes(f, [0, 3, 8], chunk=5)
    for i, kz in enumerate([0, 3, 8]):
        assert np.max(np.abs(P[i] - F[:, :, kz])) <= 1e-15
    cols = [(0, 0), (5, 3), (11, 8)]
    pts = [(0, 0), (7, 13), (11, 15)]
    G = rng.standard_normal(F.shape) + 1j * rng.standard_normal(F.shape)
    for bx in (offt.FOURIER, offt.SINE, offt.COSINE):
        Fb = offt.rfft3_basis(f, bx, offt.FOURIER)
        L = offt.dft_x_lines_basis(f, bx, cols)
        for i, (b, c) in enumerate(cols):
            assert np.max(np.abs(L[i] - Fb[:, b, c])) <= 1e-15
        g = offt.irfft3_basis(G, 16, bx, offt.FOURIER)
        Li = offt.idft_x_lines_basis(G, 16, bx, pts)
        for i, (b, c) in enumerate(pts):
            assert np.max(np.abs(Li[i] - g[:, b, c])) <= 1e-14 * np.max(np.abs(g))
