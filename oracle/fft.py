"""3D real-to-complex / complex-to-real transforms in FP64 (oracle; test infrastructure).

Conventions follow the paper's Section "Fast Fourier Transform": the inverse
transform is the plain sum over the Fourier basis exp(+i k.x) with no 1/N, so the
1/N^3 sits on the forward transform.  Layout: real [nx][ny][nz], complex
[nx][ny][nz/2+1] (Appendix A's n0 x n1 x (n2/2+1)); wavenumbers on x and y are
0..N/2-1 followed by -N/2..-1, and kz = 0..N/2 is stored.

The transforms themselves are in ``fftref.c`` (own recursive mixed-radix FFT).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_rfft3.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_irfft3.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_fft1d.argtypes = [dp, ctypes.c_int, ctypes.c_int]
        L.orc_num_threads.argtypes = []
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def fft1d(x, sign=-1):
    """Unscaled 1D DFT of a complex vector: sum_j x_j exp(sign 2 pi i j k / n)."""
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    rc = lib().orc_fft1d(_dp(a.view(np.float64)), a.shape[0], int(sign))
    if rc != 0:
        raise ValueError("orc_fft1d failed")
    return a


def rfft3(f):
    """Forward transform F(k) = N^-3 sum_x f(x) exp(-i k.x) of a real [..., nx, ny, nz] array."""
    f = np.asarray(f)
    lead = f.shape[:-3]
    nx, ny, nz = f.shape[-3:]
    src = np.ascontiguousarray(f, dtype=np.float64).reshape((-1, nx, ny, nz))
    out = np.empty((src.shape[0], nx, ny, nz // 2 + 1), dtype=np.complex128)
    for b in range(src.shape[0]):
        s = np.ascontiguousarray(src[b])
        o = out[b]
        rc = lib().orc_rfft3(_dp(s), _dp(o.view(np.float64)), nx, ny, nz)
        if rc != 0:
            raise ValueError("orc_rfft3: unsupported shape %r" % (f.shape,))
    return out.reshape(lead + (nx, ny, nz // 2 + 1))


def irfft3(F, nz=None):
    """Inverse transform f(x) = sum_{kz} w(kz) Re[sum_{kx,ky} F(k) exp(i k.x)] (unscaled)."""
    F = np.asarray(F)
    lead = F.shape[:-3]
    nx, ny, nzh = F.shape[-3:]
    if nz is None:
        nz = 2 * (nzh - 1)
    src = np.ascontiguousarray(F, dtype=np.complex128).reshape((-1, nx, ny, nzh))
    out = np.empty((src.shape[0], nx, ny, nz), dtype=np.float64)
    for b in range(src.shape[0]):
        s = np.ascontiguousarray(src[b])
        o = out[b]
        rc = lib().orc_irfft3(_dp(s.view(np.float64)), _dp(o), nx, ny, nz)
        if rc != 0:
            raise ValueError("orc_irfft3: unsupported shape %r" % (F.shape,))
    return out.reshape(lead + (nx, ny, nz))


def wavenumbers(n):
    """Integer wavenumbers (kx, ky, kz) broadcastable to [n][n][n/2+1].

    x and y: i for i < n/2, else i - n (the Nyquist index n/2 maps to -n/2);
    z: 0..n/2.
    """
    k = np.arange(n)
    k = np.where(k < n // 2, k, k - n)
    kz = np.arange(n // 2 + 1)
    return k[:, None, None], k[None, :, None], kz[None, None, :]


def hermitian_weight(n):
    """w(kz): 1 on the kz = 0 and kz = n/2 planes, 2 elsewhere (each stored mode
    with 0 < kz < n/2 stands for itself and its conjugate)."""
    w = np.full(n // 2 + 1, 2.0)
    w[0] = 1.0
    w[n // 2] = 1.0
    return w[None, None, :]


def dft_at(f, ks):
    """The forward transform's definition evaluated at selected modes only:
    F(k) = N^-3 sum_x f(x) exp(-i k.x) for each (kx_idx, ky_idx, kz) in ks.  Cost O(N^3)
    per distinct kz plus O(N^2) per mode: used to check outputs of grids too large for
    the full oracle transform."""
    f = np.asarray(f)
    nx, ny, nz = f.shape
    ks = [tuple(int(v) for v in k) for k in ks]
    kzs = sorted(set(k[2] for k in ks))
    ez = np.exp(-2j * np.pi * np.outer(np.arange(nz), kzs) / nz)            # [nz][K]
    g = (f.reshape(nx * ny, nz).astype(np.float64) @ ez).reshape(nx, ny, len(kzs))
    out = []
    for (a, b, c) in ks:
        ex = np.exp(-2j * np.pi * a * np.arange(nx) / nx)
        ey = np.exp(-2j * np.pi * b * np.arange(ny) / ny)
        out.append(ex @ g[:, :, kzs.index(c)] @ ey)
    return np.array(out) / (nx * ny * nz)


def dft_planes(f, kzs, chunk=64):
    """The forward transform on complete kz-planes: F[:, :, kz] for each kz in kzs, from
    the definition along z (a direct sum over the nz samples) followed by the 1D
    transform of every y-line and then every x-line of each plane, with the 1/N^3
    factor.  Cost O(N^3) per plane: checks complete planes of grids too large for the
    full oracle transform."""
    f = np.asarray(f)
    nx, ny, nz = f.shape
    kzs = [int(k) for k in kzs]
    ez = np.exp(-2j * np.pi * np.outer(np.arange(nz), kzs) / nz)            # [nz][K]
    g = np.empty((nx, ny, len(kzs)), dtype=np.complex128)
    for a in range(0, nx, chunk):
        b = min(nx, a + chunk)
        g[a:b] = (f[a:b].reshape(-1, nz).astype(np.float64) @ ez).reshape(b - a, ny, len(kzs))
    out = np.empty((len(kzs), nx, ny), dtype=np.complex128)
    for i in range(len(kzs)):
        p = np.stack([fft1d(g[a, :, i], -1) for a in range(nx)])            # Y transform of each x row
        out[i] = np.stack([fft1d(p[:, b], -1) for b in range(ny)], axis=1)  # X transform of each column
    return out / (nx * ny * nz)


def idft_at(F, nz, xs):
    """The inverse transform's definition at selected grid points (ix, iy, iz):
    f(x) = sum_{kz} w(kz) Re[sum_{kx,ky} F(k) exp(i k.x)]."""
    F = np.asarray(F)
    nx, ny, nzh = F.shape
    w = np.full(nzh, 2.0)
    w[0] = 1.0
    w[nz // 2] = 1.0
    out = []
    for (a, b, c) in xs:
        ex = np.exp(2j * np.pi * a * np.arange(nx) / nx)
        ey = np.exp(2j * np.pi * b * np.arange(ny) / ny)
        ez = np.exp(2j * np.pi * c * np.arange(nzh) / nz)
        g = np.tensordot(ex, F, axes=(0, 0))          # [ny][nzh]
        g = ey @ g                                     # [nzh]
        out.append(np.sum(w * np.real(g * ez)))
    return np.array(out)


# ---- sine / cosine bases (free-slip walls) -------------------------------------------------------
# Paper, Section "Fast Fourier Transform": besides exp(iks) an axis may use the sine basis
# 2 sin(ks) or the cosine basis 2 cos(ks) (the SFF / SSF bases).  Readings: on such an axis
# the N grid points are x_j = pi (j + 1/2) / N (the half-period [0, pi]); the inverse is
#   cosine: f(x) = F_0 + sum_{k=1}^{N-1} 2 F_k cos(k x)
#   sine:   f(x) = sum_{k=1}^{N-1} 2 F_k sin(k x) + F_N sin(N x)
# and the forward transform, its inverse, is F_k = (1/N) sum_j f(x_j) cos(k x_j) (cosine,
# k = 0..N-1) or (1/N) sum_j f(x_j) sin(k x_j) (sine, k = 1..N, stored at index k-1).
FOURIER, SINE, COSINE = 0, 1, 2


def _r2r_matrix(n, basis, inverse):
    j = np.arange(n)
    x = np.pi * (j + 0.5) / n
    if basis == COSINE:
        k = np.arange(n)
        M = np.cos(np.outer(k, x))                    # [k][j]
        if inverse:
            c = np.full(n, 2.0)
            c[0] = 1.0
            return (M * c[:, None]).T                 # f_j = sum_k c_k F_k cos
        return M / n
    k = np.arange(1, n + 1)
    M = np.sin(np.outer(k, x))
    if inverse:
        c = np.full(n, 2.0)
        c[-1] = 1.0
        return (M * c[:, None]).T
    return M / n


def _apply_axis(a, M, axis):
    return np.moveaxis(np.tensordot(M, np.moveaxis(a, axis, 0), axes=(1, 0)), 0, axis)


def dft_x_lines_basis(f, bx, cols):
    """The forward transform with basis bx along x (Fourier along y and z) on complete
    x-lines: F[:, ky, kz] for each (ky index, kz) in cols, from direct sums over y and z
    (1/ny, 1/nz) followed by the x basis (fft1d / nx, or the sine / cosine sums)."""
    f = np.asarray(f)
    nx, ny, nz = f.shape
    out = []
    for (b, c) in cols:
        ez = np.exp(-2j * np.pi * c * np.arange(nz) / nz) / nz
        ey = np.exp(-2j * np.pi * b * np.arange(ny) / ny) / ny
        p = np.array([ey @ (f[a].astype(np.float64) @ ez) for a in range(nx)])   # [nx]
        out.append(fft1d(p, -1) / nx if bx == FOURIER else _r2r_matrix(nx, bx, False) @ p)
    return np.array(out)


def idft_x_lines_basis(F, nz, bx, points):
    """The inverse transform with basis bx along x (Fourier along y and z) on complete
    x-lines: f[:, iy, iz] for each (iy, iz) in points, f = sum_kz w(kz) Re[sum_ky
    e^{i ky y} e^{i kz z} (x basis sum over kx)]."""
    F = np.asarray(F)
    nx, ny, nzh = F.shape
    w = np.full(nzh, 2.0)
    w[0] = 1.0
    w[nz // 2] = 1.0
    out = []
    for (b, c) in points:
        ey = np.exp(2j * np.pi * b * np.arange(ny) / ny)
        ez = w * np.exp(2j * np.pi * c * np.arange(nzh) / nz)
        h = np.array([ey @ (F[a].astype(np.complex128) @ ez) for a in range(nx)])   # [nkx]
        if bx == FOURIER:
            out.append(np.real(fft1d(h, +1)))
        else:  # a real basis: the real part may be taken before the x sum
            out.append(_r2r_matrix(nx, bx, True) @ np.real(h))
    return np.array(out)


def rfft3_basis(f, bx=FOURIER, by=FOURIER):
    """Forward 3D transform with basis bx along x and by along y (Fourier along z):
    [nx][ny][nz] real -> [nx][ny][nz/2+1] complex, 1/N normalisation on every axis."""
    f = np.asarray(f, dtype=np.float64)
    nx, ny, nz = f.shape
    if bx == FOURIER and by == FOURIER:
        return rfft3(f)
    # z first, then y, then x, each axis by its own definition
    out = np.zeros((nx, ny, nz // 2 + 1), complex)
    for a in range(nx):
        for b in range(ny):
            line = fft1d(f[a, b].astype(np.complex128), -1)[: nz // 2 + 1] / nz
            out[a, b] = line
    if by == FOURIER:
        out = np.stack([np.stack([fft1d(out[a, :, c], -1) / ny for c in range(nz // 2 + 1)], axis=1)
                        for a in range(nx)])
    else:
        out = _apply_axis(out, _r2r_matrix(ny, by, False), 1)
    if bx == FOURIER:
        out = np.stack([np.stack([fft1d(out[:, b, c], -1) / nx for c in range(nz // 2 + 1)], axis=1)
                        for b in range(ny)], axis=1)
    else:
        out = _apply_axis(out, _r2r_matrix(nx, bx, False), 0)
    return out


def irfft3_basis(F, nz, bx=FOURIER, by=FOURIER):
    """Inverse of rfft3_basis (unscaled on Fourier axes, the basis sums on sine/cosine axes)."""
    F = np.asarray(F, dtype=np.complex128)
    nx, ny, nzh = F.shape
    g = F.copy()
    if bx == FOURIER:
        g = np.stack([np.stack([fft1d(g[:, b, c], +1) for c in range(nzh)], axis=1) for b in range(ny)], axis=1)
    else:
        g = _apply_axis(g, _r2r_matrix(nx, bx, True), 0)
    if by == FOURIER:
        g = np.stack([np.stack([fft1d(g[a, :, c], +1) for c in range(nzh)], axis=1) for a in range(nx)])
    else:
        g = _apply_axis(g, _r2r_matrix(ny, by, True), 1)
    out = np.empty((nx, ny, nz))
    for a in range(nx):
        for b in range(ny):
            line = np.zeros(nz, complex)
            line[0] = g[a, b, 0].real
            line[nz // 2] = g[a, b, nz // 2].real
            line[1:nz // 2] = g[a, b, 1:nz // 2]
            line[nz // 2 + 1:] = np.conj(g[a, b, 1:nz // 2][::-1])
            out[a, b] = fft1d(line, +1).real
    return out


def rfft3_sss(f, bx, by, bz):
    """Forward 3D transform with a sine or cosine basis on every axis (the paper's SSS
    family, e.g. cos x, cos y, sin z for u_z): real [nx][ny][nz] -> real coefficients
    [nx][ny][nz], each axis by its own definition (1/N per axis), z first, then y, then x."""
    if FOURIER in (bx, by, bz):
        raise ValueError("rfft3_sss: every axis needs the sine or cosine basis")
    f = np.asarray(f, dtype=np.float64)
    nx, ny, nz = f.shape
    out = _apply_axis(f, _r2r_matrix(nz, bz, False), 2)
    out = _apply_axis(out, _r2r_matrix(ny, by, False), 1)
    return _apply_axis(out, _r2r_matrix(nx, bx, False), 0)


def irfft3_sss(F, bx, by, bz):
    """Inverse of rfft3_sss: the basis sums along x, then y, then z."""
    if FOURIER in (bx, by, bz):
        raise ValueError("irfft3_sss: every axis needs the sine or cosine basis")
    F = np.asarray(F, dtype=np.float64)
    nx, ny, nz = F.shape
    g = _apply_axis(F, _r2r_matrix(nx, bx, True), 0)
    g = _apply_axis(g, _r2r_matrix(ny, by, True), 1)
    return _apply_axis(g, _r2r_matrix(nz, bz, True), 2)


def sss_lines(a, bx, by, bz, axis, pts, inverse=False):
    """Complete lines along `axis` (0 = x, 2 = z) of the SSS transform of a (forward) or
    of its inverse, at the points pts of the two other axes (index pairs, in axis order):
    the basis sums along those two axes at the given indices, then the whole line along
    `axis`.  Cost O(N^3) per line: checks grids too large for rfft3_sss."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape
    M = [_r2r_matrix(n[0], bx, inverse), _r2r_matrix(n[1], by, inverse), _r2r_matrix(n[2], bz, inverse)]
    out = []
    for (p, q) in pts:
        if axis == 2:
            line = M[1][q] @ (M[0][p] @ a.reshape(n[0], -1)).reshape(n[1], n[2])
            out.append(M[2] @ line)
        else:
            line = (a.reshape(-1, n[2]) @ M[2][q]).reshape(n[0], n[1]) @ M[1][p]
            out.append(M[0] @ line)
    return np.array(out)
