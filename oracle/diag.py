"""Diagnostics in FP64 (oracle; test infrastructure).

Sums over the stored half spectrum carry the weight w(kz) (1 on kz = 0 and N/2,
2 elsewhere), which makes them equal to full-spectrum sums for Hermitian fields.
Energy spectrum by shells, as used for the paper's spectrum plots (Section
"Scaling of RBC spectral solver", energy spectrum and flux).
"""
import numpy as np

from . import fft


def energy(uhat):
    """E = sum w 1/2 |u^|^2 = 1/2 <|u|^2> (Parseval)."""
    n = uhat.shape[-3]
    w = fft.hermitian_weight(n)
    return float(np.sum(w * 0.5 * np.abs(uhat) ** 2))


def enstrophy(uhat):
    """Omega = sum w 1/2 |k|^2 |u^|^2."""
    n = uhat.shape[-3]
    kx, ky, kz = fft.wavenumbers(n)
    k2 = kx * kx + ky * ky + kz * kz
    w = fft.hermitian_weight(n)
    return float(np.sum(w * 0.5 * k2 * np.abs(uhat) ** 2))


def dissipation(uhat, nu):
    """epsilon = 2 nu Omega."""
    return 2.0 * nu * enstrophy(uhat)


def shell_index(n):
    """Shell s of each stored mode: the integer with (2s-1)^2 <= 4|k|^2 < (2s+1)^2
    (nearest integer to |k|, decided exactly in integers)."""
    kx, ky, kz = fft.wavenumbers(n)
    k2 = (kx * kx + ky * ky + kz * kz).astype(np.int64)
    s = np.floor(np.sqrt(k2.astype(np.float64))).astype(np.int64)
    # exact integer correction: nearest integer s to sqrt(k2)
    s = np.where(4 * k2 >= (2 * s + 1) ** 2, s + 1, s)
    s = np.where((s > 0) & (4 * k2 < (2 * s - 1) ** 2), s - 1, s)
    return np.broadcast_to(s, (n, n, n // 2 + 1))


def num_shells(n):
    """Shells 0..S-1 cover every stored mode: S = floor(sqrt(3) n / 2) + 2."""
    return int(np.floor(np.sqrt(3.0) * n / 2.0)) + 2


def spectrum(uhat, nshell=None):
    """E(s) = sum_{k in shell s} w 1/2 |u^|^2."""
    n = uhat.shape[-3]
    if nshell is None:
        nshell = num_shells(n)
    s = shell_index(n)
    w = fft.hermitian_weight(n)
    e = np.broadcast_to(w * 0.5 * np.sum(np.abs(uhat) ** 2, axis=0), s.shape)
    out = np.zeros(nshell)
    keep = s < nshell
    np.add.at(out, s[keep], e[keep])
    return out


def max_divergence(uhat):
    """max_k |k . u^(k)| / |k|, relative to max_k |u^(k)| (k = 0 excluded from the
    numerator).  Relative to the largest mode rather than mode by mode, so that modes
    holding only round-off do not dominate."""
    n = uhat.shape[-3]
    kx, ky, kz = fft.wavenumbers(n)
    kd = np.abs(kx * uhat[0] + ky * uhat[1] + kz * uhat[2])
    kn = np.sqrt((kx * kx + ky * ky + kz * kz).astype(np.float64))
    num = np.where(kn > 0, kd / np.where(kn > 0, kn, 1.0), 0.0)
    umax = np.max(np.sqrt(np.sum(np.abs(uhat) ** 2, axis=0)))
    return float(np.max(num) / umax) if umax > 0 else 0.0


def parseval(f, F):
    """(sum f^2 / N^3, sum w |F|^2): equal for F = rfft3(f)."""
    n = f.shape[-3] * f.shape[-2] * f.shape[-1]
    w = fft.hermitian_weight(f.shape[-1])
    return float(np.sum(np.asarray(f, np.float64) ** 2) / n), float(np.sum(w * np.abs(F) ** 2))


def rel_l2(a, b, n=None):
    """Relative L2 error ||a - b|| / ||b||, Hermitian-weighted for half-spectrum arrays
    when n (the real length of the last axis) is given."""
    a = np.asarray(a)
    b = np.asarray(b)
    if n is not None:
        w = fft.hermitian_weight(n)
        num = np.sum(w * np.abs(a - b) ** 2)
        den = np.sum(w * np.abs(b) ** 2)
    else:
        num = np.sum(np.abs(a - b) ** 2)
        den = np.sum(np.abs(b) ** 2)
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))


def shell_rel_l2(a, b, n, shells):
    """Relative L2 error per shell, sqrt(sum_s w |a - b|^2 / sum_s w |b|^2), for each
    shell s in ``shells`` ([...][n][n][n/2+1] half-spectrum arrays, summed over the
    leading axes)."""
    a = np.asarray(a)
    b = np.asarray(b)
    s = shell_index(n)
    w = fft.hermitian_weight(n)
    lead = tuple(range(a.ndim - 3))
    num = np.broadcast_to(w * np.sum(np.abs(a - b) ** 2, axis=lead), s.shape)
    den = np.broadcast_to(w * np.sum(np.abs(b) ** 2, axis=lead), s.shape)
    sn = np.bincount(s.ravel(), weights=num.ravel())
    sd = np.bincount(s.ravel(), weights=den.ravel())
    return np.array([np.sqrt(sn[k] / sd[k]) if sd[k] > 0 else np.sqrt(sn[k]) for k in shells])
