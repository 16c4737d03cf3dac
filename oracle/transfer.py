"""Energy transfer diagnostics in FP64 (oracle; test infrastructure).

The paper lists energy flux and shell-to-shell transfers among the solver's functions
(Section "Parallelization Strategy", closing paragraph; Section "Scaling of RBC spectral
solver" for the flux).  Definitions (the standard giver / receiver formulation of
shell-to-shell transfer, mediated by the full velocity):

  T(s)       = sum_{k in shell s} w Re[ u^*(k) . N(k) ]         (N = the nonlinear term)
  Pi(s0)     = - sum_{s <= s0} T(s)                              (flux out of the sphere)
  T_nm       = - sum_{k in band n} w Re[ u^*(k) . F[(u . grad) u^(m)](k) ]
               with u^(m) the velocity restricted to band m (energy band m gives to band n).

Bands are unions of integer shells (band_of_shell[s] = band index, -1 to exclude).  The
product is dealiased by the 2/3 mask (the input fields are 2/3-masked).
"""
import numpy as np

from . import diag, fft, ns


def shell_transfer(uhat):
    """T(s) for every integer shell."""
    N = ns.rhs(uhat)
    n = uhat.shape[-3]
    w = fft.hermitian_weight(n)
    t = np.broadcast_to(w * np.sum(np.real(np.conj(uhat) * N), axis=0), (n, n, n // 2 + 1))
    s = diag.shell_index(n)
    out = np.zeros(diag.num_shells(n))
    np.add.at(out, s.ravel(), t.ravel())
    return out


def flux(T):
    return -np.cumsum(T)


def band_index(n, band_of_shell):
    s = diag.shell_index(n)
    b = np.asarray(band_of_shell)[s]
    return b


def shell_to_shell(uhat, band_of_shell, nbands):
    """T[n][m] for bands 0..nbands-1."""
    n = uhat.shape[-3]
    kx, ky, kz = ns.deriv_wavenumbers(n)
    k = (kx, ky, kz)
    b = band_index(n, band_of_shell)
    u = fft.irfft3(uhat)
    w = fft.hermitian_weight(n)
    mask = ns.dealias_mask(n)
    out = np.zeros((nbands, nbands))
    for m in range(nbands):
        um = uhat * (b == m)
        adv = []
        for j in range(3):
            acc = 0
            for l in range(3):
                acc = acc + u[l] * fft.irfft3(1j * k[l] * um[j])
            adv.append(acc)
        A = fft.rfft3(np.stack(adv)) * mask
        e = np.broadcast_to(-w * np.sum(np.real(np.conj(uhat) * A), axis=0), b.shape)
        for nn in range(nbands):
            out[nn, m] = float(np.sum(e[b == nn]))
    return out
