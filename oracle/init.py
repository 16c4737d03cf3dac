"""Initial fields (oracle; FP64; test infrastructure).

The random numbers come from the shared seeded generators (package ``synth``);
the spectral shaping below is the oracle's own.
"""
import numpy as np

from . import diag, fft, ns


def target_spectrum(s):
    """E_target(s) = s^4 exp(-2 (s/4)^2) (decaying-turbulence initial spectrum)."""
    s = np.asarray(s, dtype=np.float64)
    return s ** 4 * np.exp(-2.0 * (s / 4.0) ** 2)


def from_real(u):
    """Spectral state of a sampled real velocity field [3][N][N][N]."""
    return fft.rfft3(u)


def random_solenoidal(noise, energy=1.0):
    """Shape a real Gaussian noise field [3][N][N][N] into a random-phase solenoidal
    spectral velocity with E(s) proportional to E_target(s) and total energy ``energy``:
      1. r2c; 2. project to solenoidal; 3. zero k = 0 and the 2/3-masked modes;
      4. rescale each shell s >= 1 to E_target(s); 5. normalise the total energy."""
    n = noise.shape[-3]
    uhat = fft.rfft3(np.asarray(noise, dtype=np.float64))
    uhat = ns.project(uhat)
    uhat = uhat * ns.dealias_mask(n)
    uhat[:, 0, 0, 0] = 0.0
    nshell = diag.num_shells(n)
    es = diag.spectrum(uhat, nshell)
    s = diag.shell_index(n)
    factor = np.zeros(nshell)
    sidx = np.arange(nshell)
    ok = (sidx >= 1) & (es > 0)
    factor[ok] = np.sqrt(target_spectrum(sidx[ok]) / es[ok])
    uhat = uhat * factor[s][None]
    e = diag.energy(uhat)
    return uhat * np.sqrt(energy / e)


def band_filling(noise, energy=1.0):
    """A solenoidal spectral velocity whose every kept mode carries O(1) of the typical
    mode amplitude (flat per mode, E(s) growing as s^2 up to the 2/3 cutoff), for parity
    checks that must see the whole kept band:
      1. r2c of the noise; 2. projection; 3. 2/3 mask and k = 0 removed;
      4. total energy normalised to ``energy``."""
    n = noise.shape[-3]
    uhat = ns.project(fft.rfft3(np.asarray(noise, dtype=np.float64)))
    uhat = uhat * ns.dealias_mask(n)
    uhat[:, 0, 0, 0] = 0.0
    return uhat * np.sqrt(energy / diag.energy(uhat))
