"""Seeded synthetic inputs shared by the GPU library's tests/benchmarks and the oracle.

Holds only random-number draws and sampled analytic initial conditions: none of
the method's arithmetic (no transforms, projections or spectra) lives here.
"""
import numpy as np


def grid(n):
    """Grid points x_j = 2 pi j / n, j = 0..n-1, of the periodic (2 pi) box."""
    return 2.0 * np.pi * np.arange(n) / n


def gaussian_field(shape, seed, dtype=np.float32):
    """i.i.d. N(0,1) values from numpy's default_rng(seed)."""
    return np.random.default_rng(seed).standard_normal(shape, dtype=dtype)


def taylor_green(n, dtype=np.float64):
    """Taylor-Green velocity u = (sin x cos y cos z, -cos x sin y cos z, 0) sampled on
    the n^3 grid; shape [3][n][n][n]."""
    x = grid(n)
    X = x[:, None, None]
    Y = x[None, :, None]
    Z = x[None, None, :]
    u = np.empty((3, n, n, n), dtype=np.float64)
    u[0] = np.sin(X) * np.cos(Y) * np.cos(Z)
    u[1] = -np.cos(X) * np.sin(Y) * np.cos(Z)
    u[2] = 0.0
    return u.astype(dtype)


def ensemble_viscosities(count=48, seed=2, lo=5e-4, hi=5e-3):
    """Per-member viscosities, uniform in [lo, hi) from default_rng(seed)."""
    return np.random.default_rng(seed).uniform(lo, hi, count)


def ensemble_sizes():
    """Grid sizes of the 48-member ensemble: 16 x 64^3, 16 x 96^3, 16 x 128^3."""
    return [64] * 16 + [96] * 16 + [128] * 16


def ensemble_seed(i):
    return 100 + i


def mlp_init(sizes=(9, 64, 64, 6), seed=7):
    """He-style normal weights and zero biases for a pointwise MLP, FP64 lists."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for a, b in zip(sizes[:-1], sizes[1:]):
        Ws.append(rng.standard_normal((b, a)) * np.sqrt(2.0 / a))
        bs.append(np.zeros(b))
    return Ws, bs
