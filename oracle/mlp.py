"""Pointwise MLP sub-grid closure in FP64 (oracle; test infrastructure).

Network: x in R^9 (filtered velocity gradients, divided by a scalar in_scale) ->
64 (GELU) -> 64 (GELU) -> 6 (stress components xx, yy, zz, xy, xz, yz, in units of
out_scale).  GELU(x) = x/2 (1 + erf(x / sqrt 2)).  Parameters in one flat vector,
order W1[64][9], b1[64], W2[64][64], b2[64], W3[6][64], b3[6] (5190 values); the
GPU stores them as BF16, and the oracle evaluates the same BF16-rounded values in FP64.
Backward: plain reverse-mode differentiation; Adam: Kingma & Ba (2015).
"""
import numpy as np
from scipy.special import erf

SIZES = (9, 64, 64, 6)


def n_params(sizes=SIZES):
    return sum(b * a + b for a, b in zip(sizes[:-1], sizes[1:]))


def unpack(theta, sizes=SIZES):
    """Flat parameter vector -> lists of weights [out][in] and biases."""
    theta = np.asarray(theta, dtype=np.float64)
    Ws, bs, o = [], [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        Ws.append(theta[o:o + a * b].reshape(b, a))
        o += a * b
        bs.append(theta[o:o + b])
        o += b
    return Ws, bs


def pack(Ws, bs):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in zip(Ws, bs)])


def bf16_round(x):
    """Round FP32/FP64 values to the nearest BF16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x):
    """BF16 bit patterns (uint16) of the RNE-rounded values."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    return ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def forward(theta, x, cache=False):
    """x: [9][M] -> y: [6][M]."""
    Ws, bs = unpack(theta)
    a1 = Ws[0] @ x + bs[0][:, None]
    h1 = gelu(a1)
    a2 = Ws[1] @ h1 + bs[1][:, None]
    h2 = gelu(a2)
    y = Ws[2] @ h2 + bs[2][:, None]
    if cache:
        return y, (x, a1, h1, a2, h2)
    return y


def backward(theta, x, dy):
    """Gradient of sum(dy * y(x)) with respect to the flat parameters."""
    Ws, bs = unpack(theta)
    y, (x, a1, h1, a2, h2) = forward(theta, x, cache=True)
    gW3 = dy @ h2.T
    gb3 = dy.sum(axis=1)
    dh2 = Ws[2].T @ dy
    da2 = dh2 * gelu_grad(a2)
    gW2 = da2 @ h1.T
    gb2 = da2.sum(axis=1)
    dh1 = Ws[1].T @ da2
    da1 = dh1 * gelu_grad(a1)
    gW1 = da1 @ x.T
    gb1 = da1.sum(axis=1)
    return pack([gW1, gW2, gW3], [gb1, gb2, gb3])


def mse_loss(y, t):
    """L = mean over the 6 M values of (y - t)^2, and dL/dy."""
    d = y - t
    n = d.size
    return float(np.sum(d * d) / n), 2.0 * d / n


def adam(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
