"""Filtered DNS, sub-grid stress and the LES right-hand side in FP64 (oracle; test
infrastructure).

Readings (stated in the design notes): the filter G is the sharp spectral box
|k_i| <= kc, applied by truncating the DNS spectrum onto the coarse grid (kc = (n-1)/3,
the coarse grid's 2/3 set, so the filtered field is exactly representable there);
tau_ij = G(u_i u_j) - G(ubar_i ubar_j): the stress the dealiased LES lacks, since its
own nonlinear term is exactly G(ubar_i ubar_j).  The first product is formed on the
DNS grid; the second on the coarse grid, where the 2/3 rule makes its kept modes exact.
Features are the nine filtered gradients d_j ubar_i on the coarse grid.  The LES right-hand side adds -i k_j tau^_ij to the
nonlinear term before masking and projection.
"""
import numpy as np

from . import fft, mlp, ns

# stress component order: xx, yy, zz, xy, xz, yz
PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def truncate(Fh, n_to, kc):
    """Copy the modes |kx|, |ky|, kz <= kc of a half spectrum (any grid) onto an
    n_to grid half spectrum, zero elsewhere."""
    n_from = Fh.shape[-3]
    lead = Fh.shape[:-3]
    out = np.zeros(lead + (n_to, n_to, n_to // 2 + 1), dtype=np.complex128)
    ks = np.arange(-kc, kc + 1)
    src = ks % n_from
    dst = ks % n_to
    out[..., dst[:, None], dst[None, :], : kc + 1] = Fh[..., src[:, None], src[None, :], : kc + 1]
    return out


def filtered_velocity(uhat_dns, n_les, kc):
    return truncate(uhat_dns, n_les, kc)


def gradients(ubar_hat):
    """g[3 i + j] = d_j ubar_i on the coarse grid, [9][n][n][n]."""
    n = ubar_hat.shape[-3]
    kx, ky, kz = ns.deriv_wavenumbers(n)
    k = (kx, ky, kz)
    out = []
    for i in range(3):
        for j in range(3):
            out.append(fft.irfft3(1j * k[j] * ubar_hat[i]))
    return np.stack(out)


def sgs_stress(uhat_dns, n_les, kc):
    """tau_ij = G(u_i u_j) - G(ubar_i ubar_j), [6][n][n][n] on the coarse grid."""
    u = fft.irfft3(uhat_dns)
    ubar = fft.irfft3(filtered_velocity(uhat_dns, n_les, kc))
    out = []
    for (i, j) in PAIRS:
        G = truncate(fft.rfft3(u[i] * u[j]), n_les, kc)
        Gb = truncate(fft.rfft3(ubar[i] * ubar[j]), n_les, kc)
        out.append(fft.irfft3(G - Gb))
    return np.stack(out)


def closure_tau(theta, ubar_hat, in_scale, out_scale):
    """Stress the network predicts from the filtered state: the nine gradient features
    are divided by in_scale, and the six network outputs multiplied by out_scale."""
    g = gradients(ubar_hat)
    n = g.shape[-1]
    y = mlp.forward(theta, g.reshape(9, -1) / in_scale)
    return (out_scale * y).reshape(6, n, n, n)


def sgs_divergence(tau):
    """-i k_j tau^_ij for the symmetric stress given by its 6 components."""
    n = tau.shape[-1]
    th = fft.rfft3(tau)
    T = [[th[0], th[3], th[4]], [th[3], th[1], th[5]], [th[4], th[5], th[2]]]
    kx, ky, kz = ns.deriv_wavenumbers(n)
    k = (kx, ky, kz)
    return np.stack([-1j * (k[0] * T[i][0] + k[1] * T[i][1] + k[2] * T[i][2]) for i in range(3)])


def les_rhs_tau(ubar_hat, tau):
    """N_LES = P M [F(u x omega) - i k_j tau^_ij] for a given real-space stress tau
    [6][n][n][n] (None: no model term).  The filtered momentum equation: the resolved
    nonlinear term of eq:NSk plus the divergence of the sub-grid stress, which enters
    with the same sign as the resolved flux -i k_j (u_i u_j)^."""
    n = ubar_hat.shape[-3]
    what = ns.curl(ubar_hat)
    u = fft.irfft3(ubar_hat)
    w = fft.irfft3(what)
    c = np.stack([u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]])
    chat = fft.rfft3(c)
    if tau is not None:
        chat = chat + sgs_divergence(tau)
    return ns.project(chat * ns.dealias_mask(n))


def les_rhs(ubar_hat, theta, in_scale, out_scale):
    """LES right-hand side with the network's stress (theta None: plain right-hand side)."""
    tau = None if theta is None else closure_tau(theta, ubar_hat, in_scale, out_scale)
    return les_rhs_tau(ubar_hat, tau)
