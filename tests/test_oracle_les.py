"""Pins for the oracle's closure network and LES operators (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import diag, fft, init, les, mlp, ns


def rand_theta(seed=0, scale=1.0):
    Ws, bs = synth.mlp_init(seed=seed)
    rng = np.random.default_rng(seed + 1)
    bs = [rng.standard_normal(b.shape) * 0.1 for b in bs]
    return mlp.bf16_round(mlp.pack([W * scale for W in Ws], bs))


def test_param_count_and_layout():
    assert mlp.n_params() == 5190
    th = np.arange(5190, dtype=float)
    Ws, bs = mlp.unpack(th)
    assert Ws[0].shape == (64, 9) and Ws[1].shape == (64, 64) and Ws[2].shape == (6, 64)
    assert np.array_equal(mlp.pack(Ws, bs), th)
    assert Ws[0][1, 0] == 9 and bs[0][0] == 576 and Ws[1][0, 0] == 640 and bs[2][5] == 5189


def test_gelu_closed_form():
    # GELU(0) = 0, GELU(x) -> x for large x, GELU(-x) = GELU(x) - x; Phi(1) = 0.841344746...
    assert mlp.gelu(0.0) == 0.0
    assert abs(mlp.gelu(1.0) - 0.8413447460685429) <= 1e-15
    x = np.linspace(-4, 4, 17)
    assert np.max(np.abs(mlp.gelu(-x) - (mlp.gelu(x) - x))) <= 1e-15
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) <= 1e-9


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 3.0e-3])
    r = mlp.bf16_round(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7 -> even (1); 1 + 3 2^-8 -> 1 + 2^-6 (even)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7 and r[3] == 1.0 + 2 ** -6
    assert r[4] == -2.5
    assert abs(r[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8
    assert np.all(mlp.bf16_bits(vals).view(np.uint16) == mlp.bf16_bits(r))


def test_backward_matches_finite_differences():
    th = rand_theta(3)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((9, 40))
    dy = rng.standard_normal((6, 40))
    g = mlp.backward(th, x, dy)

    def L(t):
        return float(np.sum(dy * mlp.forward(t, x)))

    idx = rng.choice(5190, 60, replace=False)
    idx = np.concatenate([idx, [0, 575, 576, 639, 640, 4735, 4736, 4799, 4800, 5183, 5184, 5189]])
    h = 1e-5
    for i in idx:
        e = np.zeros(5190)
        e[i] = h
        fd = (L(th + e) - L(th - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_mse_and_adam_first_step():
    y = np.array([[1.0, 2.0], [3.0, 5.0]])
    t = np.array([[0.0, 2.0], [3.0, 4.0]])
    Lv, dy = mlp.mse_loss(y, t)
    assert Lv == 0.5 and np.array_equal(dy, np.array([[0.5, 0.0], [0.0, 0.5]]))
    # the first Adam step moves each weight by lr * g / (|g| + eps)
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    th1, m, v = mlp.adam(th, np.zeros(3), np.zeros(3), g, 1, 1e-2)
    assert np.allclose(th1, th - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def band_limited_state(n, kmax, seed):
    uh = init.random_solenoidal(synth.gaussian_field((3, n, n, n), seed))
    kx, ky, kz = fft.wavenumbers(n)
    keep = (np.abs(kx) <= kmax) & (np.abs(ky) <= kmax) & (kz <= kmax)
    return uh * keep


def test_filter_truncation_and_band_limited_stress_vanishes():
    """A DNS field with |k_i| <= 10 passes the kc = 21 box unchanged, and since every
    product then lives in |k_i| <= 20 < 32 the sub-grid stress is exactly zero."""
    n_dns, n_les, kc = 96, 64, 21
    uh = band_limited_state(n_dns, 10, seed=2)
    ub = les.filtered_velocity(uh, n_les, kc)
    assert abs(diag.energy(ub) - diag.energy(uh)) <= 1e-14
    assert np.max(np.abs(les.sgs_stress(uh, n_les, kc))) <= 1e-13
    # truncation round trip (coarse -> fine -> coarse) is the identity on kept modes
    back = les.truncate(les.truncate(ub, n_dns, kc), n_les, kc)
    assert np.max(np.abs(back - ub)) == 0


def test_stress_of_single_high_mode():
    """u = (cos 25 z, 0, 0) has no resolved part for kc = 21, and u_x^2 = (1 + cos 50 z)/2,
    so tau_xx = 1/2 and every other component is 0."""
    n_dns, n_les, kc = 96, 64, 21
    z = synth.grid(n_dns)
    u = np.zeros((3, n_dns, n_dns, n_dns))
    u[0] = np.cos(25 * z)[None, None, :]
    tau = les.sgs_stress(fft.rfft3(u), n_les, kc)
    assert np.max(np.abs(tau[0] - 0.5)) <= 1e-13
    assert np.max(np.abs(tau[1:])) <= 1e-13


def test_stress_filters_the_resolved_product():
    """tau = G(u u) - G(ubar ubar): for a DNS field that is already filtered (|k_i| <= 21)
    the stress vanishes even though ubar_i ubar_j itself has modes up to 42 (pointwise
    products on the coarse grid are not subtracted unfiltered); the resolved product
    G(ubar ubar) formed on the 64 grid equals the one formed on the finer DNS grid."""
    n_dns, n_les, kc = 96, 64, 21
    uh = band_limited_state(n_dns, 21, seed=6)
    assert np.max(np.abs(les.sgs_stress(uh, n_les, kc))) <= 1e-13
    ub = les.filtered_velocity(uh, n_les, kc)
    u64 = fft.irfft3(ub)
    u96 = fft.irfft3(uh)
    a = les.truncate(fft.rfft3(u64[0] * u64[1]), n_les, kc)
    b = les.truncate(fft.rfft3(u96[0] * u96[1]), n_les, kc)
    assert np.max(np.abs(a - b)) <= 1e-15


def test_gradient_features_taylor_green():
    n = 32
    uh = fft.rfft3(synth.taylor_green(n))
    g = les.gradients(uh)
    x = synth.grid(n)
    X, Y, Z = x[:, None, None], x[None, :, None], x[None, None, :]
    # d_x u_x = cos x cos y cos z ; d_y u_x = -sin x sin y cos z ; d_z u_y = cos x sin y sin z
    assert np.max(np.abs(g[0] - np.cos(X) * np.cos(Y) * np.cos(Z))) <= 1e-14
    assert np.max(np.abs(g[1] + np.sin(X) * np.sin(Y) * np.cos(Z))) <= 1e-14
    assert np.max(np.abs(g[5] - np.cos(X) * np.sin(Y) * np.sin(Z))) <= 1e-14
    assert np.max(np.abs(g[6:])) <= 1e-14
    # trace = divergence = 0
    assert np.max(np.abs(g[0] + g[4] + g[8])) <= 1e-14


def test_sgs_divergence_of_uniform_and_linear_stress():
    """A constant stress has no divergence; tau_xz = sin z gives -d_z tau_xz = -cos z on x."""
    n = 16
    z = synth.grid(n)
    tau = np.zeros((6, n, n, n))
    tau[0] = 3.0
    assert np.max(np.abs(les.sgs_divergence(tau))) <= 1e-15
    tau[4] = np.sin(z)[None, None, :]
    d = fft.irfft3(les.sgs_divergence(tau))
    assert np.max(np.abs(d[0] + np.cos(z)[None, None, :])) <= 1e-14
    assert np.max(np.abs(d[2])) <= 1e-14  # d_x tau_xz = 0


def test_les_rhs_without_model_is_plain_rhs():
    n = 16
    uh = init.random_solenoidal(synth.gaussian_field((3, n, n, n), 8))
    assert np.max(np.abs(les.les_rhs(uh, None, 1.0, 1.0) - ns.rhs(uh))) == 0
    th = rand_theta(1, scale=0.0)  # zero weights, zero-ish biases -> constant stress -> no divergence
    th[:] = 0
    assert np.max(np.abs(les.les_rhs(uh, th, 1.0, 1.0) - ns.rhs(uh))) <= 1e-18


def band_filling_state(n, seed):
    return init.band_filling(synth.gaussian_field((3, n, n, n), seed))


@pytest.mark.parametrize("n_dns,n_les,kc", [(48, 24, 7), (96, 64, 21)])
def test_les_rhs_with_true_stress_is_truncated_dns_rhs(n_dns, n_les, kc):
    """Filtered-DNS identity (the sharp box G is the coarse grid's 2/3 set, and both
    grids are alias-free after their masks): the LES right-hand side of ubar = G u with
    the exact stress tau = G(u_i u_j) - G(ubar_i ubar_j) is the DNS right-hand side
    truncated to |k_i| <= kc, to round-off.  A flipped sign of the stress term, or the
    stress taken unfiltered, breaks it."""
    uh = band_filling_state(n_dns, seed=n_dns + 3)
    ref = les.truncate(ns.rhs(uh), n_les, kc)
    ub = les.filtered_velocity(uh, n_les, kc)
    tau = les.sgs_stress(uh, n_les, kc)
    got = les.les_rhs_tau(ub, tau)
    assert diag.rel_l2(got, ref, n_les) <= 1e-13
    # the model term matters: without it (or with its sign flipped) the identity fails
    assert diag.rel_l2(les.les_rhs_tau(ub, None), ref, n_les) >= 0.05
    assert diag.rel_l2(les.les_rhs_tau(ub, -tau), ref, n_les) >= 0.1
    # les_rhs with a network routes through the same expression
    th = rand_theta(2)
    t_net = les.closure_tau(th, ub, 3.0, 0.5)
    assert np.array_equal(les.les_rhs(ub, th, 3.0, 0.5), les.les_rhs_tau(ub, t_net))


def eddy_viscosity_theta(c=1.0):
    """Network weights whose output is exactly linear in the inputs for |x| << 1000:
    layer 1 copies the 9 inputs shifted by +1000 (GELU is the identity there in FP64),
    layer 2 is the identity, layer 3 forms y_ij = -c (x_ij + x_ji) and removes the shift
    (every weight is a BF16 value).  With x = grad ubar / in_scale and tau = out_scale y
    this is the eddy-viscosity stress tau = -2 nu_t S, nu_t = c out_scale / in_scale."""
    W1 = np.zeros((64, 9))
    W1[np.arange(9), np.arange(9)] = 1.0
    b1 = np.zeros(64)
    b1[:9] = 1000.0
    W2 = np.eye(64)
    b2 = np.zeros(64)
    W3 = np.zeros((6, 64))
    # feature 3 i + j is d_j ubar_i; outputs xx, yy, zz, xy, xz, yz
    for o, (i, j) in enumerate(les.PAIRS):
        W3[o, 3 * i + j] -= c
        W3[o, 3 * j + i] -= c
    b3 = -1000.0 * W3.sum(axis=1)
    th = mlp.pack([W1, W2, W3], [b1, b2, b3])
    assert np.array_equal(mlp.bf16_round(th), th)
    return th


def test_closure_eddy_viscosity_closed_form():
    """With the eddy-viscosity network, -i k_j tau^_ij = -nu_t |k|^2 u^ for a solenoidal
    field, so the LES right-hand side is the plain one minus nu_t |k|^2 u^: this fixes the
    sign of the model term, where in_scale and out_scale apply (nu_t = out/in, not in/out),
    and the order of the network's input and output components."""
    n = 24
    ub = band_filling_state(n, seed=11)
    in_scale, out_scale = 4.0, 0.5
    nu_t = out_scale / in_scale
    th = eddy_viscosity_theta()
    tau = les.closure_tau(th, ub, in_scale, out_scale)
    S = les.gradients(ub).reshape(3, 3, n, n, n)
    for o, (i, j) in enumerate(les.PAIRS):
        assert np.max(np.abs(tau[o] + nu_t * (S[i, j] + S[j, i]))) <= 1e-10
    got = les.les_rhs(ub, th, in_scale, out_scale)
    ref = ns.rhs(ub) - nu_t * ns.k_squared(n) * ub
    assert diag.rel_l2(got, ref, n) <= 1e-11
    assert diag.rel_l2(got, ns.rhs(ub), n) >= 0.1


def test_closure_scale_conventions():
    """tau = out_scale f(grad / in_scale): doubling out_scale doubles tau; scaling the
    filtered field and in_scale by the same factor leaves tau unchanged."""
    n = 16
    ub = band_filling_state(n, seed=12)
    th = rand_theta(5)
    t1 = les.closure_tau(th, ub, 2.0, 0.25)
    assert np.max(np.abs(les.closure_tau(th, ub, 2.0, 0.5) - 2.0 * t1)) <= 1e-15 * np.max(np.abs(t1)) * 4
    t3 = les.closure_tau(th, 3.0 * ub, 6.0, 0.25)
    assert np.max(np.abs(t3 - t1)) <= 1e-12 * np.max(np.abs(t1))
    # the network is not linear: scaling the field alone changes tau by more than the factor
    t4 = les.closure_tau(th, 3.0 * ub, 2.0, 0.25)
    assert np.max(np.abs(t4 - 3.0 * t1)) >= 1e-3 * np.max(np.abs(t1))
