"""Learned closure on the GPU against the FP64 oracle: network forward / gradients / Adam,
filtered-DNS training data, the LES step and its fallbacks."""
import numpy as np
import pytest

import synth
from oracle import diag, fft as offt, init as oinit, les as oles, mlp as omlp, ns as ons

pytestmark = pytest.mark.gpu


def theta0(seed=0, scale=1.0):
    Ws, bs = synth.mlp_init(seed=seed)
    rng = np.random.default_rng(seed + 1)
    bs = [rng.standard_normal(b.shape) * 0.1 for b in bs]
    return omlp.bf16_round(omlp.pack([W * scale for W in Ws], bs))


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def test_bf16_copy_matches_oracle_rounding(tk):
    rng = np.random.default_rng(0)
    th = rng.standard_normal(5190) * 3
    th[:4] = [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0, 1e-30]
    net = tk.Closure(th)
    assert np.array_equal(net.bf16_bits(), omlp.bf16_bits(th))


@pytest.mark.parametrize("M", [1, 255, 4096, 100003])
def test_forward_vs_oracle(tk, M):
    import torch
    th = theta0(2)
    x = np.random.default_rng(M).standard_normal((9, M)).astype(np.float32) * 2.0
    net = tk.Closure(th, in_scale=2.0, out_scale=0.5)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = 0.5 * omlp.forward(th, x.astype(np.float64) / 2.0)
    assert rel(y, ref) <= 1e-5


def test_forward_extreme_inputs_vs_oracle(tk):
    """Inputs that drive the activations far into both GELU tails (|x| up to ~100, where
    GELU(x) is x or a tiny negative number), exact zeros and values near the FP32 underflow,
    at a ragged point count: the forward still matches the oracle's exact-erf GELU."""
    import torch
    th = theta0(4)
    M = 4099
    rng = np.random.default_rng(11)
    x = (rng.standard_normal((9, M)) * 40.0).astype(np.float32)
    x[:, :64] = 0.0
    x[:, 64:128] = (rng.standard_normal((9, 64)) * 1e-30).astype(np.float32)
    net = tk.Closure(th, in_scale=1.0, out_scale=1.0)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = omlp.forward(th, x.astype(np.float64))
    assert np.all(np.isfinite(y))
    assert rel(y, ref) <= 1e-5
    assert rel(y[:, :128], ref[:, :128]) <= 1e-5


# flat parameter groups W1, b1, W2, b2, W3, b3
GROUPS = [(0, 576), (576, 640), (640, 4736), (4736, 4800), (4800, 5184), (5184, 5190)]


def assert_grad(g, gref, tol):
    """Every parameter group on its own (a wrong bias or output-layer entry would hide in
    the norm of the 4096 hidden weights)."""
    assert rel(g, gref) <= tol
    for a, b in GROUPS:
        assert rel(g[a:b], gref[a:b]) <= tol, (a, b)


@pytest.mark.parametrize("M", [1, 17, 300, 65536, 262147])
def test_loss_and_gradient_vs_oracle(tk, M):
    import torch
    th = theta0(3)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((9, M)).astype(np.float32)
    t = rng.standard_normal((6, M)).astype(np.float32)
    net = tk.Closure(th, in_scale=1.5, out_scale=2.0)
    loss = net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = net.grad.cpu().numpy()
    y = omlp.forward(th, x.astype(np.float64) / 1.5)
    Lref, dy = omlp.mse_loss(y, t.astype(np.float64) / 2.0)
    gref = omlp.backward(th, x.astype(np.float64) / 1.5, dy)
    assert abs(loss - Lref) <= 1e-5 * Lref
    assert_grad(g, gref, 1e-4)
    # reproducible: the same call gives the same bits
    net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    assert np.array_equal(net.grad.cpu().numpy(), g)
    # generic backward with a given upstream gradient
    dyr = rng.standard_normal((6, M)).astype(np.float32)
    g2 = net.backward(torch.from_numpy(x).cuda(), torch.from_numpy(dyr).cuda()).cpu().numpy()
    assert_grad(g2, omlp.backward(th, x.astype(np.float64) / 1.5, dyr.astype(np.float64)), 1e-4)


def test_adam_steps_vs_oracle(tk):
    import torch
    th = theta0(4)
    rng = np.random.default_rng(1)
    net = tk.Closure(th, lr=1e-3)
    w, m, v = th.copy(), np.zeros(5190), np.zeros(5190)
    for k in range(1, 4):
        g = rng.standard_normal(5190).astype(np.float32)
        net.grad.copy_(torch.from_numpy(g))
        net.adam_step()
        w, m, v = omlp.adam(w, m, v, g.astype(np.float64), k, 1e-3)
    assert net.opt.step == 3
    assert np.max(np.abs(net.w32.cpu().numpy() - w)) <= 1e-6
    assert np.array_equal(net.bf16_bits(), omlp.bf16_bits(net.w32.cpu().numpy()))


def test_filter_dns_vs_oracle(tk):
    import torch
    n_dns, n_les, kc = 128, 64, 21
    # white-noise solenoidal field: plenty of energy above the cutoff, so tau = O(1)
    noise = synth.gaussian_field((3, n_dns, n_dns, n_dns), 5).astype(np.float64)
    u = ons.project(offt.rfft3(noise) * ons.dealias_mask(n_dns))
    u /= np.sqrt(diag.energy(u))
    g, t, ub = tk.les_filter_dns(torch.from_numpy(u.astype(np.complex64)).cuda(), n_les, kc, with_ubar=True)
    ubar = oles.filtered_velocity(u, n_les, kc)
    assert diag.rel_l2(ub.cpu().numpy(), ubar, n_les) <= 1e-6
    gref = oles.gradients(ubar).reshape(9, -1)
    assert rel(g.cpu().numpy(), gref) <= 1e-5
    tref = oles.sgs_stress(u, n_les, kc).reshape(6, -1)
    assert rel(t.cpu().numpy(), tref) <= 1e-4


def test_les_step_vs_oracle_and_fallback(tk):
    import torch
    n = 32
    nu, h = 5e-3, 0.004
    u0 = oinit.random_solenoidal(synth.gaussian_field((3, n, n, n), 9))
    th = theta0(5, scale=0.3)
    s_in, s_out = 3.0, 0.05
    net = tk.Closure(th, in_scale=s_in, out_scale=s_out)
    s = tk.NS(n, dtype=torch.float32, nu=nu)
    ud = torch.from_numpy(u0.astype(np.complex64)).cuda()
    t, fb = tk.les_step(s, net, ud, h, 1)
    assert fb == 0 and abs(t - h) < 1e-15
    ref = ons.ifrk2_step(u0, nu, h, rhs_fn=lambda v: oles.les_rhs(v, th, s_in, s_out))[0]
    assert diag.rel_l2(ud.cpu().numpy(), ref, n) <= 1e-4
    # the model changes the step (the parity above is not the no-model path)
    plain = ons.ifrk2_step(u0, nu, h)[0]
    assert diag.rel_l2(ref, plain, n) > 1e-6
    # no model: identical to the plain solver step
    ua = torch.from_numpy(u0.astype(np.complex64)).cuda()
    ub = ua.clone()
    tk.les_step(s, None, ua, h, 2)
    s.step(ub, h, 2)
    assert torch.equal(ua, ub)
    # non-finite weights: fallback to the plain right-hand side
    bad = th.copy()
    bad[100] = np.nan
    netb = tk.Closure(bad, in_scale=s_in, out_scale=s_out)
    uc = torch.from_numpy(u0.astype(np.complex64)).cuda()
    _, fb = tk.les_step(s, netb, uc, h, 2)
    assert fb == 1 and torch.equal(uc, ub)
    # a model that blows the state up: restored and redone without the model
    huge = tk.Closure(th, in_scale=s_in, out_scale=3e38)
    ud2 = torch.from_numpy(u0.astype(np.complex64)).cuda()
    _, fb = tk.les_step(s, huge, ud2, h, 2)
    assert fb == 2 and torch.equal(ud2, ub)


def test_les_steps_in_separate_calls(tk):
    """Three calls of one LES step, with other GPU work and synchronisations between them,
    match the oracle after every step and give the bits of one call of three steps on
    another state buffer; a closure with another output scale steps to its own oracle
    result."""
    import torch
    n = 32
    nu, h = 5e-3, 0.004
    u0 = oinit.random_solenoidal(synth.gaussian_field((3, n, n, n), 11))
    th = theta0(6, scale=0.3)
    s_in, s_out = 3.0, 0.05
    net = tk.Closure(th, in_scale=s_in, out_scale=s_out)
    s = tk.NS(n, dtype=torch.float32, nu=nu)
    ua = torch.from_numpy(u0.astype(np.complex64)).cuda()
    ref = u0
    t = 0.0
    for k in range(3):
        t, fb = tk.les_step(s, net, ua, h, 1, t)
        assert fb == 0 and abs(t - (k + 1) * h) < 1e-14
        junk = torch.randn(1 << 20, device="cuda")
        assert torch.isfinite(junk.sum()).item()
        torch.cuda.synchronize()
        ref = ons.ifrk2_step(ref, nu, h, rhs_fn=lambda v: oles.les_rhs(v, th, s_in, s_out))[0]
        assert diag.rel_l2(ua.cpu().numpy(), ref, n) <= 1e-4, k
    ub = torch.from_numpy(u0.astype(np.complex64)).cuda()
    tk.les_step(s, net, ub, h, 3)
    assert torch.equal(ua, ub)
    # another output scale
    net2 = tk.Closure(th, in_scale=s_in, out_scale=2 * s_out)
    uc = torch.from_numpy(u0.astype(np.complex64)).cuda()
    tk.les_step(s, net2, uc, h, 1)
    ref2 = ons.ifrk2_step(u0, nu, h, rhs_fn=lambda v: oles.les_rhs(v, th, s_in, 2 * s_out))[0]
    assert diag.rel_l2(uc.cpu().numpy(), ref2, n) <= 1e-4


PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def apriori(y6, tau6, grad9):
    """Per-component correlation of a predicted stress with the true one (0 where the
    prediction is constant), and the sub-grid dissipation -<tau_ij S_ij> of each (S the
    filtered strain rate), from device tensors [6][M] / [9][M]."""
    y = y6.cpu().numpy().astype(np.float64)
    t = tau6.cpu().numpy().astype(np.float64)
    g = grad9.cpu().numpy().astype(np.float64).reshape(3, 3, -1)
    S = 0.5 * (g + g.transpose(1, 0, 2))
    corr = [float(np.corrcoef(y[c], t[c])[0, 1]) if np.std(y[c]) > 0 else 0.0 for c in range(6)]

    def diss(T):
        return -float(np.mean(sum((1 if i == j else 2) * T[c] * S[i, j] for c, (i, j) in enumerate(PAIRS))))

    return corr, diss(y), diss(t)


def test_a_posteriori_closure(tk):
    """The LES configuration end to end: 512^3 decaying DNS (seed 1) filtered at kc = 21
    onto 64^3 for training (a snapshot every 5 steps, 100..200), network trained on the GPU,
    then checked against what the method without it gives:
      a priori, on held-out filtered DNS (seed 2, steps 150 and 200): every predicted
        stress component correlates positively with the true one, and the predicted
        sub-grid dissipation has the true sign (energy leaves the resolved scales);
      a posteriori, LES from the filtered held-out DNS at step 100 to the time of its
        step 200, with and without the closure, scored by shell spectra against the
        filtered DNS: over the shells next to the cutoff (s = 15..21, where a sub-grid
        model acts) and over all shells the closure's mean error is at least 3% below the
        no-model run's, and the closure drains energy (the LES ends with less energy).
    A zero-output network passes neither check; the mean error stays within 5%, and the LES
    with the closure runs at least 10x the DNS steps/s."""
    import torch
    from paper_1805_07801_amd import les_train as lt

    def noise(seed, n=512):
        return torch.from_numpy(synth.gaussian_field((3, n, n, n), seed)).cuda()

    snaps, _, _, dns_rate = lt.dns_snapshots(seed=1, snap_steps=list(range(100, 201, 5)), noise_fn=noise)
    held, ub, _, _ = lt.dns_snapshots(seed=2, snap_steps=[150, 200], keep_ubar=(100, 200), noise_fn=noise)
    Ws, bs = synth.mlp_init(seed=7)
    net, log = lt.train(snaps, omlp.pack(Ws, bs), steps=4000, lr=5e-3)
    # predicting zero stress scores 1 in these normalised units
    assert log[-1][1] < 1.0 and log[-1][1] < log[0][1]
    zero = tk.Closure(np.zeros(5190), in_scale=net.in_scale, out_scale=net.out_scale)
    for (m, _, g, tau) in held:
        corr, dm, dt = apriori(net.forward(g), tau, g)
        print("a priori, held-out step %d: correlations %s, dissipation %.3e (true %.3e)"
              % (m, np.round(corr, 3), dm, dt))
        assert min(corr) >= 0.02, corr
        assert dt > 0 and dm >= 0.1 * dt
        corr0, d0, _ = apriori(zero.forward(g), tau, g)
        assert min(corr0) < 0.02 and d0 < 0.1 * dt  # the zero network fails the same checks
    ta, u0 = ub[100]
    tb, u1 = ub[200]
    ref = tk.NS(64, dtype=torch.float32, nu=1e-3)
    Eref = ref.diagnostics(u1)["spectrum"]
    um, Em, nst, les_rate, fbm = lt.les_run(net, u0, ta, tb, 1e-3)
    un, En, _, _, fbn = lt.les_run(None, u0, ta, tb, 1e-3, nsteps=nst)
    _, Ez, _, _, fbz = lt.les_run(zero, u0, ta, tb, 1e-3, nsteps=nst)
    assert fbm == 0 and fbn == 0 and fbz == 0
    em, _ = lt.spectrum_error(Em, Eref)
    en, _ = lt.spectrum_error(En, Eref)
    ec, _ = lt.spectrum_error(Em, Eref, 15, 21)
    enc, _ = lt.spectrum_error(En, Eref, 15, 21)
    ezc, _ = lt.spectrum_error(Ez, Eref, 15, 21)
    print("a posteriori: mean spectrum error s=1..21 %.4f (no model %.4f); s=15..21 %.4f (no model %.4f); "
          "energy %.5f (no model %.5f, filtered DNS %.5f); final loss %.4f"
          % (em, en, ec, enc, sum(Em), sum(En), sum(Eref), log[-1][1]))
    assert em <= 0.05
    assert ec <= 0.97 * enc and em <= 0.97 * en
    assert sum(Em) < sum(En)
    assert ezc > 0.97 * enc  # the zero network gains nothing
    # the 64^3 LES with the closure runs at least 10x the 512^3 DNS's steps/s
    print("LES with closure %.0f steps/s, DNS %.1f steps/s" % (les_rate, dns_rate))
    assert les_rate >= 10 * dns_rate
