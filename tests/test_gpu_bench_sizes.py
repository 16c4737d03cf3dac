"""Oracle parity at the sizes the benchmark times: the 1024^3 transform pair with the tuned
tiles and the pair's plan flags, IF-RK4 and Rayleigh-Benard steps at 512^3, the sine-basis
(SFF) transform at 512^3 and the energy transfer at 256^3; and the solver at its largest
grid, 1024^3, on a band-limited field whose exact spectra the oracle gives on a small grid.

Grids too large for the full oracle transform are checked on complete kz-planes, complete
x-lines, or through separable fields whose exact spectrum is a product of 1D transforms."""
import numpy as np
import pytest

import synth
from oracle import diag, fft as offt, init as oinit, ns as ons, rbc as orbc, transfer as otr

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _bench_plan(tk, n):
    import torch
    from paper_1805_07801_amd import tune
    assert tune.load_default() > 0
    return tk.FFT3D(n, dtype=torch.float32, flags=tk.TK_FFT_TIMING | tk.TK_FFT_C2R_OVERWRITE)


def test_fft_1024_separable_full_field(tk):
    """f = sum_m a_m(x) b_m(y) c_m(z) (random vectors) has the exact spectrum
    sum_m A_m(kx) B_m(ky) C_m(kz) with A = a's 1D transform / N, so the whole 1024^3
    forward output is checked, mode by mode; likewise the c2r of a separable spectrum
    G = sum_m A'_m B'_m C'_m is sum_m Re[a'_m(x) b'_m(y) c'_m(z)] with c'(z) = sum_kz w(kz)
    C'(kz) e^{i kz z}.  Tuned tiles, the pair's plan flags (c2r overwrites its input).
    Storing the fields in FP32 perturbs them by at most 2^-24 relative, far below 1e-5."""
    import torch
    from paper_1805_07801_amd import tune
    n, nh, m = 1024, 513, 3
    _say("1024^3 separable r2c")
    rng = np.random.default_rng(40)
    a, b, c = (rng.standard_normal((m, n)) for _ in range(3))
    A = np.stack([offt.fft1d(a[i], -1) / n for i in range(m)])
    B = np.stack([offt.fft1d(b[i], -1) / n for i in range(m)])
    C = np.stack([offt.fft1d(c[i], -1)[:nh] / n for i in range(m)])
    bc = [b[i][:, None] * c[i][None, :] for i in range(m)]
    f = np.empty((1, n, n, n), dtype=np.float32)
    for x0 in range(0, n, 64):
        f[0, x0:x0 + 64] = sum(a[i, x0:x0 + 64, None, None] * bc[i][None] for i in range(m))
    del bc
    try:
        plan = _bench_plan(tk, n)
        x = torch.from_numpy(f).cuda()
        del f
        X = plan.r2c(x)
        Xh = X.cpu().numpy()[0]
        del x
        w = offt.hermitian_weight(n)
        BC = [B[i][:, None] * C[i][None, :] for i in range(m)]
        num = den = 0.0
        for x0 in range(0, n, 64):
            ref = sum(A[i, x0:x0 + 64, None, None] * BC[i][None] for i in range(m))
            num += float(np.sum(w * np.abs(Xh[x0:x0 + 64] - ref) ** 2))
            den += float(np.sum(w * np.abs(ref) ** 2))
        del Xh, BC
        assert np.sqrt(num / den) <= 1e-5, np.sqrt(num / den)
        _say("1024^3 separable c2r")
        A2, B2 = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n)) for _ in range(2))
        C2 = rng.standard_normal((m, nh)) + 1j * rng.standard_normal((m, nh))
        BC2 = [B2[i][:, None] * C2[i][None, :] for i in range(m)]
        for x0 in range(0, n, 64):
            X[0, x0:x0 + 64] = torch.from_numpy(
                sum(A2[i, x0:x0 + 64, None, None] * BC2[i][None] for i in range(m)).astype(np.complex64)).cuda()
        del BC2
        y = plan.c2r(X).cpu().numpy()[0]
        del X
        wz = np.full(nh, 2.0)
        wz[0] = wz[-1] = 1.0
        a2 = [offt.fft1d(A2[i], +1) for i in range(m)]
        b2 = [offt.fft1d(B2[i], +1) for i in range(m)]
        c2 = []
        for i in range(m):
            line = np.zeros(n, dtype=np.complex128)
            line[:nh] = wz * C2[i]
            c2.append(offt.fft1d(line, +1))
        bc2 = [b2[i][:, None] * c2[i][None, :] for i in range(m)]
        num = den = 0.0
        for x0 in range(0, n, 64):
            ref = np.real(sum(a2[i][x0:x0 + 64, None, None] * bc2[i][None] for i in range(m)))
            num += float(np.sum((y[x0:x0 + 64] - ref) ** 2))
            den += float(np.sum(ref ** 2))
        assert np.sqrt(num / den) <= 1e-5, np.sqrt(num / den)
        plan.close()
    finally:
        tk.tune_clear()


def test_fft_1024_planes_of_the_bench_input(tk):
    """The benchmark's 1024^3 input (N(0,1), seed 0), tuned tiles and plan flags: complete
    kz-planes kz = 0, 1, 341, 511, 512 (each holding every x- and y-line of that kz)
    against the definition along z followed by the oracle's 1D transforms along y and x,
    each plane to relative L2 1e-5; round trip and Parseval over the whole field."""
    import torch
    n = 1024
    kzs = [0, 1, 341, 511, 512]
    _say("1024^3 planes of the seed-0 input")
    f = synth.gaussian_field((1, n, n, n), 0)
    try:
        plan = _bench_plan(tk, n)
        x = torch.from_numpy(f).cuda()
        X = plan.r2c(x)
        a, b = plan.parseval(x, X)
        assert abs(a - b) <= 1e-5 * a
        got = X[0, :, :, kzs].permute(2, 0, 1).cpu().numpy()
        ref = offt.dft_planes(f[0], kzs)
        for i, kz in enumerate(kzs):
            e = diag.rel_l2(got[i], ref[i])
            assert e <= 1e-5, (kz, e)
        back = plan.c2r(X)
        del X
        err = torch.linalg.vector_norm((back - x).double()) / torch.linalg.vector_norm(x.double())
        assert err.item() <= 1e-5
        plan.close()
    finally:
        tk.tune_clear()


def test_rk4_512_step(tk, band512):
    """One IF-RK4 step (the paper's integrator) of the 512^3 band-filling field, the fused
    stepper and tuned tiles, against the oracle: global and per shell 1..170 within 1e-4."""
    import torch
    from paper_1805_07801_amd import tune
    n = 512
    nu, h = 1e-3, 2e-4
    _say("512^3 IF-RK4 step")
    try:
        assert tune.load_default() > 0
        ud = torch.from_numpy(band512.astype(np.complex64)).cuda()
        u = ud.cpu().numpy().astype(np.complex128)
        s = tk.NS(n, dtype=torch.float32, nu=nu, scheme="rk4")
        s.step(ud, h, 1)
        got = ud.cpu().numpy()
        del ud
        ref = ons.ifrk4_step(u, nu, h)
        del u
        assert diag.rel_l2(got, ref, n) <= 1e-4
        e = diag.shell_rel_l2(got, ref, n, range(1, 171))
        assert np.max(e) <= 1e-4, (int(np.argmax(e)) + 1, float(np.max(e)))
        s.close()
    finally:
        tk.tune_clear()


def test_rbc_512_rhs_and_step(tk, band512):
    """Rayleigh-Benard (FFF) at 512^3 FP32: one right-hand side and one IF-RK2 step of a
    band-filling state (velocity and temperature with every kept mode O(1)) against the
    oracle, globally and per shell."""
    import torch
    n = 512
    Ra, Pr, box, h = 1e6, 1.0, 1.0, 1e-4
    _say("512^3 RBC right-hand side and step")
    u = 0.1 * band512
    t = offt.rfft3(synth.gaussian_field((n, n, n), 52).astype(np.float64)) * ons.dealias_mask(n)
    t[0, 0, 0] = 0
    t *= 0.1 / np.sqrt(diag.energy(np.stack([t, 0 * t, 0 * t])))
    st = torch.from_numpy(np.concatenate([u, t[None]]).astype(np.complex64)).cuda()
    st64 = st.cpu().numpy().astype(np.complex128)
    del u, t
    s = tk.RBC(n, Ra=Ra, Pr=Pr, box=box, dtype=torch.float32)
    got = s.rhs(st).cpu().numpy()
    Nu, Nt = orbc.rhs(st64[:3], st64[3], 2 * np.pi / box)
    ref = np.concatenate([Nu, Nt[None]])
    del Nu, Nt
    assert diag.rel_l2(got, ref, n) <= 1e-5
    e = diag.shell_rel_l2(got, ref, n, range(1, 171))
    assert np.max(e) <= 1e-4, (int(np.argmax(e)) + 1, float(np.max(e)))
    del got, ref
    s.step(st, h, 1)
    got = st.cpu().numpy()
    del st
    nu, kappa = orbc.viscosities(Ra, Pr)
    uu, tt = orbc.ifrk2_step(st64[:3], st64[3], nu, kappa, h, a=2 * np.pi / box)
    del st64
    ref = np.concatenate([uu, tt[None]])
    del uu, tt
    assert diag.rel_l2(got, ref, n) <= 1e-4
    e = diag.shell_rel_l2(got, ref, n, range(1, 171))
    assert np.max(e) <= 1e-4, (int(np.argmax(e)) + 1, float(np.max(e)))
    s.close()


def test_sff_512_whole_lines(tk):
    """The 512^3 pair with the sine basis along x (as benchmarked): complete x-lines of the
    forward output on several (ky, kz) columns against the definitions (direct sums over y
    and z, the sine sums over x), and complete x-lines of the inverse of a random spectrum
    at several (y, z) points."""
    import torch
    n = 512
    _say("512^3 SFF lines")
    f = synth.gaussian_field((1, n, n, n), 0)
    plan = tk.FFT3D(n, dtype=torch.float32, basis_x=1)
    X = plan.r2c(torch.from_numpy(f).cuda())
    cols = [(0, 0), (1, 0), (0, 256), (255, 1), (256, 256), (511, 100), (300, 17)]
    ref = offt.dft_x_lines_basis(f[0], offt.SINE, cols)
    for i, (b, c) in enumerate(cols):
        e = diag.rel_l2(X[0, :, b, c].cpu().numpy(), ref[i])
        assert e <= 1e-5, ((b, c), e)
    rng = np.random.default_rng(9)
    G = (rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape)).astype(np.complex64)
    g = plan.c2r(torch.from_numpy(G).cuda()).cpu().numpy()[0]
    pts = [(0, 0), (3, 511), (256, 255), (511, 7)]
    ref = offt.idft_x_lines_basis(G[0], n, offt.SINE, pts)
    for i, (b, c) in enumerate(pts):
        e = diag.rel_l2(g[:, b, c], ref[i])
        assert e <= 1e-5, ((b, c), e)
    plan.close()


def test_energy_transfer_256(tk):
    """Shell transfer T(s) at 256^3 FP32 of a band-filling field (every shell up to the
    cutoff carries energy) against the oracle; T sums to zero (energy conservation of the
    nonlinear term)."""
    import torch
    n = 256
    _say("256^3 energy transfer")
    u = oinit.band_filling(synth.gaussian_field((3, n, n, n), 23))
    s = tk.NS(n, dtype=torch.float32, nu=0.0)
    got = np.array(s.energy_transfer(torch.from_numpy(u.astype(np.complex64)).cuda()))
    ref = otr.shell_transfer(u)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-5 * scale
    assert abs(np.sum(got)) <= 1e-5 * scale * len(got)
    s.close()


def _embed(small, n):
    """A band-limited spectral state on the n^3 grid from its modes on a small grid (oracle
    layout [c][m][m][m/2+1], every nonzero mode with |k_i| < m/2): (indices, values) of the
    nonzero modes at their places on the n^3 grid."""
    m = small.shape[1]
    c, i, j, l = np.nonzero(np.abs(small) > 1e-14 * np.max(np.abs(small)))
    wrap = lambda a: np.where(a < m // 2, a, a - m) % n
    return (c, wrap(i), wrap(j), l), small[c, i, j, l]


def test_ns_1024_taylor_green_rhs_and_step(tk):
    """The solver at its largest grid, 1024^3 FP32 with the fused stepper: the right-hand
    side of the Taylor-Green field and one IF-RK2 step against the oracle.  Taylor-Green
    holds modes |k_i| <= 1, its right-hand side |k_i| <= 2 and one step's second stage
    |k_i| <= 4, all inside the 2/3 set of a 16^3 grid, so the oracle's 16^3 results are the
    exact 1024^3 spectra; every other mode of the 1024^3 results must stay zero."""
    import torch
    n, m = 1024, 16
    nu, h = 0.01, 0.01
    u16 = offt.rfft3(synth.taylor_green(m))
    r16 = ons.rhs(u16)
    s16 = ons.ifrk2_step(u16, nu, h)[0]
    _say("1024^3 Taylor-Green right-hand side and step")
    s = tk.NS(n, dtype=torch.float32, nu=nu)
    try:
        (c, i, j, l), v = _embed(u16, n)
        u = torch.zeros((3, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
        at = lambda a: torch.from_numpy(a.astype(np.int64)).cuda()
        u[at(c), at(i), at(j), at(l)] = torch.from_numpy(v.astype(np.complex64)).cuda()
        for ref, got_fn in ((r16, lambda: s.rhs(u)), (s16, lambda: (s.step(u, h, 1), u)[1])):
            got = got_fn()
            (rc, ri, rj, rl), rv = _embed(ref, n)
            g = got[at(rc), at(ri), at(rj), at(rl)].cpu().numpy().astype(np.complex128)
            rn = np.linalg.norm(rv)
            assert np.linalg.norm(g - rv) <= 1e-5 * rn
            # the rest of the 1024^3 spectrum (the reference's modes cleared) stays zero
            got[at(rc), at(ri), at(rj), at(rl)] = 0
            rest = float(torch.linalg.vector_norm(got))
            assert rest <= 1e-5 * rn, rest / rn
            del got
    finally:
        s.close()
