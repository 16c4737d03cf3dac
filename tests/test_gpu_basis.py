"""Sine / cosine bases (SFF, SSF, ...) on the GPU against the FP64 oracle definitions."""
import numpy as np
import pytest

from oracle import diag, fft as offt

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("shape,bx,by", [((16, 24, 8), 1, 0), ((32, 16, 12), 2, 0), ((12, 32, 16), 0, 1),
                                         ((24, 8, 8), 2, 2), ((64, 48, 16), 1, 2), ((8, 96, 8), 2, 1),
                                         ((192, 8, 8), 1, 0), ((8, 256, 8), 0, 2), ((384, 12, 8), 2, 1),
                                         ((8, 768, 8), 1, 2), ((1024, 8, 8), 1, 2), ((8, 1024, 8), 2, 1)])
def test_basis_vs_oracle(tk, shape, bx, by, dt):
    import torch
    tdt = torch.float32 if dt == "f32" else torch.float64
    rng = np.random.default_rng(sum(shape) + bx + 3 * by)
    f = rng.standard_normal((1,) + shape)
    plan = tk.FFT3D(*shape, dtype=tdt, basis_x=bx, basis_y=by)
    X = plan.r2c(torch.from_numpy(f.astype(np.float32 if dt == "f32" else np.float64)).cuda())
    ref = offt.rfft3_basis(f[0], bx, by)
    tol = 1e-5 if dt == "f32" else 1e-12
    assert diag.rel_l2(X.cpu().numpy()[0], ref) <= tol
    G = rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape)
    g = plan.c2r(torch.from_numpy(G[None].astype(np.complex64 if dt == "f32" else np.complex128)).cuda())
    assert diag.rel_l2(g.cpu().numpy()[0], offt.irfft3_basis(G, shape[2], bx, by)) <= tol


@pytest.mark.parametrize("n", [256, 512])
def test_sff_round_trip_large(tk, n):
    import torch
    import synth
    f = torch.from_numpy(synth.gaussian_field((n, n, n), 0)).cuda()
    plan = tk.FFT3D(n, basis_x=1)
    back = plan.c2r(plan.r2c(f))
    err = torch.linalg.vector_norm((back - f.view_as(back)).double()) / torch.linalg.vector_norm(f.double())
    assert err.item() <= 1e-5
    plan2 = tk.FFT3D(n, basis_x=2, basis_y=2)
    back = plan2.c2r(plan2.r2c(f))
    err = torch.linalg.vector_norm((back - f.view_as(back)).double()) / torch.linalg.vector_norm(f.double())
    assert err.item() <= 1e-5


SSS_BASES = [(2, 2, 1), (1, 1, 2), (1, 2, 1), (2, 1, 2), (1, 1, 1), (2, 2, 2)]


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("shape,b", [((8, 8, 8), SSS_BASES[0]), ((12, 16, 24), SSS_BASES[1]),
                                     ((16, 12, 48), SSS_BASES[2]), ((32, 24, 16), SSS_BASES[3]),
                                     ((24, 32, 96), SSS_BASES[4]), ((64, 48, 128), SSS_BASES[5]),
                                     ((16, 16, 192), SSS_BASES[0]), ((8, 12, 384), SSS_BASES[1]),
                                     ((8, 8, 768), SSS_BASES[2]), ((8, 8, 1024), SSS_BASES[3]),
                                     ((96, 64, 12), SSS_BASES[4])])
def test_sss_vs_oracle(tk, shape, b, dt):
    """SSS family (sine / cosine on every axis, real spectral data): forward and inverse
    against the oracle definitions, every z length kernel (8 ... 1024), both dtypes; c2r
    preserves its input and the in-place plan gives the same output bit for bit."""
    import torch
    tdt = torch.float32 if dt == "f32" else torch.float64
    npdt = np.float32 if dt == "f32" else np.float64
    rng = np.random.default_rng(sum(shape) + sum(b))
    f = rng.standard_normal((2,) + shape)
    plan = tk.FFT3D(*shape, batch=2, dtype=tdt, basis_x=b[0], basis_y=b[1], basis_z=b[2])
    X = plan.r2c(torch.from_numpy(f.astype(npdt)).cuda())
    assert X.dtype == tdt and tuple(X.shape) == (2,) + shape
    tol = 1e-5 if dt == "f32" else 1e-12
    Xh = X.cpu().numpy()
    for m in range(2):
        assert diag.rel_l2(Xh[m], offt.rfft3_sss(f[m], *b)) <= tol
    G = rng.standard_normal((2,) + shape).astype(npdt)
    Gd = torch.from_numpy(G).cuda()
    g = plan.c2r(Gd)
    assert np.array_equal(Gd.cpu().numpy(), G), "c2r modified its input"
    gh = g.cpu().numpy()
    for m in range(2):
        assert diag.rel_l2(gh[m], offt.irfft3_sss(G[m].astype(np.float64), *b)) <= tol
    plan.close()
    p2 = tk.FFT3D(*shape, batch=2, dtype=tdt, basis_x=b[0], basis_y=b[1], basis_z=b[2],
                  flags=tk.TK_FFT_C2R_OVERWRITE)
    assert torch.equal(p2.c2r(Gd), g)
    p2.close()


def test_sss_rejects_fourier_xy_with_sine_z(tk):
    import ctypes
    h = ctypes.c_void_p()
    st = tk.lib().fft3d_plan_create_basis3(ctypes.byref(h), 16, 16, 16, 1, tk.TK_F32, 0, 1, 1, 0)
    assert st == tk.TK_EUNSUPPORTED and h.value is None


def test_sss_512_whole_lines(tk):
    """512^3 FP32 SSS (cos, cos, sin: the u_z basis): complete z-lines and x-lines of the
    forward output against the definitions, complete z-lines of the inverse of a random
    coefficient field, and the round trip over the whole field."""
    import torch
    import synth
    n = 512
    b = (2, 2, 1)
    f = synth.gaussian_field((1, n, n, n), 0)
    plan = tk.FFT3D(n, dtype=torch.float32, basis_x=b[0], basis_y=b[1], basis_z=b[2])
    x = torch.from_numpy(f).cuda()
    X = plan.r2c(x)
    zp = [(0, 0), (1, 511), (255, 256), (511, 3)]
    ref = offt.sss_lines(f[0], *b, axis=2, pts=zp)
    for i, (p, q) in enumerate(zp):
        assert diag.rel_l2(X[0, p, q, :].cpu().numpy(), ref[i]) <= 1e-5, (p, q)
    xp = [(0, 0), (7, 300), (511, 511)]
    ref = offt.sss_lines(f[0], *b, axis=0, pts=xp)
    for i, (p, q) in enumerate(xp):
        assert diag.rel_l2(X[0, :, p, q].cpu().numpy(), ref[i]) <= 1e-5, (p, q)
    back = plan.c2r(X)
    err = torch.linalg.vector_norm((back - x).double()) / torch.linalg.vector_norm(x.double())
    assert err.item() <= 1e-5
    G = synth.gaussian_field((1, n, n, n), 3)
    g = plan.c2r(torch.from_numpy(G).cuda())
    ip = [(0, 0), (100, 17), (511, 256)]
    ref = offt.sss_lines(G[0], *b, axis=2, pts=ip, inverse=True)
    for i, (p, q) in enumerate(ip):
        assert diag.rel_l2(g[0, p, q, :].cpu().numpy(), ref[i]) <= 1e-5, (p, q)
    plan.close()
