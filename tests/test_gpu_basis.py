"""Sine / cosine bases (SFF, SSF, ...) on the GPU against the FP64 oracle definitions."""
import numpy as np
import pytest

from oracle import diag, fft as offt

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("shape,bx,by", [((16, 24, 8), 1, 0), ((32, 16, 12), 2, 0), ((12, 32, 16), 0, 1),
                                         ((24, 8, 8), 2, 2), ((64, 48, 16), 1, 2), ((8, 96, 8), 2, 1)])
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
