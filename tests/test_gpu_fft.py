"""Parity of the HIP 3D transform with the FP64 oracle (GPU).

Tolerance: relative L2 (Hermitian-weighted over the half spectrum) <= 1e-5 for FP32 and
<= 1e-12 for FP64, forward and inverse, on the same seeded inputs.
"""
import numpy as np
import pytest

import synth
from oracle import diag, fft as offt

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-12}


def _torch_dtype(name):
    import torch
    return torch.float32 if name == "f32" else torch.float64


def _run_pair(tk, shape, batch, dt, seed=0):
    import torch
    nx, ny, nz = shape
    f = synth.gaussian_field((batch, nx, ny, nz), seed, dtype=np.float32 if dt == "f32" else np.float64)
    plan = tk.FFT3D(nx, ny, nz, batch=batch, dtype=_torch_dtype(dt))
    x = torch.from_numpy(f).cuda()
    X = plan.r2c(x)
    X_np = X.cpu().numpy()
    # inverse of a (non-Hermitian) random spectrum: the w(kz) Re[...] definition
    rng = np.random.default_rng(seed + 1)
    G = (rng.standard_normal(X_np.shape) + 1j * rng.standard_normal(X_np.shape)).astype(X_np.dtype)
    Gd = torch.from_numpy(G).cuda()
    g = plan.c2r(Gd)
    torch.cuda.synchronize()
    assert np.array_equal(Gd.cpu().numpy(), G), "c2r modified its input"
    return f, X_np, G, g.cpu().numpy(), plan, x, X


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("n", [8, 12, 16, 24, 32, 48, 64, 96, 128])
def test_fft_cubic_vs_oracle(tk, n, dt):
    f, X, G, g, plan, x, Xd = _run_pair(tk, (n, n, n), 1, dt, seed=n)
    ref = offt.rfft3(f[0].astype(np.float64))
    assert diag.rel_l2(X[0], ref, n) <= TOL[dt]
    gref = offt.irfft3(G[0].astype(np.complex128), n)
    assert diag.rel_l2(g[0], gref) <= TOL[dt]
    # round trip and Parseval (FP64 reductions on the device)
    back = plan.c2r(Xd).cpu().numpy()
    assert diag.rel_l2(back, f) <= TOL[dt]
    a, b = plan.parseval(x, Xd)
    assert abs(a - b) <= 10 * TOL[dt] * a


@pytest.mark.parametrize("shape", [(16, 24, 32), (96, 8, 12), (12, 128, 8), (48, 16, 192), (8, 8, 1024), (1024, 8, 8), (8, 768, 12)])
def test_fft_noncubic_batched(tk, shape):
    batch = 2
    f, X, G, g, plan, x, Xd = _run_pair(tk, shape, batch, "f32", seed=sum(shape))
    for b in range(batch):
        assert diag.rel_l2(X[b], offt.rfft3(f[b].astype(np.float64)), shape[2]) <= TOL["f32"]
        assert diag.rel_l2(g[b], offt.irfft3(G[b].astype(np.complex128), shape[2])) <= TOL["f32"]


@pytest.mark.parametrize("n", [256, 384, 512])
def test_fft_large_vs_oracle(tk, n):
    f, X, G, g, plan, x, Xd = _run_pair(tk, (n, n, n), 1, "f32", seed=0)
    ref = offt.rfft3(f[0].astype(np.float64))
    assert diag.rel_l2(X[0], ref, n) <= TOL["f32"]
    del ref
    gref = offt.irfft3(G[0].astype(np.complex128), n)
    assert diag.rel_l2(g[0], gref) <= TOL["f32"]


@pytest.mark.parametrize("n", [8, 12, 24, 48, 96, 192, 384, 768, 16, 32, 64, 128, 256, 512, 1024])
def test_every_tile_candidate_matches_oracle(tk, n):
    """The autotuner may only choose among candidates that all reproduce the oracle."""
    import torch
    shapes = {0: (8, 8, n), 1: (8, n, 8), 2: (n, 8, 8)}
    try:
        for p in range(3):
            shape = shapes[p]
            f = synth.gaussian_field((1,) + shape, n + p)
            ref = offt.rfft3(f[0].astype(np.float64))
            for (a, E, v) in tk.tile_candidates(n, torch.float32, p):
                tk.tune_set(n, torch.float32, p, a, E, v)
                plan = tk.FFT3D(*shape, dtype=torch.float32)
                assert f"E={E}" in plan.describe(p)
                X = plan.r2c(torch.from_numpy(f).cuda())
                assert diag.rel_l2(X.cpu().numpy()[0], ref, shape[2]) <= TOL["f32"], (p, a, E, v)
                back = plan.c2r(X).cpu().numpy()
                assert diag.rel_l2(back, f) <= TOL["f32"], (p, a, E, v)
                plan.close()
            tk.tune_set(n, torch.float32, p, 0, 0)
    finally:
        tk.tune_clear()


@pytest.mark.parametrize("L", [256, 512, 1024])
def test_persistent_candidates_full_rounds_and_tail(tk, L):
    """The persistent strided variants (all three tile orders, with one or two workgroups
    per CU) at sizes where every workgroup takes one or more full tiles and the leftover
    columns are cut into narrow tail tiles (ncols = 256 * 65, or 64 * 65 at 1024 points)."""
    import torch
    m = 256 if L < 1024 else 64
    try:
        for p, shape in ((1, (m, L, 128)), (2, (L, m, 128))):
            f = synth.gaussian_field((1,) + shape, 7 + p)
            ref = offt.rfft3(f[0].astype(np.float64))
            cands = [c for c in tk.tile_candidates(L, torch.float32, p) if c[2] in (1, 2, 3, 7, 8, 9)]
            assert cands, "no persistent candidate compiled for L=%d" % L
            x = torch.from_numpy(f).cuda()
            for (a, E, v) in cands:
                tk.tune_set(L, torch.float32, p, a, E, v)
                plan = tk.FFT3D(*shape, dtype=torch.float32)
                assert "v=%d" % v in plan.describe(p)
                X = plan.r2c(x)
                assert diag.rel_l2(X.cpu().numpy()[0], ref, shape[2]) <= TOL["f32"], (p, a, E)
                back = plan.c2r(X).cpu().numpy()
                assert diag.rel_l2(back, f) <= TOL["f32"], (p, a, E)
                plan.close()
            tk.tune_set(L, torch.float32, p, 0, 0)
    finally:
        tk.tune_clear()



def test_two_1024_members_split_per_plane(tk):
    """Two 1024^3 members in one plan: the X pass's per-thread offsets would exceed 32 bits
    across the members, so it runs once per member; every member's transform must equal the
    single-member plan's, bit for bit, both directions."""
    import torch
    n = 1024
    g = torch.Generator(device="cuda").manual_seed(11)
    x = torch.randn((2, n, n, n), generator=g, device="cuda", dtype=torch.float32)
    p2 = tk.FFT3D(n, batch=2, dtype=torch.float32)
    X2 = p2.r2c(x)
    p1 = tk.FFT3D(n, batch=1, dtype=torch.float32)
    for b in range(2):
        X1 = p1.r2c(x[b:b + 1].contiguous())
        assert torch.equal(X1, X2[b:b + 1]), b
        del X1
    y2 = p2.c2r(X2)
    for b in range(2):
        y1 = p1.c2r(X2[b:b + 1].contiguous())
        assert torch.equal(y1, y2[b:b + 1]), b
        del y1
    err = (torch.linalg.vector_norm((y2 - x).double()) / torch.linalg.vector_norm(x.double())).item()
    assert err <= TOL["f32"]
    p1.close()
    p2.close()


@pytest.mark.parametrize("shape,basis", [((64, 64, 64), (0, 0)), ((512, 512, 512), (0, 0)), ((48, 32, 24), (1, 2))])
def test_c2r_overwrite_equals_preserving_c2r(tk, shape, basis):
    """TK_FFT_C2R_OVERWRITE runs the same passes in place on the input: the real output
    equals the preserving plan's bit for bit."""
    import torch
    nx, ny, nz = shape
    g = torch.Generator(device="cuda").manual_seed(nx + ny)
    x = torch.randn((1, nx, ny, nz), generator=g, device="cuda", dtype=torch.float32)
    kw = {} if basis == (0, 0) else {"basis_x": basis[0], "basis_y": basis[1]}
    p0 = tk.FFT3D(nx, ny, nz, dtype=torch.float32, **kw)
    p1 = tk.FFT3D(nx, ny, nz, dtype=torch.float32, flags=tk.TK_FFT_C2R_OVERWRITE, **kw)
    X = p0.r2c(x)
    y0 = p0.c2r(X)
    Xc = X.clone()
    y1 = p1.c2r(Xc)
    assert torch.equal(y0, y1)
    assert not torch.equal(Xc, X)  # the input was used as workspace
    import ctypes
    sz = ctypes.c_size_t()
    assert tk.lib().fft3d_workspace_size(p1.h, ctypes.byref(sz)) == tk.TK_OK and sz.value == 0
    assert tk.lib().fft3d_workspace_size(p0.h, ctypes.byref(sz)) == tk.TK_OK and sz.value == X.numel() * 8
    p0.close()
    p1.close()
