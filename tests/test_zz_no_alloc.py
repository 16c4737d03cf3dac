"""The allocation-free c2r entry point (static device scratch as its workspace) against
the allocating one, through the C ABI: two calls in a row, the second on a smaller grid,
bit-identical to fft3d_c2r (same kernels) and within the FFT tolerance of the oracle; and
captured in a HIP graph, as the callers it is for use it."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import diag, fft as offt

pytestmark = pytest.mark.gpu


def _case(tk, n, batch, dtype, seed):
    import torch
    print("no-alloc c2r case n=%d batch=%d dtype=%s seed=%d" % (n, batch, dtype, seed), flush=True)
    plan = tk.FFT3D(n, batch=batch, dtype=dtype)
    f = synth.gaussian_field((batch, n, n, n), seed, dtype=np.float32 if dtype == torch.float32 else np.float64)
    X = plan.r2c(torch.from_numpy(f).cuda())
    X0 = X.clone()
    ref = plan.c2r(X)
    got = torch.full_like(ref, float("nan"))
    plan.c2r_noalloc(X, got)
    torch.cuda.synchronize()
    assert torch.equal(X, X0), "input not preserved"
    assert torch.equal(got, ref), "no-alloc c2r differs from fft3d_c2r"
    Xn = X.cpu().numpy()
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    for b in range(batch):
        g = offt.irfft3(Xn[b].astype(np.complex128), n)
        assert diag.rel_l2(got[b].cpu().numpy(), g) <= tol
    plan.close()


def test_noalloc_c2r_matches_allocating_c2r_twice(tk):
    import torch
    # the first call fills most of the scratch (256^3 FP32: 64.5 MiB), the second is smaller
    _case(tk, 256, 1, torch.float32, 31)
    _case(tk, 48, 2, torch.float64, 32)


def test_noalloc_c2r_rejects_a_workspace_beyond_the_scratch(tk):
    import torch
    plan = tk.FFT3D(256, batch=2, dtype=torch.float32)  # 129 MiB of workspace
    X = plan.empty_cplx()
    y = plan.empty_real()
    st = tk.lib().fft3d_c2r_noalloc(plan.h, tk._ptr(X), tk._ptr(y), tk._stream())
    assert st == tk.TK_EINVAL
    assert b"exceeds the static scratch" in tk.lib().tk_last_error()
    plan.close()
    # a plan that overwrites its input needs no workspace at any size
    plan = tk.FFT3D(256, batch=2, dtype=torch.float32, flags=tk.TK_FFT_C2R_OVERWRITE)
    f = synth.gaussian_field((2, 256, 256, 256), 33)
    x = torch.from_numpy(f).cuda()
    X = plan.r2c(x)
    y = torch.empty_like(x)
    plan.c2r_noalloc(X, y)
    torch.cuda.synchronize()
    assert diag.rel_l2(y.cpu().numpy(), f) <= 1e-5
    plan.close()


def test_noalloc_c2r_under_graph_capture(tk):
    """The callers this entry point is for: a HIP graph captured around it (and the r2c that
    feeds it), replayed several times with eager work and synchronisation between the
    replays; every replay equals the eager result bit for bit."""
    import torch
    n = 128
    print("no-alloc c2r under graph capture n=%d" % n, flush=True)
    plan = tk.FFT3D(n, dtype=torch.float32)
    x = torch.from_numpy(synth.gaussian_field((1, n, n, n), 34)).cuda()
    X = plan.empty_cplx()
    y = plan.empty_real()
    plan.r2c(x, X)
    plan.c2r_noalloc(X, y)  # eager: kernels loaded and the scratch address taken before capture
    torch.cuda.synchronize()
    ref = y.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.r2c(x, X)
        plan.c2r_noalloc(X, y)
    for k in range(3):
        y.fill_(float("nan"))
        X.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, ref), k
    assert diag.rel_l2(y.cpu().numpy(), x.cpu().numpy()) <= 1e-5
    plan.close()
