"""C-ABI checks that need no GPU: the library loads, exports every symbol tk.h declares,
and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_1805_07801_amd as tk
    if not os.path.exists(tk.LIB_PATH):
        from paper_1805_07801_amd import build
        build.build(force=False)
    return tk.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "fft3d_r2c" in names and "ns_step" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_error_text(lib):
    assert lib.tk_version() >= 10000
    assert isinstance(lib.tk_last_error(), bytes)


@pytest.mark.parametrize("n", [0, 7, 10, 2048, 9, 6, 1536])
def test_plan_rejects_unsupported_sizes(lib, n):
    import paper_1805_07801_amd as tk
    h = ctypes.c_void_p()
    st = lib.fft3d_plan_create(ctypes.byref(h), n, 16, 16, 1, tk.TK_F32, 0)
    assert st == tk.TK_EUNSUPPORTED
    assert h.value is None
    assert b"unsupported" in lib.tk_last_error()


def test_plan_rejects_bad_arguments(lib):
    import paper_1805_07801_amd as tk
    h = ctypes.c_void_p()
    assert lib.fft3d_plan_create(None, 16, 16, 16, 1, tk.TK_F32, 0) == tk.TK_EINVAL
    assert lib.fft3d_plan_create(ctypes.byref(h), 16, 16, 16, 0, tk.TK_F32, 0) == tk.TK_EINVAL
    assert lib.fft3d_plan_create(ctypes.byref(h), 16, 16, 16, 1, 7, 0) == tk.TK_EUNSUPPORTED
    assert lib.fft3d_r2c(None, None, None, None) == tk.TK_EINVAL
    assert lib.fft3d_plan_destroy(None) == tk.TK_OK


def test_solver_entry_points_reject_null_handles(lib):
    import paper_1805_07801_amd as tk
    t = (ctypes.c_float * 6)()
    assert lib.ns_pass_times(None, None, 1, t, None) == tk.TK_EINVAL
    assert lib.ns_step(None, None, 0.1, 1, None, None) == tk.TK_EINVAL
    assert lib.ns_rhs(None, None, None, None) == tk.TK_EINVAL
    assert lib.ns_destroy(None) == tk.TK_OK


def test_plan_rejects_unknown_and_conflicting_flags(lib):
    import paper_1805_07801_amd as tk
    h = ctypes.c_void_p()
    assert lib.fft3d_plan_create(ctypes.byref(h), 16, 16, 16, 1, tk.TK_F32, 0x100) == tk.TK_EINVAL
    assert b"unknown plan flags" in lib.tk_last_error()
    both = tk.TK_FFT_C2R_Y_FIRST | tk.TK_FFT_C2R_OVERWRITE
    assert lib.fft3d_plan_create(ctypes.byref(h), 16, 16, 16, 1, tk.TK_F32, both) == tk.TK_EINVAL
    assert h.value is None


def test_newer_entry_points_reject_bad_arguments(lib):
    """Argument checks that come before any device call: the allocation-free inverse, the
    convection solver, ensembles, the closure network, Adam and the LES step."""
    import paper_1805_07801_amd as tk
    assert lib.fft3d_c2r_noalloc(None, None, None, None) == tk.TK_EINVAL
    assert lib.rbc_step(None, None, 0.1, 1, None, None) == tk.TK_EINVAL
    assert lib.rbc_destroy(None) == tk.TK_OK
    assert lib.ns_batch_step(None, None, 0.1, 1, None, None) == tk.TK_EINVAL
    assert lib.ns_batch_destroy(None) == tk.TK_OK
    assert lib.sgs_mlp_forward(None, None, None, 1, None) == tk.TK_EINVAL
    assert lib.sgs_adam_step(None, None, None, None) == tk.TK_EINVAL
    w = tk.TkMlp()  # NULL weights
    assert lib.sgs_mlp_forward(ctypes.byref(w), None, None, 1, None) == tk.TK_EINVAL
    assert lib.les_step(None, None, None, 0.1, 1, None, None, None) == tk.TK_EINVAL


def test_tile_table_on_the_host(lib):
    """The tile registry answers without a device: every candidate of a pass can be set, the
    persistent strided variants with one and with two workgroups per CU are among the
    512-point ones, and a tile that is not compiled is refused."""
    import paper_1805_07801_amd as tk
    n = lib.fft3d_tile_candidates(512, tk.TK_F32, 1, None, None, None, 0)
    assert n > 10
    a, e, v = (ctypes.c_int * n)(), (ctypes.c_int * n)(), (ctypes.c_int * n)()
    assert lib.fft3d_tile_candidates(512, tk.TK_F32, 1, a, e, v, n) == n
    variants = set(v)
    assert {0, 2, 4, 6, 8} <= variants
    try:
        for i in range(n):
            assert lib.fft3d_tune_set(512, tk.TK_F32, 1, a[i], e[i], v[i]) == tk.TK_OK
        assert lib.fft3d_tune_set(512, tk.TK_F32, 1, 3, 8, 0) == tk.TK_EUNSUPPORTED
    finally:
        lib.fft3d_tune_clear()
