"""Python binding of libtk (MI355X / gfx950): argument marshalling over the C ABI in
include/tk.h.  Every step of the computation runs in libtk's HIP kernels; PyTorch only
provides device memory and streams.  There is no CPU fallback: if libtk.so is missing
or cannot be loaded, every call raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtk.so")

TK_OK, TK_EINVAL, TK_EUNSUPPORTED, TK_ENOMEM, TK_EHIP, TK_ESTATE = 0, -1, -2, -3, -4, -5
TK_F32, TK_F64 = 0, 1
TK_FFT_TIMING, TK_FFT_NO_TUNE, TK_FFT_C2R_Y_FIRST, TK_FFT_C2R_OVERWRITE = 0x1, 0x2, 0x4, 0x8
TK_SCRATCH_BYTES = 80 << 20

_lib = None


class TkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("tk status %d: %s" % (status, msg))
        self.status = status


class TkMlp(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("in_scale", ctypes.c_float), ("out_scale", ctypes.c_float)]


class TkAdam(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("m", ctypes.c_void_p), ("v", ctypes.c_void_p), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("step", ctypes.c_int)]


class RbcConfig(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("dtype", ctypes.c_int), ("Ra", ctypes.c_double), ("Pr", ctypes.c_double),
                ("box", ctypes.c_double), ("cfl", ctypes.c_double), ("flags", ctypes.c_uint)]


class NsConfig(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("dtype", ctypes.c_int), ("nu", ctypes.c_double), ("cfl", ctypes.c_double),
                ("scheme", ctypes.c_int), ("flags", ctypes.c_uint)]


def _declare(L):
    vp, i, u, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint, ctypes.c_double, ctypes.c_size_t
    P = ctypes.POINTER
    sigs = {
        "tk_last_error": ([], ctypes.c_char_p),
        "tk_version": ([], i),
        "tk_sum_squares": ([vp, ctypes.c_long, i, P(d), vp], i),
        "fft3d_plan_create": ([P(vp), i, i, i, i, i, u], i),
        "fft3d_plan_create_basis": ([P(vp), i, i, i, i, i, i, i, u], i),
        "fft3d_plan_create_basis3": ([P(vp), i, i, i, i, i, i, i, i, u], i),
        "fft3d_workspace_size": ([vp, P(sz)], i),
        "fft3d_set_workspace": ([vp, vp], i),
        "fft3d_r2c": ([vp, vp, vp, vp], i),
        "fft3d_c2r": ([vp, vp, vp, vp], i),
        "fft3d_c2r_noalloc": ([vp, vp, vp, vp], i),
        "fft3d_parseval": ([vp, vp, vp, P(d), vp], i),
        "fft3d_pass_times": ([vp, P(ctypes.c_float)], i),
        "fft3d_describe": ([vp, i, ctypes.c_char_p, i], i),
        "fft3d_plan_destroy": ([vp], i),
        "fft3d_autotune": ([i, i, i, i, i, i, ctypes.c_char_p, i], i),
        "fft3d_tune_set": ([i, i, i, i, i, i], i),
        "fft3d_tune_clear": ([], i),
        "ns_autotune": ([i, i, i, ctypes.c_char_p, i], i),
        "ns_batch_autotune": ([i, i, i, ctypes.c_char_p, i], i),
        "fft3d_tile_candidates": ([i, i, i, P(i), P(i), P(i), i], i),
        "ns_create": ([P(vp), P(NsConfig)], i),
        "ns_rhs": ([vp, vp, vp, vp], i),
        "ns_step": ([vp, vp, d, i, P(d), vp], i),
        "ns_diagnostics": ([vp, vp, P(d), P(d), P(d), i, P(d), vp], i),
        "ns_init_random": ([vp, vp, vp, d, vp], i),
        "ns_last_dt": ([vp, P(d)], i),
        "ns_pass_times": ([vp, vp, i, P(ctypes.c_float), vp], i),
        "ns_destroy": ([vp], i),
        "ns_energy_transfer": ([vp, vp, P(d), i, vp], i),
        "rbc_create": ([P(vp), P(RbcConfig)], i),
        "rbc_rhs": ([vp, vp, vp, vp], i),
        "rbc_step": ([vp, vp, d, i, P(d), vp], i),
        "rbc_diagnostics": ([vp, vp, P(d), P(d), P(d), P(d), vp], i),
        "rbc_last_dt": ([vp, P(d)], i),
        "rbc_pass_times": ([vp, vp, i, P(ctypes.c_float), vp], i),
        "rbc_destroy": ([vp], i),
        "ns_shell_to_shell": ([vp, vp, P(i), i, i, P(d), vp], i),
        "ns_batch_create": ([P(vp), i, P(i), P(d), i, d, u], i),
        "ns_batch_step": ([vp, P(vp), d, i, P(d), vp], i),
        "ns_batch_init_random": ([vp, i, vp, vp, d, vp], i),
        "ns_batch_diagnostics": ([vp, i, vp, P(d), P(d), P(d), vp], i),
        "ns_batch_last_dt": ([vp, P(d)], i),
        "ns_batch_destroy": ([vp], i),
        "sgs_mlp_forward": ([P(TkMlp), vp, vp, ctypes.c_long, vp], i),
        "sgs_mlp_backward": ([P(TkMlp), vp, vp, ctypes.c_long, vp, vp], i),
        "sgs_mlp_loss_grad": ([P(TkMlp), vp, vp, ctypes.c_long, vp, P(d), vp], i),
        "sgs_adam_step": ([P(TkAdam), vp, vp, vp], i),
        "sgs_weights_to_bf16": ([vp, vp, i, vp], i),
        "les_step": ([vp, P(TkMlp), vp, d, i, P(d), P(i), vp], i),
        "les_filter_dns": ([vp, i, i, i, vp, vp, vp, vp], i),
    }
    for name, (args, res) in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


def load(path=None):
    """Load libtk.so (built in-tree by build.py); raises if it is not there."""
    global _lib
    if _lib is None:
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise TkError(TK_ESTATE, "libtk.so not built (%s); run paper_1805_07801_amd/build.py" % p)
        _lib = _declare(ctypes.CDLL(p))
    return _lib


def lib():
    return load()


def check(status):
    if status != TK_OK:
        raise TkError(status, lib().tk_last_error().decode())
    return status


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dtype_code(dtype):
    import torch
    if dtype in (torch.float32, torch.complex64):
        return TK_F32
    if dtype in (torch.float64, torch.complex128):
        return TK_F64
    raise TkError(TK_EUNSUPPORTED, "dtype %s" % dtype)


def sum_squares(x, stream=None):
    """sum x_i^2 of a real GPU tensor, FP64 accumulation in the library."""
    out = ctypes.c_double()
    check(lib().tk_sum_squares(_ptr(x), x.numel(), _dtype_code(x.dtype), ctypes.byref(out), _stream(stream)))
    return out.value


def autotune(nx, ny=None, nz=None, batch=1, dtype=None, iters=5):
    """Time every tile candidate of each pass on this GPU and keep the fastest one that
    matches the default tile (see fft3d_autotune).  Returns the text report."""
    import torch
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    buf = ctypes.create_string_buffer(1 << 16)
    check(lib().fft3d_autotune(nx, ny, nz, batch, _dtype_code(dtype or torch.float32), iters, buf, 1 << 16))
    return buf.value.decode()


def ns_autotune(n, iters=5, dtype=None):
    """Time every compiled variant of the solver passes P1, P2 / P4, P3, P5 and the fused
    P5 + P1 of an n^3 grid and record the fastest one that matches the reference (see
    ns_autotune).  Returns the text report."""
    import torch
    buf = ctypes.create_string_buffer(1 << 14)
    check(lib().ns_autotune(n, _dtype_code(dtype or torch.float32), iters, buf, 1 << 14))
    return buf.value.decode()


def ns_batch_autotune(n, members=16, iters=5):
    """Time every compiled thread count and persistent grid of the ensemble kernels of grid
    size n and record the fastest that matches the default shape (see ns_batch_autotune).
    Returns the text report."""
    buf = ctypes.create_string_buffer(1 << 14)
    check(lib().ns_batch_autotune(n, members, iters, buf, 1 << 14))
    return buf.value.decode()


def tile_candidates(L, dtype, pass_):
    """[(a, E, v)] compiled tile candidates of (L, dtype, pass): pass 0 = Z (a = threads),
    1 = Y and 2 = X (a = columns per tile), v = the strided kernel variant (see
    fft3d_tune_set); passes 3, 4, 5 = solver P1, P3, P5 of an L^3 grid, 6 = its Y passes,
    7 = the fused P5 + P1."""
    code = _dtype_code(dtype)
    n = lib().fft3d_tile_candidates(L, code, pass_, None, None, None, 0)
    a = (ctypes.c_int * max(n, 1))()
    e = (ctypes.c_int * max(n, 1))()
    v = (ctypes.c_int * max(n, 1))()
    lib().fft3d_tile_candidates(L, code, pass_, a, e, v, n)
    return [(a[i], e[i], v[i]) for i in range(n)]


def tune_set(L, dtype, pass_, a, E, v=0):
    check(lib().fft3d_tune_set(L, _dtype_code(dtype), pass_, a, E, v))


def tune_clear():
    check(lib().fft3d_tune_clear())


def tune_save(path, entries):
    """Persist tuned tiles [(L, dtype_code, pass, a, E, v)] as JSON lines."""
    import json
    with open(path, "w") as f:
        for L, dt, p, a, E, v in entries:
            f.write(json.dumps({"L": L, "dtype": dt, "pass": p, "a": a, "E": E, "v": v}) + "\n")


def tune_load(path):
    """Apply tuned tiles saved by tune_save; returns how many were applied."""
    import json
    n = 0
    with open(path) as f:
        for line in f:
            if line.strip():
                e = json.loads(line)
                check(lib().fft3d_tune_set(e["L"], e["dtype"], e["pass"], e["a"], e["E"], e.get("v", 0)))
                n += 1
    return n


class FFT3D:
    """Plan for batched 3D r2c / c2r transforms of [batch][nx][ny][nz] real fields."""

    def __init__(self, nx, ny=None, nz=None, batch=1, dtype=None, flags=0, basis_x=0, basis_y=0, basis_z=0):
        """basis_x / basis_y / basis_z: 0 Fourier, 1 sine, 2 cosine.  A sine / cosine z basis
        (the SSS family) needs sine / cosine x and y bases; its spectral data are real
        [batch][nx][ny][nz]."""
        import torch
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        dtype = dtype or torch.float32
        self.shape = (nx, ny, nz)
        self.batch = batch
        self.dtype = dtype
        self.sss = basis_z != 0
        if self.sss:
            self.cdtype = dtype
        else:
            self.cdtype = torch.complex64 if _dtype_code(dtype) == TK_F32 else torch.complex128
        h = ctypes.c_void_p()
        if basis_z:
            check(lib().fft3d_plan_create_basis3(ctypes.byref(h), nx, ny, nz, batch, _dtype_code(dtype), basis_x,
                                                 basis_y, basis_z, flags))
        elif basis_x or basis_y:
            check(lib().fft3d_plan_create_basis(ctypes.byref(h), nx, ny, nz, batch, _dtype_code(dtype), basis_x,
                                                basis_y, flags))
        else:
            check(lib().fft3d_plan_create(ctypes.byref(h), nx, ny, nz, batch, _dtype_code(dtype), flags))
        self.h = h

    def spectral_shape(self):
        nx, ny, nz = self.shape
        return (self.batch, nx, ny, nz) if self.sss else (self.batch, nx, ny, nz // 2 + 1)

    def _check_real(self, t):
        nx, ny, nz = self.shape
        if t.dtype != self.dtype or not t.is_cuda or not t.is_contiguous() or t.numel() != self.batch * nx * ny * nz:
            raise TkError(TK_EINVAL, "real tensor must be contiguous %s on GPU with %d elements"
                          % (self.dtype, self.batch * nx * ny * nz))

    def _check_cplx(self, t):
        n = 1
        for d in self.spectral_shape():
            n *= d
        if t.dtype != self.cdtype or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
            raise TkError(TK_EINVAL, "spectral tensor must be contiguous %s on GPU with %d elements" % (self.cdtype, n))

    def empty_cplx(self):
        import torch
        return torch.empty(self.spectral_shape(), dtype=self.cdtype, device="cuda")

    def empty_real(self):
        import torch
        return torch.empty((self.batch,) + self.shape, dtype=self.dtype, device="cuda")

    def r2c(self, real, out=None, stream=None):
        self._check_real(real)
        out = self.empty_cplx() if out is None else out
        self._check_cplx(out)
        check(lib().fft3d_r2c(self.h, _ptr(real), _ptr(out), _stream(stream)))
        return out

    def c2r(self, cplx, out=None, stream=None):
        self._check_cplx(cplx)
        out = self.empty_real() if out is None else out
        self._check_real(out)
        check(lib().fft3d_c2r(self.h, _ptr(cplx), _ptr(out), _stream(stream)))
        return out

    def c2r_noalloc(self, cplx, out, stream=None):
        """c2r through the allocation-free entry point (static device scratch as the
        workspace); `out` must be given."""
        self._check_cplx(cplx)
        self._check_real(out)
        check(lib().fft3d_c2r_noalloc(self.h, _ptr(cplx), _ptr(out), _stream(stream)))
        return out

    def parseval(self, real, cplx, stream=None):
        out = (ctypes.c_double * 2)()
        check(lib().fft3d_parseval(self.h, _ptr(real), _ptr(cplx), out, _stream(stream)))
        return out[0], out[1]

    def pass_times(self):
        t = (ctypes.c_float * 6)()
        check(lib().fft3d_pass_times(self.h, t))
        return list(t)

    def describe(self, p):
        buf = ctypes.create_string_buffer(256)
        check(lib().fft3d_describe(self.h, p, buf, 256))
        return buf.value.decode()

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            lib().fft3d_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def num_shells(n):
    """Shells 0..S-1 cover every stored mode: S = floor(sqrt(3) n / 2) + 2."""
    return int(0.8660254037844386 * n) + 2


class NS:
    """Pseudo-spectral Navier-Stokes solver on an n^3 periodic grid (state u^ of shape
    [3][n][n][n/2+1], complex, on the GPU)."""

    def __init__(self, n, dtype=None, nu=0.0, cfl=0.0, scheme="rk2"):
        import torch
        dtype = dtype or torch.float32
        self.n = n
        self.dtype = dtype
        self.cdtype = torch.complex64 if _dtype_code(dtype) == TK_F32 else torch.complex128
        self.nu = nu
        cfg = NsConfig(n, _dtype_code(dtype), float(nu), float(cfl), {"rk2": 0, "rk4": 1}[scheme], 0)
        h = ctypes.c_void_p()
        check(lib().ns_create(ctypes.byref(h), ctypes.byref(cfg)))
        self.h = h

    def _check_state(self, t):
        n = self.n
        if t.dtype != self.cdtype or not t.is_cuda or not t.is_contiguous() or t.numel() != 3 * n * n * (n // 2 + 1):
            raise TkError(TK_EINVAL, "state must be a contiguous %s GPU tensor [3][n][n][n/2+1]" % self.cdtype)

    def empty_state(self):
        import torch
        n = self.n
        return torch.zeros((3, n, n, n // 2 + 1), dtype=self.cdtype, device="cuda")

    def rhs(self, u, out=None, stream=None):
        self._check_state(u)
        out = self.empty_state() if out is None else out
        self._check_state(out)
        check(lib().ns_rhs(self.h, _ptr(u), _ptr(out), _stream(stream)))
        return out

    def step(self, u, dt, nsteps=1, t=0.0, stream=None):
        """Advance u in place; returns the new time."""
        self._check_state(u)
        tt = ctypes.c_double(t)
        check(lib().ns_step(self.h, _ptr(u), float(dt), int(nsteps), ctypes.byref(tt), _stream(stream)))
        return tt.value

    def last_dt(self):
        d = ctypes.c_double()
        check(lib().ns_last_dt(self.h, ctypes.byref(d)))
        return d.value

    def pass_times(self, u, iters=5, stream=None):
        """Mean ms per pass of one right-hand side of u: P1, P2, P3, P4, P5 and the time
        stepper's fused P5+P1 (see ns_pass_times)."""
        self._check_state(u)
        t = (ctypes.c_float * 6)()
        check(lib().ns_pass_times(self.h, _ptr(u), int(iters), t, _stream(stream)))
        return dict(zip(["P1", "P2", "P3", "P4", "P5", "P5+P1"], [t[i] for i in range(6)]))

    def diagnostics(self, u, nshell=None, stream=None):
        self._check_state(u)
        nshell = num_shells(self.n) if nshell is None else nshell
        e, eps, md = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        spec = (ctypes.c_double * max(nshell, 1))()
        check(lib().ns_diagnostics(self.h, _ptr(u), ctypes.byref(e), ctypes.byref(eps), spec, nshell,
                                   ctypes.byref(md), _stream(stream)))
        return {"energy": e.value, "dissipation": eps.value, "max_div": md.value,
                "spectrum": [spec[i] for i in range(nshell)]}

    def energy_transfer(self, u, nshell=None, stream=None):
        """T(s) per integer shell (FP64); flux = -cumsum(T)."""
        self._check_state(u)
        nshell = num_shells(self.n) if nshell is None else nshell
        T = (ctypes.c_double * nshell)()
        check(lib().ns_energy_transfer(self.h, _ptr(u), T, nshell, _stream(stream)))
        return [T[i] for i in range(nshell)]

    def shell_to_shell(self, u, band_of_shell, nbands, stream=None):
        """[receiver][giver] transfer matrix between bands of integer shells."""
        self._check_state(u)
        ns_ = len(band_of_shell)
        b = (ctypes.c_int * ns_)(*[int(v) for v in band_of_shell])
        T = (ctypes.c_double * (nbands * nbands))()
        check(lib().ns_shell_to_shell(self.h, _ptr(u), b, ns_, nbands, T, _stream(stream)))
        return [[T[r * nbands + m] for m in range(nbands)] for r in range(nbands)]

    def init_random(self, noise, energy=1.0, out=None, stream=None):
        """Random solenoidal state from real noise [3][n][n][n] (see ns_init_random)."""
        n = self.n
        if noise.dtype != self.dtype or not noise.is_cuda or not noise.is_contiguous() or noise.numel() != 3 * n ** 3:
            raise TkError(TK_EINVAL, "noise must be a contiguous %s GPU tensor [3][n][n][n]" % self.dtype)
        out = self.empty_state() if out is None else out
        self._check_state(out)
        check(lib().ns_init_random(self.h, _ptr(noise), _ptr(out), float(energy), _stream(stream)))
        return out

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            lib().ns_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ensemble:
    """Independent FP32 solves of mixed grid sizes advanced together (ns_batch_*): one
    persistent kernel per pass over all members, one HIP-graph launch per step."""

    def __init__(self, sizes, nus, cfl=0.0, grid=0):
        import torch
        self.sizes = list(sizes)
        self.count = len(self.sizes)
        n = (ctypes.c_int * self.count)(*self.sizes)
        nu = (ctypes.c_double * self.count)(*[float(v) for v in nus])
        self.nus = [float(v) for v in nus]
        h = ctypes.c_void_p()
        check(lib().ns_batch_create(ctypes.byref(h), self.count, n, nu, TK_F32, float(cfl), int(grid) << 16))
        self.h = h
        self.t = [0.0] * self.count

    def empty_state(self, i):
        import torch
        n = self.sizes[i]
        return torch.zeros((3, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")

    def init_random(self, i, noise, energy=1.0, out=None, stream=None):
        out = self.empty_state(i) if out is None else out
        check(lib().ns_batch_init_random(self.h, i, _ptr(noise), _ptr(out), float(energy), _stream(stream)))
        return out

    def step(self, states, dt=0.0, nsteps=1, stream=None):
        """Advance every member state (list of tensors) in place; returns member times."""
        import torch
        if len(states) != self.count:
            raise TkError(TK_EINVAL, "need %d states" % self.count)
        for i, u in enumerate(states):
            n = self.sizes[i]
            if u.dtype != torch.complex64 or not u.is_cuda or not u.is_contiguous() or u.numel() != 3 * n * n * (n // 2 + 1):
                raise TkError(TK_EINVAL, "member %d state has the wrong shape/dtype" % i)
        ptrs = (ctypes.c_void_p * self.count)(*[u.data_ptr() for u in states])
        t = (ctypes.c_double * self.count)(*self.t)
        check(lib().ns_batch_step(self.h, ptrs, float(dt), int(nsteps), t, _stream(stream)))
        self.t = list(t)
        return self.t

    def last_dt(self):
        d = (ctypes.c_double * self.count)()
        check(lib().ns_batch_last_dt(self.h, d))
        return list(d)

    def diagnostics(self, i, u, stream=None):
        e, eps, md = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        check(lib().ns_batch_diagnostics(self.h, i, _ptr(u), ctypes.byref(e), ctypes.byref(eps), ctypes.byref(md),
                                         _stream(stream)))
        return {"energy": e.value, "dissipation": eps.value, "max_div": md.value}

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            lib().ns_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MLP_NPARAM = 5190


class Closure:
    """Pointwise sub-grid stress network (BF16 parameters on the GPU, FP32 master copy and
    Adam moments) with its input/output scales."""

    def __init__(self, theta, in_scale=1.0, out_scale=1.0, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        import torch
        th = torch.as_tensor(theta, dtype=torch.float32).reshape(-1)
        if th.numel() != MLP_NPARAM:
            raise TkError(TK_EINVAL, "need %d parameters" % MLP_NPARAM)
        self.w32 = th.cuda().contiguous()
        self.m = torch.zeros_like(self.w32)
        self.v = torch.zeros_like(self.w32)
        self.wb = torch.empty(MLP_NPARAM, dtype=torch.int16, device="cuda")
        check(lib().sgs_weights_to_bf16(_ptr(self.w32), _ptr(self.wb), MLP_NPARAM, _stream()))
        self.grad = torch.zeros(MLP_NPARAM, dtype=torch.float32, device="cuda")
        self.in_scale = float(in_scale)
        self.out_scale = float(out_scale)
        self.opt = TkAdam(self.w32.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), lr, beta1, beta2, eps, 0)

    def desc(self):
        return TkMlp(self.wb.data_ptr(), self.in_scale, self.out_scale)

    def bf16_bits(self):
        return self.wb.cpu().numpy().view("uint16")

    def forward(self, x9, out=None):
        import torch
        M = x9.shape[-1]
        out = torch.empty((6, M), dtype=torch.float32, device="cuda") if out is None else out
        d = self.desc()
        check(lib().sgs_mlp_forward(ctypes.byref(d), _ptr(x9), _ptr(out), M, _stream()))
        return out

    def backward(self, x9, dy6):
        d = self.desc()
        check(lib().sgs_mlp_backward(ctypes.byref(d), _ptr(x9), _ptr(dy6), x9.shape[-1], _ptr(self.grad), _stream()))
        return self.grad

    def loss_grad(self, x9, t6):
        d = self.desc()
        loss = ctypes.c_double()
        check(lib().sgs_mlp_loss_grad(ctypes.byref(d), _ptr(x9), _ptr(t6), x9.shape[-1], _ptr(self.grad),
                                      ctypes.byref(loss), _stream()))
        return loss.value

    def adam_step(self):
        check(lib().sgs_adam_step(ctypes.byref(self.opt), _ptr(self.grad), _ptr(self.wb), _stream()))


def les_filter_dns(uhat_dns, n_les, kc, with_ubar=False):
    """(grad9 [9][M], tau6 [6][M], ubar_hat or None) for the box filter |k_i| <= kc."""
    import torch
    n = uhat_dns.shape[-3]
    M = n_les ** 3
    g = torch.empty((9, M), dtype=torch.float32, device="cuda")
    t = torch.empty((6, M), dtype=torch.float32, device="cuda")
    ub = torch.empty((3, n_les, n_les, n_les // 2 + 1), dtype=torch.complex64, device="cuda") if with_ubar else None
    check(lib().les_filter_dns(_ptr(uhat_dns), n, n_les, kc, _ptr(g), _ptr(t), _ptr(ub), _stream()))
    return g, t, ub


def les_step(ns, closure, u, dt, nsteps=1, t=0.0):
    """LES steps with the closure (None: plain right-hand side).  Returns (t, fallback)."""
    tt = ctypes.c_double(t)
    fb = ctypes.c_int(-1)
    d = closure.desc() if closure is not None else None
    check(lib().les_step(ns.h, ctypes.byref(d) if d is not None else None, _ptr(u), float(dt), int(nsteps),
                         ctypes.byref(tt), ctypes.byref(fb), _stream()))
    return tt.value, fb.value


class RBC:
    """Boussinesq convection in the periodic FFF basis; state [4][n][n][n/2+1] (u, theta)."""

    def __init__(self, n, Ra, Pr=1.0, box=1.0, dtype=None, cfl=0.0):
        import torch
        dtype = dtype or torch.float32
        self.n = n
        self.dtype = dtype
        self.cdtype = torch.complex64 if _dtype_code(dtype) == TK_F32 else torch.complex128
        cfg = RbcConfig(n, _dtype_code(dtype), float(Ra), float(Pr), float(box), float(cfl), 0)
        h = ctypes.c_void_p()
        check(lib().rbc_create(ctypes.byref(h), ctypes.byref(cfg)))
        self.h = h

    def _check(self, t):
        n = self.n
        if t.dtype != self.cdtype or not t.is_cuda or not t.is_contiguous() or t.numel() != 4 * n * n * (n // 2 + 1):
            raise TkError(TK_EINVAL, "state must be a contiguous %s GPU tensor [4][n][n][n/2+1]" % self.cdtype)

    def rhs(self, s4, out=None, stream=None):
        import torch
        self._check(s4)
        out = torch.empty_like(s4) if out is None else out
        check(lib().rbc_rhs(self.h, _ptr(s4), _ptr(out), _stream(stream)))
        return out

    def step(self, s4, dt, nsteps=1, t=0.0, stream=None):
        self._check(s4)
        tt = ctypes.c_double(t)
        check(lib().rbc_step(self.h, _ptr(s4), float(dt), int(nsteps), ctypes.byref(tt), _stream(stream)))
        return tt.value

    def diagnostics(self, s4, stream=None):
        self._check(s4)
        v = [ctypes.c_double() for _ in range(4)]
        check(lib().rbc_diagnostics(self.h, _ptr(s4), *[ctypes.byref(x) for x in v], _stream(stream)))
        return {"kinetic": v[0].value, "thermal": v[1].value, "uz_theta": v[2].value, "nusselt": v[3].value}

    def pass_times(self, s4, iters=5, stream=None):
        """Mean ms of the right-hand side's passes P1..P5 (see rbc_pass_times)."""
        self._check(s4)
        t = (ctypes.c_float * 5)()
        check(lib().rbc_pass_times(self.h, _ptr(s4), iters, t, _stream(stream)))
        return dict(zip(["P1", "P2", "P3", "P4", "P5"], list(t)))

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            lib().rbc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
