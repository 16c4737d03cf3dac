// 3D FFT plans: pass selection and the r2c / c2r pass sequences.
//
// Forward (paper, Section "Parallelization Strategy", steps 1-5 on one device):
//   Z r2c  real_in -> cplx_out ;  Y c2c in place ;  X c2c in place with 1/(nx ny nz).
// The two all-to-all exchanges of the pencil algorithm have no counterpart: the layout
// is never permuted (Appendix A), the Y and X passes read strided columns.
// Inverse: X c2c^-1 cplx_in -> workspace ; Y c2c^-1 in place ; Z c2r workspace -> real_out.
#include <cstring>
#include <mutex>
#include <new>

#include "fft_api.hpp"
#include "reduce.hpp"
#include "tune.hpp"

namespace tk {

// Default tile: the widest W (longest contiguous runs) whose LDS tile still lets two
// workgroups share a CU; ties go to fewer threads.
const StridedKernel *pick_strided(int L, tk_dtype dt, int want_W, int want_E, int want_v) {
    const StridedKernel *best = nullptr;
    for (const auto &k : strided_kernels()) {
        if (k.L != L || k.dt != dt) continue;
        if (want_W > 0) {
            if (k.W == want_W && k.E == want_E && k.var == want_v) return &k;
            continue;
        }
        if (k.var != 0) continue;
        auto score = [](const StridedKernel &q) { return (q.lds <= 81920 ? 100000 : 0) + q.W * 10 - q.nt / 256; };
        if (!best || score(k) > score(*best)) best = &k;
    }
    return best;
}

const ZKernel *pick_z(int N, tk_dtype dt, int want_nt, int want_E) {
    const ZKernel *best = nullptr;
    for (const auto &k : z_kernels()) {
        if (k.N != N || k.dt != dt) continue;
        if (want_nt > 0) {
            if (k.nt == want_nt && k.E == want_E) return &k;
            continue;
        }
        if (!best || std::abs(k.nt - 256) + k.E < std::abs(best->nt - 256) + best->E) best = &k;
    }
    return best;
}

// The strided kernels address a tile's points as a 64-bit base shared by the workgroup
// plus a 32-bit byte offset per thread, which spans the planes of SO elements a tile
// touches and TPL rows of SI.  When that exceeds 32 bits (several 1024^3 members in one
// call) the pass is launched once per plane, where a tile never crosses a plane.
tk_status strided_pass(const StridedKernel *k, const void *src, void *dst, long ncols, long CB, long SO,
                       long SI, const void *tw, int inv, double scale, hipStream_t s, int rev) {
    const long esz = k->dt == TK_F32 ? 8 : 16;
    const long in_plane = (CB + (long)(k->L / k->E) * SI) * esz;
    const long crossing = ((k->W + CB - 2) / CB) * SO * esz;
    const long lim = 1L << 32;
    if (in_plane + crossing < lim) {
        StridedArgs a{src, dst, ncols, CB, SO, SI, tw, inv, scale, -1, -1, rev};
        k->fn(a, s);
        return launch_check("strided pass");
    }
    if (in_plane >= lim) return fail(TK_EUNSUPPORTED, "strided pass: a plane spans more than 4 GB");
    for (long p = 0; p < ncols / CB; ++p) {
        const long q = rev ? ncols / CB - 1 - p : p;
        StridedArgs a{(const char *)src + q * SO * esz, (char *)dst + q * SO * esz, CB, CB, SO, SI, tw, inv, scale,
                      -1, -1, rev};
        k->fn(a, s);
    }
    return launch_check("strided pass");
}

static tk_status r2r_pass(const R2RKernel *k, int basis, const void *src, void *dst, long ncols, long CB, long SO,
                          long SI, const void *tw, const void *twq, int inv, double scale, hipStream_t s) {
    // kind: 0 DCT-II, 1 DST-II, 2 DCT-III, 3 DST-III
    const int kind = (inv ? 2 : 0) + (basis == 1 ? 1 : 0);
    R2RArgs a{src, dst, ncols, CB, SO, SI, tw, twq, kind, scale};
    k->fn(a, s);
    return launch_check("sine/cosine pass");
}

tk_status fft_y_pass(const FftAxes &ax, const void *src, void *dst, long nfields, int inv, hipStream_t s, int rev) {
    const long nzh = ax.nz / 2 + 1;
    if (ax.by != 0)
        return r2r_pass(ax.ry, ax.by, src, dst, nfields * ax.nx * nzh, nzh, (long)ax.ny * nzh, nzh, ax.twy, ax.twqy,
                        inv, 1.0, s);
    return strided_pass(ax.ky, src, dst, nfields * ax.nx * nzh, nzh, (long)ax.ny * nzh, nzh, ax.twy, inv, 1.0, s,
                        rev);
}

tk_status fft_x_pass(const FftAxes &ax, const void *src, void *dst, long nfields, int inv, double scale,
                     hipStream_t s, int rev) {
    const long nzh = ax.nz / 2 + 1;
    const long cb = (long)ax.ny * nzh;
    if (ax.bx != 0)
        return r2r_pass(ax.rx, ax.bx, src, dst, nfields * cb, cb, (long)ax.nx * cb, cb, ax.twx, ax.twqx, inv, scale,
                        s);
    return strided_pass(ax.kx, src, dst, nfields * cb, cb, (long)ax.nx * cb, cb, ax.twx, inv, scale, s, rev);
}

tk_status axes_set_basis(FftAxes *ax, int bx, int by, int bz) {
    if (bx < 0 || bx > 2 || by < 0 || by > 2 || bz < 0 || bz > 2)
        return fail(TK_EINVAL, "basis must be 0 (Fourier), 1 (sine), 2 (cosine)");
    if (bz != 0 && (bx == 0 || by == 0))
        return fail(TK_EUNSUPPORTED, "a sine / cosine z basis needs sine / cosine x and y bases (SSS family)");
    ax->bx = bx;
    ax->by = by;
    ax->bz = bz;
    tk_status st;
    for (int axis = 0; axis < 2; ++axis) {
        const int b = axis == 0 ? bx : by;
        if (!b) continue;
        const int L = axis == 0 ? ax->nx : ax->ny;
        const R2RKernel *k = nullptr;
        for (const auto &q : r2r_kernels())
            if (q.L == L && q.dt == ax->dt) k = &q;
        if (!k) return fail(TK_EUNSUPPORTED, "no sine/cosine kernel for length %d", L);
        const void *tq = twiddle_table(4 * L, ax->dt, &st);
        if (!tq) return st;
        if (axis == 0) {
            ax->rx = k;
            ax->twqx = tq;
        } else {
            ax->ry = k;
            ax->twqy = tq;
        }
    }
    if (bz) {
        for (const auto &q : z_r2r_kernels())
            if (q.L == ax->nz && q.dt == ax->dt) ax->rz = &q;
        if (!ax->rz) return fail(TK_EUNSUPPORTED, "no z sine/cosine kernel for length %d", ax->nz);
        ax->twqz = twiddle_table(4 * ax->nz, ax->dt, &st);
        if (!ax->twqz) return st;
    }
    return TK_OK;
}

// SSS family: kinds 0 DCT-II, 1 DST-II, 2 DCT-III, 3 DST-III (as the strided sine/cosine pass)
tk_status sss_z_pass(const FftAxes &ax, const void *src, void *dst, long nfields, int inv, hipStream_t s) {
    ZR2RArgs a{src, dst, nfields * ax.nx * ax.ny / 2, ax.twz, ax.twqz, (inv ? 2 : 0) + (ax.bz == 1 ? 1 : 0), 1.0};
    ax.rz->fn(a, s);
    return launch_check("z sine/cosine pass");
}

tk_status sss_y_pass(const FftAxes &ax, const void *src, void *dst, long nfields, int inv, hipStream_t s) {
    const long nzc = ax.nz / 2;  // complex pairs along z
    return r2r_pass(ax.ry, ax.by, src, dst, nfields * ax.nx * nzc, nzc, (long)ax.ny * nzc, nzc, ax.twy, ax.twqy,
                    inv, 1.0, s);
}

tk_status sss_x_pass(const FftAxes &ax, const void *src, void *dst, long nfields, int inv, double scale,
                     hipStream_t s) {
    const long cb = (long)ax.ny * (ax.nz / 2);
    return r2r_pass(ax.rx, ax.bx, src, dst, nfields * cb, cb, (long)ax.nx * cb, cb, ax.twx, ax.twqx, inv, scale, s);
}

tk_status fft_z_r2c(const FftAxes &ax, const void *src, void *dst, long nfields, double scale, hipStream_t s,
                    int rev) {
    ZArgs a{src, dst, nfields * ax.nx * ax.ny, ax.twz, scale, rev};
    ax.kz->r2c(a, s);
    return launch_check("z r2c pass");
}

tk_status fft_z_c2r(const FftAxes &ax, const void *src, void *dst, long nfields, hipStream_t s, int rev) {
    ZArgs a{src, dst, nfields * ax.nx * ax.ny, ax.twz, 1.0, rev};
    ax.kz->c2r(a, s);
    return launch_check("z c2r pass");
}

tk_status axes_init(FftAxes *ax, int nx, int ny, int nz, tk_dtype dt, bool use_tune) {
    if (!supported_len(nx) || !supported_len(ny) || !supported_len(nz))
        return fail(TK_EUNSUPPORTED, "unsupported size %dx%dx%d (need 2^a or 3*2^a in [8,1024])", nx, ny, nz);
    if (dt != TK_F32 && dt != TK_F64) return fail(TK_EUNSUPPORTED, "unsupported dtype %d", (int)dt);
    ax->nx = nx;
    ax->ny = ny;
    ax->nz = nz;
    ax->dt = dt;
    tk_status st;
    ax->twx = twiddle_table(nx, dt, &st);
    if (!ax->twx) return st;
    ax->twy = twiddle_table(ny, dt, &st);
    if (!ax->twy) return st;
    ax->twz = twiddle_table(nz, dt, &st);
    if (!ax->twz) return st;
    TileChoice ty{}, tx{}, tz{};
    if (use_tune) {
        ty = tuned_tile(ny, dt, 1);
        tx = tuned_tile(nx, dt, 2);
        tz = tuned_tile(nz, dt, 0);
    }
    ax->ky = pick_strided(ny, dt, ty.a, ty.E, ty.v);
    if (!ax->ky) ax->ky = pick_strided(ny, dt, 0, 0, 0);
    ax->kx = pick_strided(nx, dt, tx.a, tx.E, tx.v);
    if (!ax->kx) ax->kx = pick_strided(nx, dt, 0, 0, 0);
    ax->kz = pick_z(nz, dt, tz.a, tz.E);
    if (!ax->kz) ax->kz = pick_z(nz, dt, 0, 0);
    if (!ax->kx || !ax->ky || !ax->kz) return fail(TK_EUNSUPPORTED, "no kernel for %dx%dx%d", nx, ny, nz);
    return TK_OK;
}

}  // namespace tk

using namespace tk;

// With TK_FFT_TIMING a plan records HIP events around every pass into a ring of
// NSET sets (no synchronisation); fft3d_pass_times averages the sets recorded since
// its previous call.
static const int NSET = 256;

struct tk_fft3d_s {
    FftAxes ax;
    int batch;
    unsigned flags;
    void *ws;
    bool ws_owned;
    bool timing;
    std::vector<hipEvent_t> ev;  // NSET x 8
    int nr2c, nc2r;
};

// Bytes of the spectral data: the half spectrum, or for the SSS family a real field.
static size_t cplx_bytes(const tk_fft3d_s *p) {
    const size_t esz = p->ax.dt == TK_F32 ? 8 : 16;
    if (p->ax.bz) return esz / 2 * (size_t)p->batch * p->ax.nx * p->ax.ny * p->ax.nz;
    return esz * (size_t)p->batch * p->ax.nx * p->ax.ny * (p->ax.nz / 2 + 1);
}

extern "C" tk_status fft3d_plan_create(tk_fft3d_t *plan, int nx, int ny, int nz, int batch, tk_dtype dt,
                                       unsigned flags) {
    if (!plan) return fail(TK_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (batch < 1) return fail(TK_EINVAL, "batch must be >= 1 (got %d)", batch);
    const unsigned known = TK_FFT_TIMING | TK_FFT_NO_TUNE | TK_FFT_C2R_Y_FIRST | TK_FFT_C2R_OVERWRITE;
    if (flags & ~known) return fail(TK_EINVAL, "unknown plan flags 0x%x", flags & ~known);
    if ((flags & TK_FFT_C2R_Y_FIRST) && (flags & TK_FFT_C2R_OVERWRITE))
        return fail(TK_EINVAL, "TK_FFT_C2R_Y_FIRST and TK_FFT_C2R_OVERWRITE exclude each other");
    tk_fft3d_s *p = new (std::nothrow) tk_fft3d_s();
    if (!p) return fail(TK_ENOMEM, "host allocation failed");
    tk_status st = axes_init(&p->ax, nx, ny, nz, dt, !(flags & TK_FFT_NO_TUNE));
    if (st != TK_OK) {
        delete p;
        return st;
    }
    p->batch = batch;
    p->flags = flags;
    p->ws = nullptr;
    p->ws_owned = false;
    p->timing = (flags & TK_FFT_TIMING) != 0;
    p->nr2c = p->nc2r = 0;
    if (p->timing) {
        p->ev.resize(NSET * 8);
        for (int i = 0; i < NSET * 8; ++i) {
            if (hipEventCreate(&p->ev[i]) != hipSuccess) {
                for (int j = 0; j < i; ++j) hipEventDestroy(p->ev[j]);
                delete p;
                return fail(TK_EHIP, "hipEventCreate failed");
            }
        }
    }
    *plan = p;
    return TK_OK;
}

extern "C" tk_status fft3d_plan_create_basis(tk_fft3d_t *plan, int nx, int ny, int nz, int batch, tk_dtype dt,
                                             int basis_x, int basis_y, unsigned flags) {
    return fft3d_plan_create_basis3(plan, nx, ny, nz, batch, dt, basis_x, basis_y, TK_FOURIER, flags);
}

extern "C" tk_status fft3d_plan_create_basis3(tk_fft3d_t *plan, int nx, int ny, int nz, int batch, tk_dtype dt,
                                              int basis_x, int basis_y, int basis_z, unsigned flags) {
    TK_TRY(fft3d_plan_create(plan, nx, ny, nz, batch, dt, flags));
    tk_status st = axes_set_basis(&(*plan)->ax, basis_x, basis_y, basis_z);
    if (st != TK_OK) {
        fft3d_plan_destroy(*plan);
        *plan = nullptr;
    }
    return st;
}

extern "C" tk_status fft3d_workspace_size(tk_fft3d_t p, size_t *bytes) {
    if (!p || !bytes) return fail(TK_EINVAL, "NULL argument");
    *bytes = (p->flags & TK_FFT_C2R_OVERWRITE) ? 0 : cplx_bytes(p);
    return TK_OK;
}

extern "C" tk_status fft3d_set_workspace(tk_fft3d_t p, void *dev_ptr) {
    if (!p) return fail(TK_EINVAL, "plan is NULL");
    if (p->ws_owned && p->ws) hipFree(p->ws);
    p->ws = dev_ptr;
    p->ws_owned = false;
    return TK_OK;
}

extern "C" tk_status fft3d_r2c(tk_fft3d_t p, const void *real_in, void *cplx_out, void *stream) {
    if (!p || !real_in || !cplx_out) return fail(TK_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const FftAxes &ax = p->ax;
    const double scale = 1.0 / ((double)ax.nx * ax.ny * ax.nz);
    hipEvent_t *ev = p->timing ? &p->ev[(p->nr2c % NSET) * 8] : nullptr;
    if (ev) TK_HIP_CHECK(hipEventRecord(ev[0], s));
    if (ax.bz) {
        TK_TRY(sss_z_pass(ax, real_in, cplx_out, p->batch, 0, s));
        if (ev) TK_HIP_CHECK(hipEventRecord(ev[1], s));
        TK_TRY(sss_y_pass(ax, cplx_out, cplx_out, p->batch, 0, s));
        if (ev) TK_HIP_CHECK(hipEventRecord(ev[2], s));
        TK_TRY(sss_x_pass(ax, cplx_out, cplx_out, p->batch, 0, scale, s));
        if (ev) {
            TK_HIP_CHECK(hipEventRecord(ev[3], s));
            p->nr2c++;
        }
        return TK_OK;
    }
    // sweep directions: each pass starts where the previous one ended (its last writes are
    // still in the memory-side cache) when the two visit the data in the same order
    TK_TRY(fft_z_r2c(ax, real_in, cplx_out, p->batch, 1.0, s));
    if (ev) TK_HIP_CHECK(hipEventRecord(ev[1], s));
    TK_TRY(fft_y_pass(ax, cplx_out, cplx_out, p->batch, 0, s, 1));
    if (ev) TK_HIP_CHECK(hipEventRecord(ev[2], s));
    TK_TRY(fft_x_pass(ax, cplx_out, cplx_out, p->batch, 0, scale, s));
    if (ev) {
        TK_HIP_CHECK(hipEventRecord(ev[3], s));
        p->nr2c++;
    }
    return TK_OK;
}

// The inverse passes.  ws == nullptr: in place on the input (TK_FFT_C2R_OVERWRITE);
// else the X (or Y) inverse writes ws out of place and the input is preserved.
static tk_status c2r_run(tk_fft3d_s *p, const void *cplx_in, void *ws, void *real_out, hipStream_t s) {
    const FftAxes &ax = p->ax;
    hipEvent_t *ev = p->timing ? &p->ev[(p->nc2r % NSET) * 8] : nullptr;
    if (ev) TK_HIP_CHECK(hipEventRecord(ev[4], s));
    if (ax.bz) {
        // SSS family: X, then Y, in place on ws (or on the input), then Z into the output
        void *w = ws ? ws : const_cast<void *>(cplx_in);
        TK_TRY(sss_x_pass(ax, cplx_in, w, p->batch, 1, 1.0, s));
        if (ev) TK_HIP_CHECK(hipEventRecord(ev[5], s));
        TK_TRY(sss_y_pass(ax, w, w, p->batch, 1, s));
        if (ev) TK_HIP_CHECK(hipEventRecord(ev[6], s));
        TK_TRY(sss_z_pass(ax, w, real_out, p->batch, 1, s));
        if (ev) {
            TK_HIP_CHECK(hipEventRecord(ev[7], s));
            p->nc2r++;
        }
        return TK_OK;
    }
    const bool y_first = ws && (p->flags & TK_FFT_C2R_Y_FIRST);
    if (!ws) {
        // in place on the input: X backwards (the forward X pass wrote those columns last),
        // Y, then Z into the output
        void *w = const_cast<void *>(cplx_in);
        TK_TRY(fft_x_pass(ax, w, w, p->batch, 1, 1.0, s, 1));
        if (ev) TK_HIP_CHECK(hipEventRecord(ev[5], s));
        TK_TRY(fft_y_pass(ax, w, w, p->batch, 1, s));
        ws = w;
    } else if (y_first) {
        // the X and Y inverses commute: the one out-of-place pass is then the Y pass
        TK_TRY(fft_y_pass(ax, cplx_in, ws, p->batch, 1, s));
        if (ev) TK_HIP_CHECK(hipEventRecord(ev[5], s));
        TK_TRY(fft_x_pass(ax, ws, ws, p->batch, 1, 1.0, s));
    } else {
        // X backwards over the columns the forward X pass wrote last, then Y, then Z
        TK_TRY(fft_x_pass(ax, cplx_in, ws, p->batch, 1, 1.0, s, 1));
        if (ev) TK_HIP_CHECK(hipEventRecord(ev[5], s));
        TK_TRY(fft_y_pass(ax, ws, ws, p->batch, 1, s));
    }
    if (ev) TK_HIP_CHECK(hipEventRecord(ev[6], s));
    // Z forwards: backwards (from the x planes the Y pass wrote last) it ran as fast, but the
    // next forward Z pass, reading the planes this one had just written, ran 12% slower
    TK_TRY(fft_z_c2r(ax, ws, real_out, p->batch, s, 0));
    if (ev) {
        TK_HIP_CHECK(hipEventRecord(ev[7], s));
        p->nc2r++;
    }
    return TK_OK;
}

extern "C" tk_status fft3d_c2r(tk_fft3d_t p, const void *cplx_in, void *real_out, void *stream) {
    if (!p || !cplx_in || !real_out) return fail(TK_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (p->flags & TK_FFT_C2R_OVERWRITE) return c2r_run(p, cplx_in, nullptr, real_out, s);
    if (!p->ws) {
        if (hipMalloc(&p->ws, cplx_bytes(p)) != hipSuccess) {
            p->ws = nullptr;
            return fail(TK_ENOMEM, "workspace allocation of %zu bytes failed", cplx_bytes(p));
        }
        p->ws_owned = true;
    }
    return c2r_run(p, cplx_in, p->ws, real_out, s);
}

// Workspace of fft3d_c2r_noalloc: a file-scope device array that each device holds from
// the moment this code object is loaded on it until the process ends.  In host code its
// name is only a host-side stand-in: the device address comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address is passed on.
static __device__ __align__(256) unsigned char scratch[TK_SCRATCH_BYTES];

static const int kMaxDevices = 64;

static tk_status scratch_address(void **out) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    TK_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(TK_EUNSUPPORTED, "device ordinal %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(TK_EHIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
        addr[dev] = ptr;
    }
    *out = addr[dev];
    return TK_OK;
}

extern "C" tk_status fft3d_c2r_noalloc(tk_fft3d_t p, const void *cplx_in, void *real_out, void *stream) {
    if (!p || !cplx_in || !real_out) return fail(TK_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (p->flags & TK_FFT_C2R_OVERWRITE) return c2r_run(p, cplx_in, nullptr, real_out, s);
    const size_t need = cplx_bytes(p);
    if (need > TK_SCRATCH_BYTES)
        return fail(TK_EINVAL, "fft3d_c2r_noalloc: workspace of %zu bytes exceeds the static scratch of %zu bytes",
                    need, (size_t)TK_SCRATCH_BYTES);
    void *ws = nullptr;
    TK_TRY(scratch_address(&ws));
    return c2r_run(p, cplx_in, ws, real_out, s);
}

extern "C" tk_status fft3d_pass_times(tk_fft3d_t p, float t[6]) {
    if (!p || !t) return fail(TK_EINVAL, "NULL argument");
    if (!p->timing) return fail(TK_ESTATE, "plan was created without TK_FFT_TIMING");
    const int nf = std::min(p->nr2c, NSET), ni = std::min(p->nc2r, NSET);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < nf; ++k) {
        hipEvent_t *ev = &p->ev[k * 8];
        TK_HIP_CHECK(hipEventSynchronize(ev[3]));
        for (int i = 0; i < 3; ++i) {
            float ms;
            TK_HIP_CHECK(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            acc[i] += ms;
        }
    }
    for (int k = 0; k < ni; ++k) {
        hipEvent_t *ev = &p->ev[k * 8];
        TK_HIP_CHECK(hipEventSynchronize(ev[7]));
        for (int i = 0; i < 3; ++i) {
            float ms;
            TK_HIP_CHECK(hipEventElapsedTime(&ms, ev[4 + i], ev[5 + i]));
            acc[3 + i] += ms;
        }
    }
    for (int i = 0; i < 3; ++i) {
        t[i] = nf ? (float)(acc[i] / nf) : 0.f;
        t[3 + i] = ni ? (float)(acc[3 + i] / ni) : 0.f;
    }
    p->nr2c = p->nc2r = 0;
    return TK_OK;
}

extern "C" tk_status fft3d_parseval(tk_fft3d_t p, const void *real, const void *cplx, double out[2], void *stream) {
    if (!p || !real || !cplx || !out) return fail(TK_EINVAL, "NULL argument");
    const FftAxes &ax = p->ax;
    if (ax.bz) return fail(TK_EUNSUPPORTED, "fft3d_parseval: the half-spectrum sums do not apply to the SSS family");
    long npts = (long)ax.nx * ax.ny * ax.nz;
    double a = 0, b = 0;
    TK_TRY(reduce_sumsq_real(real, npts, ax.dt, &a, (hipStream_t)stream));
    TK_TRY(reduce_sumsq_half(cplx, (long)ax.nx * ax.ny, ax.nz, ax.dt, &b, (hipStream_t)stream));
    out[0] = a / (double)npts;
    out[1] = b;
    return TK_OK;
}

extern "C" tk_status fft3d_describe(tk_fft3d_t p, int pass, char *buf, int len) {
    if (!p || !buf || len <= 0) return fail(TK_EINVAL, "bad argument");
    const FftAxes &ax = p->ax;
    int n = 0;
    if (pass == 0 && ax.bz)
        n = snprintf(buf, len, "z N=%d %s (line pairs)", ax.nz, ax.bz == 1 ? "sine" : "cosine");
    else if (pass == 0)
        n = snprintf(buf, len, "z N=%d LPW=%d E=%d nt=%d lds=%d", ax.nz, ax.kz->LPW, ax.kz->E, ax.kz->nt, ax.kz->lds);
    else if (pass == 1 || pass == 2) {
        const StridedKernel *k = pass == 1 ? ax.ky : ax.kx;
        n = snprintf(buf, len, "%c L=%d W=%d E=%d v=%d nt=%d lds=%d", pass == 1 ? 'y' : 'x', k->L, k->W, k->E, k->var,
                     k->nt, k->lds);
    } else
        return fail(TK_EINVAL, "pass must be 0, 1 or 2");
    (void)n;
    return TK_OK;
}

extern "C" tk_status fft3d_plan_destroy(tk_fft3d_t p) {
    if (!p) return TK_OK;
    if (p->ws_owned && p->ws) hipFree(p->ws);
    for (hipEvent_t e : p->ev) hipEventDestroy(e);
    delete p;
    return TK_OK;
}

extern "C" tk_status tk_sum_squares(const void *x, long n, tk_dtype dt, double *out, void *stream) {
    if (!x || !out || n < 0) return fail(TK_EINVAL, "bad arguments");
    if (dt != TK_F32 && dt != TK_F64) return fail(TK_EUNSUPPORTED, "dtype");
    if (n == 0) {
        *out = 0;
        return TK_OK;
    }
    return reduce_sumsq_real(x, n, dt, out, (hipStream_t)stream);
}
