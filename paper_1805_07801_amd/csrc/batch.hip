// Ensembles of independent Navier-Stokes solves of mixed grid sizes.
//
// The members are grouped by grid size.  Each pass of a right-hand side (P1 .. P5, see
// ns_kernels.hpp) is one persistent kernel per size class: a grid sized to the GPU walks
// the class's work list of (instance, tile) items with the same tile functions the single
// solver uses.  The classes run their chains of passes on separate streams of one HIP
// graph (one IF-RK2 step of all members), captured once and replayed, so a step costs one
// graph launch and the classes' kernels overlap.
#include <algorithm>
#include <array>
#include <functional>
#include <cmath>
#include <new>

#include "ns_api.hpp"

namespace tk {

#define TK_BATCH_SIZES(X) X(16) X(24) X(32) X(48) X(64) X(96) X(128)

constexpr int BNT = 256;  // threads per workgroup of every batch kernel

// Tile shapes with 256 threads for every size: strided / X passes W = 256 E / N columns,
// fused Z pass LPW = 256 / (N/2 / E2) lines.
template <int N> struct BCfg {
    static constexpr int E = default_E(N);
    static constexpr int W = BNT * E / N;
    static constexpr int L2 = N / 2;
    static constexpr int E2 = default_E(L2);
    static constexpr int LPW = BNT / (L2 / E2);
    static constexpr int lds_x = N * (W + 1) + N;                      // exchange + twiddles
    static constexpr int lds_z = LPW * lds_line_len<L2>() + N;         // lines + twiddles
    static_assert(W * (N / E) == BNT && LPW * (L2 / E2) == BNT, "batch tile shape");
};

struct BInst {
    int n, K, KZC, KZP;  // KZP: transit row length (ns_kzp)
    float2 *u, *w6, *aux;  // state, transit workspace, RK accumulator (the stage input stays in registers)
    NsState *st;
    const float2 *tw;
    double nu;
};

struct BItem {
    int inst, tile;
};

static bool batch_size_ok(int n) {
#define TK_OK_N(N) if (n == N) return true;
    TK_BATCH_SIZES(TK_OK_N)
#undef TK_OK_N
    return false;
}

// ---- persistent pass kernels -------------------------------------------------------------------
// One kernel per pass and grid size: a size class's work list holds the (instance, tile)
// items of its members only, so each kernel's registers and LDS fit its own tiles (a single
// kernel switching over every size took the largest size's registers for all of them).
template <int N>
__global__ __launch_bounds__(BNT) void kb_p1(const BInst *__restrict__ inst, const BItem *__restrict__ items,
                                             int nitems) {
    __shared__ float2 smem[BCfg<N>::lds_x];
    float2 *tw = smem;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BItem w = items[it];
        const BInst &d = inst[w.inst];
        __syncthreads();
        load_twiddles<float>(tw, d.tw, N, threadIdx.x, BNT);
        __syncthreads();
        ns_p1_tile<float, N, BCfg<N>::E, BCfg<N>::W>(d.u, d.w6, d.K, 0, w.tile, smem + N, tw);
    }
}

template <int N>
__global__ __launch_bounds__(BNT) void kb_y(const BInst *__restrict__ inst, const BItem *__restrict__ items,
                                            int nitems, int nf, int inv) {
    __shared__ float2 smem[BCfg<N>::lds_x];
    float2 *tw = smem;
    constexpr long KZP = ns_kzp<N>();
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BItem w = items[it];
        const BInst &d = inst[w.inst];
        __syncthreads();
        load_twiddles<float>(tw, d.tw, N, threadIdx.x, BNT);
        __syncthreads();
        strided_tile<float, N, BCfg<N>::E, BCfg<N>::W>(d.w6, d.w6, (long)nf * N * KZP, KZP, N * KZP, KZP, inv, 1.0f,
                                                       inv ? d.K : -1, inv ? -1 : d.K, w.tile, smem + N, tw);
    }
}

template <int N>
__global__ __launch_bounds__(BNT) void kb_p3(const BInst *__restrict__ inst, const BItem *__restrict__ items,
                                             int nitems, int with_umax) {
    __shared__ float2 smem[BCfg<N>::lds_z];
    float2 *tw = smem;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BItem w = items[it];
        const BInst &d = inst[w.inst];
        unsigned *um = with_umax ? &d.st->umax : nullptr;
        __syncthreads();
        load_twiddles<float>(tw, d.tw, N, threadIdx.x, BNT);
        __syncthreads();
        ns_p3_tile<float, N / 2, BCfg<N>::E2, BCfg<N>::LPW>(d.w6, (long)N * N, d.KZC, w.tile, smem + N, tw, um);
    }
}

// P5 fused with the next right-hand side's P1 (the stage input, or the new state, stays in
// registers; see ns_p5_tile).
template <int N>
__global__ __launch_bounds__(BNT) void kb_p51(const BInst *__restrict__ inst, const BItem *__restrict__ items,
                                              int nitems, int mode) {
    __shared__ float2 smem[BCfg<N>::lds_x];
    float2 *tw = smem;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BItem w = items[it];
        const BInst &d = inst[w.inst];
        __syncthreads();
        load_twiddles<float>(tw, d.tw, N, threadIdx.x, BNT);
        __syncthreads();
        ns_p5_tile<float, N, BCfg<N>::E, BCfg<N>::W, true>(d.w6, nullptr, d.u, d.aux, nullptr, nullptr, d.st, d.nu,
                                                           mode, d.K, d.KZC, w.tile, smem + N, tw, d.w6);
    }
}

// Step size of the members of grid size n (the other members belong to other size classes).
__global__ void kb_set_h(const BInst *__restrict__ inst, int count, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count && inst[i].n == n) {
        NsState *st = inst[i].st;
        double h = st->hfix;
        if (st->cfl_dx > 0) {
            const double um = (double)__uint_as_float(st->umax);
            h = um > 0 ? st->cfl_dx / um : st->hfix;
        }
        st->h = h;
        st->t += h;
        st->umax = 0u;
    }
}

// The pass kernels of one size class.
struct BClassFns {
    int n;
    void (*p1)(const BInst *, const BItem *, int);
    void (*y)(const BInst *, const BItem *, int, int, int);
    void (*p3)(const BInst *, const BItem *, int, int);
    void (*p51)(const BInst *, const BItem *, int, int);
};
static BClassFns class_fns(int n) {
#define TK_FNS(N) \
    if (n == N) return {N, &kb_p1<N>, &kb_y<N>, &kb_p3<N>, &kb_p51<N>};
    TK_BATCH_SIZES(TK_FNS)
#undef TK_FNS
    return {0, nullptr, nullptr, nullptr, nullptr};
}

// Tiles per instance of each pass.
// ncols_per_ky: the KZP transit columns of each kept ky row (P1 and P5).
static long tiles_x(int n, int K, int ncols_per_ky) {
    long W = 0;
#define TK_W(N) if (n == N) W = BCfg<N>::W;
    TK_BATCH_SIZES(TK_W)
#undef TK_W
    return ((long)(2 * K + 1) * ncols_per_ky + W - 1) / W;
}
static long tiles_y(int n, int cols, int nf) {
    long W = 0;
#define TK_W(N) if (n == N) W = BCfg<N>::W;
    TK_BATCH_SIZES(TK_W)
#undef TK_W
    return ((long)nf * n * cols + W - 1) / W;
}
static long tiles_z(int n) {
    long LPW = 0;
#define TK_W(N) if (n == N) LPW = BCfg<N>::LPW;
    TK_BATCH_SIZES(TK_W)
#undef TK_W
    return ((long)n * n + LPW - 1) / LPW;
}

}  // namespace tk

using namespace tk;

struct tk_nsb_s {
    int count = 0;
    int grid = 1024;
    std::vector<int> n;
    std::vector<double> nu;
    double cfl = 0;
    std::vector<BInst> hinst;
    BInst *dinst = nullptr;
    std::vector<NsState> hstate;
    NsState *dstate = nullptr;
    // per size class c: work lists 0 = P5, 1 = Y over 6 fields, 2 = Z lines, 3 = Y over 3
    // fields, 4 = P1, at items[c][list]
    std::vector<int> cls_n;
    std::vector<std::array<BItem *, 5>> items;
    std::vector<std::array<int, 5>> nitems;
    std::vector<void *> bufs;
    double *dscratch = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<NsGrid> grids;  // per instance (for init and diagnostics)
};

static void nsb_free(tk_nsb_s *b) {
    if (b->gexec) hipGraphExecDestroy(b->gexec);
    if (b->graph) hipGraphDestroy(b->graph);
    for (void *p : b->bufs) hipFree(p);
    for (auto &c : b->items)
        for (BItem *it : c)
            if (it) hipFree(it);
    if (b->dinst) hipFree(b->dinst);
    if (b->dstate) hipFree(b->dstate);
    if (b->dscratch) hipFree(b->dscratch);
    delete b;
}

// One IF-RK2 step of every member as one graph: each size class runs its own chain of
// passes (Y, P3, step size, Y, P5 fused with the second stage's P1, then Y, P3, Y, P5
// fused with the next step's P1) on a stream of its own, forked from and joined to the
// capture stream, so the classes' kernels overlap on the GPU.  On entry the workspace
// holds P1 of the state (nsb_p1 before the first step of a call).
static tk_status nsb_capture(tk_nsb_s *b) {
    const int nc = (int)b->cls_n.size();
    hipStream_t cs;
    TK_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    std::vector<hipStream_t> ss(nc, nullptr);
    std::vector<hipEvent_t> ev(nc + 1, nullptr);
    tk_status st = TK_OK;
    auto cleanup = [&] {
        for (auto q : ss)
            if (q) hipStreamDestroy(q);
        for (auto e : ev)
            if (e) hipEventDestroy(e);
        hipStreamDestroy(cs);
    };
    for (int c = 0; c < nc; ++c)
        if (hipStreamCreateWithFlags(&ss[c], hipStreamNonBlocking) != hipSuccess) st = TK_EHIP;
    for (int c = 0; c <= nc; ++c)
        if (hipEventCreateWithFlags(&ev[c], hipEventDisableTiming) != hipSuccess) st = TK_EHIP;
    if (st != TK_OK) {
        cleanup();
        return fail(TK_EHIP, "ensemble stream setup failed");
    }
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = hipEventRecord(ev[nc], cs);
    for (int c = 0; c < nc && e == hipSuccess; ++c) {
        hipStream_t q = ss[c];
        e = hipStreamWaitEvent(q, ev[nc], 0);
        if (e != hipSuccess) break;
        const BClassFns f = class_fns(b->cls_n[c]);
        const auto &it = b->items[c];
        const auto &ni = b->nitems[c];
        auto g = [&](int list) { return (unsigned)std::max(1, std::min(b->grid, ni[list])); };
        for (int stage = 0; stage < 2; ++stage) {
            hipLaunchKernelGGL(f.y, dim3(g(1)), dim3(BNT), 0, q, b->dinst, it[1], ni[1], 6, 1);
            hipLaunchKernelGGL(f.p3, dim3(g(2)), dim3(BNT), 0, q, b->dinst, it[2], ni[2], stage == 0);
            if (stage == 0)
                hipLaunchKernelGGL(kb_set_h, dim3(cdiv(b->count, 64)), dim3(64), 0, q, b->dinst, b->count, f.n);
            hipLaunchKernelGGL(f.y, dim3(g(3)), dim3(BNT), 0, q, b->dinst, it[3], ni[3], 3, 0);
            hipLaunchKernelGGL(f.p51, dim3(g(0)), dim3(BNT), 0, q, b->dinst, it[0], ni[0],
                               stage == 0 ? (int)RK2_S1 : (int)RK2_S2);
        }
        e = hipEventRecord(ev[c], q);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev[c], 0);
    }
    hipGraph_t gr = nullptr;
    const hipError_t le = hipGetLastError();
    const hipError_t ee = hipStreamEndCapture(cs, &gr);
    cleanup();
    if (e != hipSuccess || le != hipSuccess) {
        if (gr) hipGraphDestroy(gr);
        return fail(TK_EHIP, "ensemble graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : le));
    }
    if (ee != hipSuccess) return fail(TK_EHIP, "ensemble graph capture failed: %s", hipGetErrorString(ee));
    e = hipGraphInstantiate(&b->gexec, gr, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(gr);
        return fail(TK_EHIP, "ensemble graph instantiation failed: %s", hipGetErrorString(e));
    }
    b->graph = gr;
    return TK_OK;
}

// P1 of every member's state into its workspace (before the first step of a call).
static tk_status nsb_p1(tk_nsb_s *b, hipStream_t s) {
    for (size_t c = 0; c < b->cls_n.size(); ++c) {
        const BClassFns f = class_fns(b->cls_n[c]);
        const int ni = b->nitems[c][4];
        const unsigned g = (unsigned)std::max(1, std::min(b->grid, ni));
        hipLaunchKernelGGL(f.p1, dim3(g), dim3(BNT), 0, s, b->dinst, b->items[c][4], ni);
    }
    return launch_check("ensemble P1");
}

extern "C" tk_status ns_batch_create(tk_nsb_t *out, int count, const int *n, const double *nu, tk_dtype dt,
                                     double cfl, unsigned flags) {
    if (!out || !n || !nu) return fail(TK_EINVAL, "NULL argument");
    *out = nullptr;
    if (count < 1) return fail(TK_EINVAL, "count must be >= 1");
    if (dt != TK_F32) return fail(TK_EUNSUPPORTED, "ensembles run in FP32");
    if (cfl < 0 || !std::isfinite(cfl)) return fail(TK_EINVAL, "cfl must be finite and >= 0");
    for (int i = 0; i < count; ++i) {
        if (!batch_size_ok(n[i])) return fail(TK_EUNSUPPORTED, "ensemble member %d: n=%d not in {16..128}", i, n[i]);
        if (!(nu[i] >= 0) || !std::isfinite(nu[i])) return fail(TK_EINVAL, "member %d: bad nu", i);
    }
    tk_nsb_s *b = new (std::nothrow) tk_nsb_s();
    if (!b) return fail(TK_ENOMEM, "host allocation failed");
    b->count = count;
    b->n.assign(n, n + count);
    b->nu.assign(nu, nu + count);
    b->cfl = cfl;
    if (flags >> 16) b->grid = (int)(flags >> 16);  // persistent grid size override
    b->grids.resize(count);
    b->hinst.resize(count);
    b->hstate.resize(count);
    int maxshell = 0;
    for (int i = 0; i < count; ++i) {
        tk_status st = ns_grid_init(&b->grids[i], n[i], TK_F32);
        if (st != TK_OK) {
            nsb_free(b);
            return st;
        }
        const size_t fb = (size_t)n[i] * n[i] * (n[i] / 2 + 1) * sizeof(float2);
        void *w6 = nullptr, *aux = nullptr;
        if (hipMalloc(&w6, 6 * fb) != hipSuccess || hipMalloc(&aux, 3 * fb) != hipSuccess) {
            if (w6) hipFree(w6);
            nsb_free(b);
            return fail(TK_ENOMEM, "ensemble workspace allocation failed");
        }
        b->bufs.push_back(w6);
        b->bufs.push_back(aux);
        // the accumulator starts at zero: passes write only the 2/3-rule modes
        if (hipMemset(aux, 0, 3 * fb) != hipSuccess || hipMemset(w6, 0, 6 * fb) != hipSuccess) {
            nsb_free(b);
            return fail(TK_EHIP, "ensemble workspace clear failed");
        }
        BInst &d = b->hinst[i];
        d.n = n[i];
        d.K = b->grids[i].K;
        d.KZC = b->grids[i].KZC;
        d.KZP = b->grids[i].KZP;
        d.u = nullptr;
        d.w6 = (float2 *)w6;
        d.aux = (float2 *)aux;
        d.tw = (const float2 *)b->grids[i].ax.twx;
        d.nu = nu[i];
        maxshell = std::max(maxshell, ns_num_shells(n[i]));
    }
    if (hipMalloc((void **)&b->dinst, sizeof(BInst) * count) != hipSuccess ||
        hipMalloc((void **)&b->dstate, sizeof(NsState) * count) != hipSuccess ||
        hipMalloc((void **)&b->dscratch, sizeof(double) * (NS_DIAG_BLOCKS + 2) * (NS_DIAG_HEAD + maxshell)) !=
            hipSuccess) {
        nsb_free(b);
        return fail(TK_ENOMEM, "ensemble tables allocation failed");
    }
    for (int i = 0; i < count; ++i) b->hinst[i].st = b->dstate + i;
    // size classes, largest grids first; per class its work lists
    std::vector<int> sizes(n, n + count);
    std::sort(sizes.begin(), sizes.end(), std::greater<int>());
    sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
    b->cls_n = sizes;
    b->items.assign(sizes.size(), {nullptr, nullptr, nullptr, nullptr, nullptr});
    b->nitems.assign(sizes.size(), {0, 0, 0, 0, 0});
    for (size_t c = 0; c < sizes.size(); ++c) {
        for (int list = 0; list < 5; ++list) {
            std::vector<BItem> v;
            for (int i = 0; i < count; ++i) {
                const BInst &d = b->hinst[i];
                if (d.n != sizes[c]) continue;
                long nt = list == 0 ? tiles_x(d.n, d.K, d.KZP)
                          : list == 1 ? tiles_y(d.n, d.KZP, 6)
                          : list == 2 ? tiles_z(d.n)
                          : list == 3 ? tiles_y(d.n, d.KZP, 3)
                                      : tiles_x(d.n, d.K, d.KZP);
                for (long t = 0; t < nt; ++t) v.push_back({i, (int)t});
            }
            b->nitems[c][list] = (int)v.size();
            if (hipMalloc((void **)&b->items[c][list], sizeof(BItem) * v.size()) != hipSuccess ||
                hipMemcpy(b->items[c][list], v.data(), sizeof(BItem) * v.size(), hipMemcpyHostToDevice) !=
                    hipSuccess) {
                nsb_free(b);
                return fail(TK_ENOMEM, "work list upload failed");
            }
        }
    }
    tk_status st = nsb_capture(b);
    if (st != TK_OK) {
        nsb_free(b);
        return st;
    }
    *out = b;
    return TK_OK;
}

extern "C" tk_status ns_batch_step(tk_nsb_t b, void *const *uhat, double dt, int nsteps, double *t, void *stream) {
    if (!b || !uhat) return fail(TK_EINVAL, "NULL argument");
    if (nsteps < 0) return fail(TK_EINVAL, "nsteps must be >= 0");
    if (b->cfl <= 0 && !(dt > 0 && std::isfinite(dt))) return fail(TK_EINVAL, "dt must be > 0 without CFL");
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < b->count; ++i) {
        if (!uhat[i]) return fail(TK_EINVAL, "uhat[%d] is NULL", i);
        b->hinst[i].u = (float2 *)uhat[i];
        NsState &h = b->hstate[i];
        h = NsState{};
        h.t = t ? t[i] : 0.0;
        h.hfix = dt > 0 ? dt : 0.0;
        h.h = h.hfix;
        h.cfl_dx = b->cfl > 0 ? b->cfl * 2.0 * M_PI / b->n[i] : 0.0;
    }
    TK_HIP_CHECK(hipMemcpyAsync(b->dinst, b->hinst.data(), sizeof(BInst) * b->count, hipMemcpyHostToDevice, s));
    TK_HIP_CHECK(hipMemcpyAsync(b->dstate, b->hstate.data(), sizeof(NsState) * b->count, hipMemcpyHostToDevice, s));
    if (nsteps > 0) TK_TRY(nsb_p1(b, s));
    for (int k = 0; k < nsteps; ++k) TK_HIP_CHECK(hipGraphLaunch(b->gexec, s));
    TK_HIP_CHECK(hipMemcpyAsync(b->hstate.data(), b->dstate, sizeof(NsState) * b->count, hipMemcpyDeviceToHost, s));
    TK_HIP_CHECK(hipStreamSynchronize(s));
    if (t)
        for (int i = 0; i < b->count; ++i) t[i] = b->hstate[i].t;
    return TK_OK;
}

extern "C" tk_status ns_batch_init_random(tk_nsb_t b, int i, const void *noise, void *u, double energy,
                                          void *stream) {
    if (!b || !noise || !u) return fail(TK_EINVAL, "NULL argument");
    if (i < 0 || i >= b->count) return fail(TK_EINVAL, "member index %d out of range", i);
    if (!(energy > 0) || !std::isfinite(energy)) return fail(TK_EINVAL, "energy must be > 0");
    return ns_init_random_grid(b->grids[i], noise, u, energy, b->dscratch, (hipStream_t)stream);
}

extern "C" tk_status ns_batch_diagnostics(tk_nsb_t b, int i, const void *u, double *energy, double *dissipation,
                                          double *max_div, void *stream) {
    if (!b || !u) return fail(TK_EINVAL, "NULL argument");
    if (i < 0 || i >= b->count) return fail(TK_EINVAL, "member index %d out of range", i);
    const int nsh = ns_num_shells(b->n[i]);
    std::vector<double> h(NS_DIAG_HEAD + nsh);
    TK_TRY(ns_diag_run(u, b->n[i], TK_F32, nsh, b->dscratch, h.data(), (hipStream_t)stream));
    if (energy) *energy = h[0];
    if (dissipation) *dissipation = 2.0 * b->nu[i] * h[1];
    if (max_div) *max_div = h[3] > 0 ? std::sqrt(h[2] / h[3]) : 0.0;
    if (!std::isfinite(h[0])) return fail(TK_ESTATE, "member %d: energy is not finite", i);
    return TK_OK;
}

extern "C" tk_status ns_batch_last_dt(tk_nsb_t b, double *dt) {
    if (!b || !dt) return fail(TK_EINVAL, "NULL argument");
    for (int i = 0; i < b->count; ++i) dt[i] = b->hstate[i].h;
    return TK_OK;
}

extern "C" tk_status ns_batch_destroy(tk_nsb_t b) {
    if (b) nsb_free(b);
    return TK_OK;
}
