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
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <string>

#include "ns_api.hpp"
#include "reduce.hpp"
#include "tune.hpp"

namespace tk {

#define TK_BATCH_SIZES(X) X(16) X(24) X(32) X(48) X(64) X(96) X(128)

constexpr int BNT = 256;  // threads per workgroup of the default batch kernels

// Tile shapes with NT threads: strided / X passes W = NT E / N columns, fused Z pass LPW =
// NT / (N/2 / E2) lines.  NT is a tuning choice per grid size (ns_batch_autotune).
template <int N, int NT = BNT> struct BCfg {
    static constexpr int E = default_E(N);
    static constexpr int W = NT * E / N;
    static constexpr int L2 = N / 2;
    static constexpr int E2 = default_E(L2);
    static constexpr int LPW = NT / (L2 / E2);
    static constexpr int lds_x = N * (W + 1) + N;                      // exchange + twiddles
    static constexpr int lds_z = LPW * lds_line_len<L2>() + N;         // lines + twiddles
    static constexpr bool ok = W >= 1 && W * (N / E) == NT && LPW >= 1 && LPW * (L2 / E2) == NT &&
                               (long)lds_x * 8 <= 65536 && (long)lds_z * 8 <= 65536;
};

// Compiled thread counts of the batch kernels (variant v = index; 0 is the default).
constexpr int BNT_VARIANTS[3] = {256, 128, 512};
constexpr int BNT_NVAR = 3;
// Persistent grid choices: 256 << v workgroups, v = 0 .. BGRID_MAXV.
constexpr int BGRID_MAXV = 6;

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
template <int N, int NT>
__global__ __launch_bounds__(NT) void kb_p1(const BInst *__restrict__ inst, const BItem *__restrict__ items,
                                             int nitems) {
    __shared__ float2 smem[BCfg<N, NT>::lds_x];
    float2 *tw = smem;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BItem w = items[it];
        const BInst &d = inst[w.inst];
        __syncthreads();
        load_twiddles<float>(tw, d.tw, N, threadIdx.x, NT);
        __syncthreads();
        ns_p1_tile<float, N, BCfg<N, NT>::E, BCfg<N, NT>::W>(d.u, d.w6, d.K, 0, w.tile, smem + N, tw);
    }
}

template <int N, int NT>
__global__ __launch_bounds__(NT) void kb_y(const BInst *__restrict__ inst, const BItem *__restrict__ items,
                                            int nitems, int nf, int inv) {
    __shared__ float2 smem[BCfg<N, NT>::lds_x];
    float2 *tw = smem;
    constexpr long KZP = ns_kzp<N>();
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BItem w = items[it];
        const BInst &d = inst[w.inst];
        __syncthreads();
        load_twiddles<float>(tw, d.tw, N, threadIdx.x, NT);
        __syncthreads();
        strided_tile<float, N, BCfg<N, NT>::E, BCfg<N, NT>::W>(d.w6, d.w6, (long)nf * N * KZP, KZP, N * KZP, KZP, inv, 1.0f,
                                                       inv ? d.K : -1, inv ? -1 : d.K, w.tile, smem + N, tw);
    }
}

template <int N, int NT>
__global__ __launch_bounds__(NT) void kb_p3(const BInst *__restrict__ inst, const BItem *__restrict__ items,
                                             int nitems, int with_umax) {
    __shared__ float2 smem[BCfg<N, NT>::lds_z];
    float2 *tw = smem;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BItem w = items[it];
        const BInst &d = inst[w.inst];
        unsigned *um = with_umax ? &d.st->umax : nullptr;
        __syncthreads();
        load_twiddles<float>(tw, d.tw, N, threadIdx.x, NT);
        __syncthreads();
        ns_p3_tile<float, N / 2, BCfg<N, NT>::E2, BCfg<N, NT>::LPW>(d.w6, (long)N * N, d.KZC, w.tile, smem + N, tw, um);
    }
}

// P5 fused with the next right-hand side's P1 (the stage input, or the new state, stays in
// registers; see ns_p5_tile).
template <int N, int NT>
__global__ __launch_bounds__(NT) void kb_p51(const BInst *__restrict__ inst, const BItem *__restrict__ items,
                                              int nitems, int mode) {
    __shared__ float2 smem[BCfg<N, NT>::lds_x];
    float2 *tw = smem;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BItem w = items[it];
        const BInst &d = inst[w.inst];
        __syncthreads();
        load_twiddles<float>(tw, d.tw, N, threadIdx.x, NT);
        __syncthreads();
        ns_p5_tile<float, N, BCfg<N, NT>::E, BCfg<N, NT>::W, true>(d.w6, nullptr, d.u, d.aux, nullptr, nullptr, d.st, d.nu,
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

// The pass kernels of one size class, with nt threads per workgroup.
struct BClassFns {
    int n, nt;
    void (*p1)(const BInst *, const BItem *, int);
    void (*y)(const BInst *, const BItem *, int, int, int);
    void (*p3)(const BInst *, const BItem *, int, int);
    void (*p51)(const BInst *, const BItem *, int, int);
    int W, LPW;
};
template <int N, int NT> static BClassFns class_fns_nt() {
    if constexpr (BCfg<N, NT>::ok)
        return {N, NT, &kb_p1<N, NT>, &kb_y<N, NT>, &kb_p3<N, NT>, &kb_p51<N, NT>, BCfg<N, NT>::W, BCfg<N, NT>::LPW};
    else
        return {0, 0, nullptr, nullptr, nullptr, nullptr, 0, 0};
}
static BClassFns class_fns(int n, int nt) {
#define TK_FNS(N)                                           \
    if (n == N) {                                           \
        if (nt == 256) return class_fns_nt<N, 256>();       \
        if (nt == 128) return class_fns_nt<N, 128>();       \
        if (nt == 512) return class_fns_nt<N, 512>();       \
    }
    TK_BATCH_SIZES(TK_FNS)
#undef TK_FNS
    return {0, 0, nullptr, nullptr, nullptr, nullptr, 0, 0};
}

// Tiles per instance of each pass for a class of W columns (X and Y passes) and LPW lines
// (Z pass) per tile.  ncols_per_ky: the KZP transit columns of each kept ky row (P1 and P5).
static long tiles_x(int W, int K, int ncols_per_ky) { return ((long)(2 * K + 1) * ncols_per_ky + W - 1) / W; }
static long tiles_y(int W, int n, int cols, int nf) { return ((long)nf * n * cols + W - 1) / W; }
static long tiles_z(int LPW, int n) { return ((long)n * n + LPW - 1) / LPW; }

}  // namespace tk

using namespace tk;

struct tk_nsb_s {
    int count = 0;
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
    std::vector<BClassFns> cls_fns;  // per class: kernels of its thread count
    std::vector<int> cls_grid;       // per class: persistent grid size (workgroups)
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
        const BClassFns &f = b->cls_fns[c];
        const auto &it = b->items[c];
        const auto &ni = b->nitems[c];
        const int G = b->cls_grid[c];
        auto g = [&](int list) { return (unsigned)std::max(1, std::min(G, ni[list])); };
        for (int stage = 0; stage < 2; ++stage) {
            hipLaunchKernelGGL(f.y, dim3(g(1)), dim3(f.nt), 0, q, b->dinst, it[1], ni[1], 6, 1);
            hipLaunchKernelGGL(f.p3, dim3(g(2)), dim3(f.nt), 0, q, b->dinst, it[2], ni[2], stage == 0);
            if (stage == 0)
                hipLaunchKernelGGL(kb_set_h, dim3(cdiv(b->count, 64)), dim3(64), 0, q, b->dinst, b->count, f.n);
            hipLaunchKernelGGL(f.y, dim3(g(3)), dim3(f.nt), 0, q, b->dinst, it[3], ni[3], 3, 0);
            hipLaunchKernelGGL(f.p51, dim3(g(0)), dim3(f.nt), 0, q, b->dinst, it[0], ni[0],
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
        const BClassFns &f = b->cls_fns[c];
        const int ni = b->nitems[c][4];
        const unsigned g = (unsigned)std::max(1, std::min(b->cls_grid[c], ni));
        hipLaunchKernelGGL(f.p1, dim3(g), dim3(f.nt), 0, s, b->dinst, b->items[c][4], ni);
    }
    return launch_check("ensemble P1");
}

// Tile shape of a size class: the tuned one (tile table pass 8: a = threads per workgroup,
// v = persistent grid 256 << v), else 256 threads and 1024 workgroups; force_nt / force_grid
// (> 0) override both for every class.
static tk_status nsb_class_config(int n, int force_nt, int force_grid, BClassFns *f, int *grid) {
    const TileChoice c = tuned_tile(n, TK_F32, 8);
    int nt = c.a > 0 ? c.a : BNT;
    int G = c.a > 0 ? (256 << c.v) : 1024;
    if (force_nt > 0) nt = force_nt;
    if (force_grid > 0) G = force_grid;
    *f = class_fns(n, nt);
    if (!f->p1) return fail(TK_EUNSUPPORTED, "no ensemble kernels with %d threads for n=%d", nt, n);
    *grid = G;
    return TK_OK;
}

static tk_status nsb_create(tk_nsb_t *out, int count, const int *n, const double *nu, tk_dtype dt, double cfl,
                            unsigned flags, int force_nt) {
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
    const int force_grid = (int)(flags >> 16);  // persistent grid size override
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
    b->cls_fns.resize(sizes.size());
    b->cls_grid.resize(sizes.size());
    b->items.assign(sizes.size(), {nullptr, nullptr, nullptr, nullptr, nullptr});
    b->nitems.assign(sizes.size(), {0, 0, 0, 0, 0});
    for (size_t c = 0; c < sizes.size(); ++c) {
        tk_status st = nsb_class_config(sizes[c], force_nt, force_grid, &b->cls_fns[c], &b->cls_grid[c]);
        if (st != TK_OK) {
            nsb_free(b);
            return st;
        }
        const int W = b->cls_fns[c].W, LPW = b->cls_fns[c].LPW;
        for (int list = 0; list < 5; ++list) {
            std::vector<BItem> v;
            for (int i = 0; i < count; ++i) {
                const BInst &d = b->hinst[i];
                if (d.n != sizes[c]) continue;
                long nt = list == 0 ? tiles_x(W, d.K, d.KZP)
                          : list == 1 ? tiles_y(W, d.n, d.KZP, 6)
                          : list == 2 ? tiles_z(LPW, d.n)
                          : list == 3 ? tiles_y(W, d.n, d.KZP, 3)
                                      : tiles_x(W, d.K, d.KZP);
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

extern "C" tk_status ns_batch_create(tk_nsb_t *out, int count, const int *n, const double *nu, tk_dtype dt,
                                     double cfl, unsigned flags) {
    return nsb_create(out, count, n, nu, dt, cfl, flags, 0);
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

// ---- autotuning of the ensemble tiles ----------------------------------------------------------
// Steps of an ensemble on the member states u (device pointers), fixed step size dt: the
// per-call setup of ns_batch_step, then `iters` graph launches timed with HIP events.
static tk_status nsb_time_steps(tk_nsb_s *b, void *const *u, double dt, int iters, hipStream_t s, float *ms) {
    for (int i = 0; i < b->count; ++i) {
        b->hinst[i].u = (float2 *)u[i];
        NsState &h = b->hstate[i];
        h = NsState{};
        h.hfix = h.h = dt;
    }
    TK_HIP_CHECK(hipMemcpyAsync(b->dinst, b->hinst.data(), sizeof(BInst) * b->count, hipMemcpyHostToDevice, s));
    TK_HIP_CHECK(hipMemcpyAsync(b->dstate, b->hstate.data(), sizeof(NsState) * b->count, hipMemcpyHostToDevice, s));
    TK_TRY(nsb_p1(b, s));
    hipEvent_t e0, e1;
    TK_HIP_CHECK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(TK_EHIP, "hipEventCreate failed");
    }
    hipError_t e = hipEventRecord(e0, s);
    for (int k = 0; k < iters && e == hipSuccess; ++k) e = hipGraphLaunch(b->gexec, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return fail(TK_EHIP, "ensemble timing: %s", hipGetErrorString(e));
    *ms = t / std::max(1, iters);
    return TK_OK;
}

struct NsbTuneBufs {
    std::vector<void *> p;
    ~NsbTuneBufs() {
        for (void *q : p)
            if (q) hipFree(q);
    }
};

extern "C" tk_status ns_batch_autotune(int n, int members, int iters, char *report, int report_len) {
    if (!batch_size_ok(n)) return fail(TK_EUNSUPPORTED, "ensemble grid n=%d not in {16..128}", n);
    if (members < 1 || iters < 1) return fail(TK_EINVAL, "members and iters must be >= 1");
    hipStream_t s = nullptr;
    const size_t fb = (size_t)n * n * (n / 2 + 1) * sizeof(float2);
    NsbTuneBufs B;
    std::vector<void *> in(members), st(members), ref(members);
    NsGrid g;
    TK_TRY(ns_grid_init(&g, n, TK_F32));
    void *noise = nullptr, *dscr = nullptr;
    TK_HIP_CHECK(hipMalloc(&noise, 3 * (size_t)n * n * n * sizeof(float)));
    B.p.push_back(noise);
    TK_HIP_CHECK(hipMalloc(&dscr, sizeof(double) * (NS_DIAG_BLOCKS + 2) * (NS_DIAG_HEAD + ns_num_shells(n))));
    B.p.push_back(dscr);
    for (int i = 0; i < members; ++i) {
        TK_HIP_CHECK(hipMalloc(&in[i], 3 * fb));
        B.p.push_back(in[i]);
        TK_HIP_CHECK(hipMalloc(&st[i], 3 * fb));
        B.p.push_back(st[i]);
        TK_HIP_CHECK(hipMalloc(&ref[i], 3 * fb));
        B.p.push_back(ref[i]);
        TK_TRY(fill_pattern(noise, 3L * n * n * n, TK_F32, 4000u + i, s));
        TK_TRY(ns_init_random_grid(g, noise, in[i], 1.0, (double *)dscr, s));
    }
    std::vector<int> ns(members, n);
    std::vector<double> nus(members);
    for (int i = 0; i < members; ++i) nus[i] = 1e-3 * (1 + i % 4);
    const double dt = 1e-3;
    auto restore = [&]() -> tk_status {
        for (int i = 0; i < members; ++i) TK_HIP_CHECK(hipMemcpyAsync(st[i], in[i], 3 * fb, hipMemcpyDeviceToDevice, s));
        return TK_OK;
    };
    std::string rep;
    char line[256];
    float best = 1e30f;
    int bnt = 0, bgv = 0;
    bool have_ref = false;
    // the reference is the default shape (256 threads, 1024 workgroups), run first
    std::vector<std::pair<int, int>> cands = {{BNT, 2}};
    for (int v = 0; v < BNT_NVAR; ++v)
        for (int gv = 0; gv <= BGRID_MAXV; ++gv)
            if (!(BNT_VARIANTS[v] == BNT && gv == 2)) cands.push_back({BNT_VARIANTS[v], gv});
    for (const auto &c : cands) {
        const int nt = c.first, G = 256 << c.second;
        if (!class_fns(n, nt).p1) continue;
        tk_nsb_t b = nullptr;
        TK_TRY(nsb_create(&b, members, ns.data(), nus.data(), TK_F32, 0.0, (unsigned)G << 16, nt));
        tk_status stt = restore();
        float ms = 0;
        if (stt == TK_OK) stt = nsb_time_steps(b, st.data(), dt, 2, s, &ms);
        bool ok = true;
        if (stt == TK_OK && !have_ref) {
            for (int i = 0; i < members && stt == TK_OK; ++i)
                if (hipMemcpyAsync(ref[i], st[i], 3 * fb, hipMemcpyDeviceToDevice, s) != hipSuccess) stt = TK_EHIP;
            have_ref = true;
        } else if (stt == TK_OK) {
            double num = 0, den = 0;
            for (int i = 0; i < members && stt == TK_OK; ++i) {
                double a, d;
                stt = reduce_diff(st[i], ref[i], 6L * n * n * (n / 2 + 1), TK_F32, &a, &d, s);
                num += a;
                den += d;
            }
            ok = den > 0 && std::sqrt(num / den) <= 1e-5;
        }
        if (stt == TK_OK) stt = restore();
        if (stt == TK_OK) stt = nsb_time_steps(b, st.data(), dt, iters, s, &ms);
        nsb_free(b);
        TK_TRY(stt);
        snprintf(line, sizeof(line), "ensemble n=%d members=%d nt=%d grid=%d: %.4f ms/step %s\n", n, members, nt, G, ms,
                 ok ? "ok" : "REJECTED");
        rep += line;
        if (ok && ms < best) best = ms, bnt = nt, bgv = c.second;
    }
    if (bnt > 0) set_tuned_tile(n, TK_F32, 8, {bnt, default_E(n), bgv});
    snprintf(line, sizeof(line), "chosen pass 8 L=%d: a=%d E=%d v=%d (%.4f ms)\n", n, bnt, default_E(n), bgv, best);
    rep += line;
    TK_HIP_CHECK(hipStreamSynchronize(s));
    if (report && report_len > 0) {
        strncpy(report, rep.c_str(), report_len - 1);
        report[report_len - 1] = 0;
    }
    return TK_OK;
}

namespace tk {
bool batch_tile_ok(int n, int nt) { return batch_size_ok(n) && class_fns(n, nt).p1 != nullptr; }
}  // namespace tk
