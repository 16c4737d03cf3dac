// Pass kernels of the 3D transform (templates) and the launcher registry types.
//
// Z pass  (paper, Section "Parallelization Strategy", step 1): real lines of N points
//         along the contiguous z axis -> N/2+1 complex, as an N/2-point complex FFT of
//         the packed (even, odd) samples plus the real-FFT split; the inverse undoes it.
// Y and X passes (steps 3 and 5): complex transforms along a strided axis.  The layout
//         never changes (Appendix A's transpose-free scheme): a workgroup owns a tile of
//         W neighbouring columns x L points, so every global access is a run of W
//         consecutive complex values; the columns' points stay in registers and only the
//         exchanges between radix stages go through LDS.
#pragma once

#include "fft_core.hpp"

namespace tk {

// ---- registry types ------------------------------------------------------------------------
// Column c of a strided pass has its element i at  (c / CB) * SO + (c % CB) + i * SI
// (in complex elements).  Y pass: CB = nz/2+1, SO = ny CB, SI = CB.  X pass: CB = ny
// (nz/2+1), SO = nx CB, SI = CB.
struct StridedArgs {
    const void *src;
    void *dst;
    long ncols, CB, SO, SI;
    const void *tw;  // W_L^j table, L = line length
    int inv;         // 0: exp(-i..) forward; 1: exp(+i..) inverse
    double scale;    // applied on store
    // Row masks (used by the 2/3-dealiased solver): with kl >= 0 only rows r with
    // min(r, L - r) <= kl are read (the others are taken as zero); with ks >= 0 only such
    // rows are written.  -1: every row.
    int kl = -1, ks = -1;
    int rev = 0;  // sweep the columns from the last one (see sweep_tile)
};
using StridedFn = void (*)(const StridedArgs &, hipStream_t);

// var 0: one tile per workgroup, one sweep over the tiles; var 1..3: persistent workgroups
// with the next tile's loads issued ahead (k_strided_pp), tile order var; var 4: one tile
// per workgroup, each XCD sweeping its own eighth of the tiles; var 5, 6: as 0 and 4 with
// split exchanges (real and imaginary parts in turn through half the LDS); var 7..9: as
// 1..3 with the registers held to what two resident workgroups per CU allow.
struct StridedKernel {
    int L;
    tk_dtype dt;
    int W, E, nt, lds;
    StridedFn fn;
    int var;
};

struct ZArgs {
    const void *src;
    void *dst;
    long nlines;
    const void *tw;  // W_N^j table, N = real line length
    double scale;    // r2c only
    int rev = 0;     // sweep the lines from the last one (see sweep_tile)
};
using ZFn = void (*)(const ZArgs &, hipStream_t);

struct ZKernel {
    int N;
    tk_dtype dt;
    int LPW, E, nt, lds;
    ZFn r2c, c2r;
};

const std::vector<StridedKernel> &strided_kernels();
const std::vector<ZKernel> &z_kernels();

// Sine / cosine transforms along a strided axis (same column addressing as StridedArgs).
struct R2RArgs {
    const void *src;
    void *dst;
    long ncols, CB, SO, SI;
    const void *tw;   // W_L^j
    const void *twq;  // W_{4L}^j, j < L
    int kind;         // 0 DCT-II, 1 DST-II (forward), 2 DCT-III, 3 DST-III (inverse)
    double scale;
};
using R2RFn = void (*)(const R2RArgs &, hipStream_t);
struct R2RKernel {
    int L;
    tk_dtype dt;
    int W, E;
    R2RFn fn;
};
const std::vector<R2RKernel> &r2r_kernels();

// Sine / cosine transforms along the contiguous z axis of real data: npairs pairs of
// consecutive real lines of L points (lines 2p and 2p + 1), src -> dst (not in place).
struct ZR2RArgs {
    const void *src;
    void *dst;
    long npairs;
    const void *tw;   // W_L^j
    const void *twq;  // W_{4L}^j, j < L
    int kind;         // 0 DCT-II, 1 DST-II (forward), 2 DCT-III, 3 DST-III (inverse)
    double scale;
};
using ZR2RFn = void (*)(const ZR2RArgs &, hipStream_t);
struct ZR2RKernel {
    int L;
    tk_dtype dt;
    ZR2RFn fn;
};
const std::vector<ZR2RKernel> &z_r2r_kernels();

#define TK_FOR_EACH_LEN(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

// ---- strided complex pass ----------------------------------------------------------------------
template <int L, int E, int W> constexpr int strided_es() { return W + 1; }

__device__ __forceinline__ bool row_kept(int r, int L, int k) { return k < 0 || r <= k || r >= L - k; }

// Addressing of one column tile (columns c0 .. c0 + width - 1, width <= W) for thread
// (col, jt) = (tid % W, tid / W), which handles the points x[jt + i TPL] of column c0 + col:
// point i sits at element tb + i TPL SI + lo / sizeof(C), where tb (the tile's first
// element) is uniform over the workgroup and lo is a 32-bit byte offset, so a load is one
// scalar base plus one vector offset and a thread keeps a single address register.
// lo < 2^31 for every supported grid: a tile spans at most (W - 1) / CB + 2 planes of SO
// elements plus L rows of SI, under 300 MB for lengths up to 1024.  Lanes outside the
// tile get lo = 0 (a valid address whose value they discard).
struct TileAddr {
    long tb;
    unsigned lo;
    bool valid;
};

template <typename T, int W>
__device__ __forceinline__ TileAddr tile_addr(long c0, int width, long ncols, long CB, long SO, long SI) {
    const int col = threadIdx.x % W;
    const int jt = threadIdx.x / W;
    const long c = c0 + col;
    const bool valid = col < width && c < ncols;
    const long tb = (c0 / CB) * SO + c0 % CB;
    const long e = valid ? (c / CB) * SO + c % CB - tb + (long)jt * SI : 0;
    return {tb, (unsigned)(e * (long)sizeof(V2<T>)), valid};
}

template <typename P> __device__ __forceinline__ const P *at_bytes(const P *p, unsigned lo) {
    return reinterpret_cast<const P *>(reinterpret_cast<const char *>(p) + lo);
}
template <typename P> __device__ __forceinline__ P *at_bytes(P *p, unsigned lo) {
    return reinterpret_cast<P *>(reinterpret_cast<char *>(p) + lo);
}

// v[i] = x[jt + i TPL] of the thread's column.  MASK: rows outside the kl mask (and
// columns outside the tile) read as zero without touching memory.  Without MASK every
// row is read, branch-free: a lane outside the tile reads the tile's first column and
// transforms it in its own LDS column, and its result is never stored.
template <typename T, int L, int E, int W, bool MASK>
__device__ __forceinline__ void strided_load(V2<T> (&v)[E], const V2<T> *src, const TileAddr &a, long SI,
                                             int kl) {
    constexpr int TPL = L / E;
    const int jt = threadIdx.x / W;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const V2<T> *row = src + a.tb + (long)(i * TPL) * SI;
        if constexpr (MASK) {
            v[i] = (a.valid && row_kept(jt + i * TPL, L, kl)) ? *at_bytes(row, a.lo) : mk<T>(0, 0);
        } else {
            v[i] = *at_bytes(row, a.lo);
        }
    }
}

// Stores of the transformed points, conjugated back for the inverse and scaled; with
// MASK only rows inside the ks mask are written.
template <typename T, int L, int E, int W, bool MASK>
__device__ __forceinline__ void strided_store(const V2<T> (&v)[E], V2<T> *dst, const TileAddr &a, long SI, int inv,
                                              T scale, int ks) {
    constexpr int TPL = L / E;
    const int jt = threadIdx.x / W;
    if (!a.valid) return;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        V2<T> x = v[i];
        if (inv) x.y = -x.y;
        x.x *= scale;
        x.y *= scale;
        V2<T> *row = dst + a.tb + (long)(i * TPL) * SI;
        if (!MASK || row_kept(jt + i * TPL, L, ks)) *at_bytes(row, a.lo) = x;
    }
}

// One column tile: W columns x L points.  lds: L (W + 1) complex for the exchanges (SPLIT:
// L (W + 1) scalars); tw: the W_L^j table already in LDS.  Contains barriers: every thread
// calls it.
template <typename T, int L, int E, int W, bool MASK = true, bool SPLIT = false>
__device__ __forceinline__ void strided_tile(const V2<T> *src, V2<T> *dst, long ncols, long CB, long SO, long SI,
                                             int inv, T scale, int kl, int ks, long tile, V2<T> *lds,
                                             const V2<T> *tw) {
    using C = V2<T>;
    constexpr int ES = strided_es<L, E, W>();
    const TileAddr a = tile_addr<T, W>(tile * W, W, ncols, CB, SO, SI);
    C v[E];
    strided_load<T, L, E, W, MASK>(v, src, a, SI, kl);
    if (inv) {
#pragma unroll
        for (int i = 0; i < E; ++i) v[i].y = -v[i].y;
    }
    C *d = SPLIT ? reinterpret_cast<C *>(reinterpret_cast<T *>(lds) + threadIdx.x % W) : lds + threadIdx.x % W;
    line_fft<T, L, E, ES, 1, 0, false, SPLIT>(v, d, threadIdx.x / W, tw);
    strided_store<T, L, E, W, MASK>(v, dst, a, SI, inv, scale, ks);
}

template <typename T, int L, int E, int W> constexpr int strided_lds_elems() { return L * strided_es<L, E, W>(); }

template <typename T, int L, int E, int W, bool MASK, bool SPLIT = false>
__global__ __launch_bounds__(W *(L / E)) void k_strided(const V2<T> *src, V2<T> *dst, long ncols, long CB,
                                                         long SO, long SI, const V2<T> *__restrict__ twg,
                                                         int inv, T scale, int kl, int ks, int rev,
                                                         int regions) {
    using C = V2<T>;
    constexpr int NT = W * (L / E);
    __shared__ C lds[SPLIT ? (strided_lds_elems<T, L, E, W>() + 1) / 2 : strided_lds_elems<T, L, E, W>()];
    __shared__ C tw[L];
    load_twiddles<T>(tw, twg, L, threadIdx.x, NT);
    __syncthreads();
    // regions: each XCD sweeps its own eighth of the tiles (the 8 sweeps run side by side)
    unsigned t = regions ? xcd_tile(blockIdx.x, gridDim.x) : sweep_tile(blockIdx.x, gridDim.x, 0);
    if (rev) t = gridDim.x - 1 - t;
    strided_tile<T, L, E, W, MASK, SPLIT>(src, dst, ncols, CB, SO, SI, inv, scale, kl, ks, t, lds, tw);
}

// Row masks select the MASK instantiation; plain transforms run the branch-free one.
// REGIONS: tile order by XCD regions instead of one sweep (variants 4, 6); SPLIT: the
// exchanges move real and imaginary parts separately through half the LDS (5, 6).
template <typename T, int L, int E, int W, int REGIONS = 0, bool SPLIT = false>
void launch_strided(const StridedArgs &a, hipStream_t s) {
    constexpr int NT = W * (L / E);
    unsigned nb = cdiv(a.ncols, W);
    if (a.kl >= 0 || a.ks >= 0)
        hipLaunchKernelGGL((k_strided<T, L, E, W, true, SPLIT>), dim3(nb), dim3(NT), 0, s, (const V2<T> *)a.src,
                           (V2<T> *)a.dst, a.ncols, a.CB, a.SO, a.SI, (const V2<T> *)a.tw, a.inv, (T)a.scale, a.kl,
                           a.ks, a.rev, REGIONS);
    else
        hipLaunchKernelGGL((k_strided<T, L, E, W, false, SPLIT>), dim3(nb), dim3(NT), 0, s, (const V2<T> *)a.src,
                           (V2<T> *)a.dst, a.ncols, a.CB, a.SO, a.SI, (const V2<T> *)a.tw, a.inv, (T)a.scale, a.kl,
                           a.ks, a.rev, REGIONS);
}

// ---- persistent strided pass ----------------------------------------------------------------------
// G workgroups (as many as are resident on the chip at once) share the tiles: each takes q
// full tiles, then at most one narrow tail tile of wt columns, so the columns left after
// the last full round are spread over every workgroup instead of idling most of the chip
// behind a few whole tiles.  The loads of the next tile are issued before the current
// tile's transform: a workgroup barrier waits for LDS traffic only, so they stay in flight
// across the exchanges.  Tiles of a workgroup never share columns, so an in-place pass
// stays correct.  The order in which the tiles are dealt decides which columns are in
// flight together, and with it how well the rows' DRAM pages and the XCDs' L2s are used;
// the best one depends on the row pitch, so it is a tuning choice:
//   order 1: round k takes tiles k G .. k G + G - 1, workgroup g the (k G + g)-th;
//   order 2: as 1, with the workgroups numbered XCD by XCD (they are dealt to the 8 XCDs
//            in turn), so each XCD takes a contiguous run of a round's tiles;
//   order 3: workgroup g takes the consecutive tiles g q .. g q + q - 1.
// WPE: waves per SIMD the register allocation must leave room for (1: no limit; the
// variants with two resident workgroups per CU ask for 2 NT / 256).
template <typename T, int L, int E, int W, bool MASK, int WPE>
__global__ __launch_bounds__(W *(L / E)) __attribute__((amdgpu_waves_per_eu(WPE))) void k_strided_pp(const V2<T> *src, V2<T> *dst, long ncols, long CB,
                                                            long SO, long SI, const V2<T> *__restrict__ twg,
                                                            int inv, T scale, int kl, int ks, long q, int wt,
                                                            int ntail, int order, int rev) {
    using C = V2<T>;
    constexpr int NT = W * (L / E);
    constexpr int ES = strided_es<L, E, W>();
    __shared__ C lds[strided_lds_elems<T, L, E, W>()];
    __shared__ C tw[L];
    load_twiddles<T>(tw, twg, L, threadIdx.x, NT);
    __syncthreads();
    const long G = gridDim.x;
    const long g = (order == 2 && (G & 7) == 0) ? (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    const bool has_tail = g < ntail;
    const long nu = q + (has_tail ? 1 : 0);
    // unit u -> round (q = the tail); rev runs the tail first, then the rounds backwards
    auto round_of = [&](long u) { return !rev ? u : (has_tail ? (u == 0 ? q : q - u) : q - 1 - u); };
    auto addr_of = [&](long u) {
        const long k = round_of(u);
        return k < q ? tile_addr<T, W>((order == 3 ? g * q + k : k * G + g) * W, W, ncols, CB, SO, SI)
                     : tile_addr<T, W>(q * G * W + g * wt, wt, ncols, CB, SO, SI);
    };
    C nx[E];
    TileAddr an = addr_of(0);
    if (nu > 0) strided_load<T, L, E, W, MASK>(nx, src, an, SI, kl);
    for (long u = 0; u < nu; ++u) {
        const TileAddr a = an;
        C v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = nx[i];
        if (u + 1 < nu) {
            an = addr_of(u + 1);
            strided_load<T, L, E, W, MASK>(nx, src, an, SI, kl);
        }
        if (inv) {
#pragma unroll
            for (int i = 0; i < E; ++i) v[i].y = -v[i].y;
        }
        line_fft<T, L, E, ES>(v, lds + threadIdx.x % W, threadIdx.x / W, tw);
        strided_store<T, L, E, W, MASK>(v, dst, a, SI, inv, scale, ks);
    }
}

// Number of workgroups of `kernel` (nt threads) resident on the current device at once.
int resident_groups(const void *kernel, int nt);

template <typename T, int L, int E, int W, int ORDER, int WPE = 1>
void launch_strided_pp(const StridedArgs &a, hipStream_t s) {
    constexpr int NT = W * (L / E);
    const bool mask = a.kl >= 0 || a.ks >= 0;
    const void *kp = mask ? reinterpret_cast<const void *>(&k_strided_pp<T, L, E, W, true, WPE>)
                          : reinterpret_cast<const void *>(&k_strided_pp<T, L, E, W, false, WPE>);
    const long G = resident_groups(kp, NT);
    const long q = (a.ncols / W) / G;
    const long left = a.ncols - q * G * W;
    int wt = W, ntail = 0;
    if (left > 0) {
        long w = (left + G - 1) / G;
        w = (w + 7) / 8 * 8;
        wt = (int)(w < W ? w : W);
        ntail = (int)((left + wt - 1) / wt);
    }
    if (mask)
        hipLaunchKernelGGL((k_strided_pp<T, L, E, W, true, WPE>), dim3((unsigned)G), dim3(NT), 0, s,
                           (const V2<T> *)a.src, (V2<T> *)a.dst, a.ncols, a.CB, a.SO, a.SI, (const V2<T> *)a.tw,
                           a.inv, (T)a.scale, a.kl, a.ks, q, wt, ntail, ORDER, a.rev);
    else
        hipLaunchKernelGGL((k_strided_pp<T, L, E, W, false, WPE>), dim3((unsigned)G), dim3(NT), 0, s,
                           (const V2<T> *)a.src, (V2<T> *)a.dst, a.ncols, a.CB, a.SO, a.SI, (const V2<T> *)a.tw,
                           a.inv, (T)a.scale, a.kl, a.ks, q, wt, ntail, ORDER, a.rev);
}

// ---- Z pass: real lines <-> half spectra ----------------------------------------------------------
// Thread (ln, jt) of a workgroup handles line l0 + ln, points jt + i TPL of the L = N/2
// complex values z[n] = x[2n] + i x[2n+1].
// r2c split:  X[k] = 1/2 (Z[k] + conj Z[L-k]) - i/2 W_N^k (Z[k] - conj Z[L-k]),  k < L;
//             X[L] = Re Z[0] - Im Z[0].
// c2r merge:  Z'[k] = (X[k] + conj X[L-k]) + i conj(W_N^k) (X[k] - conj X[L-k]), with
//             only the real parts of X[0] and X[L] taken; z = sum_k Z'[k] exp(+2 pi i kn/L)
//             done as conj(DFT(conj Z')); x[2n] = Re z[n], x[2n+1] = Im z[n].
template <typename T, int L, int E, int LPW>
__global__ __launch_bounds__(LPW *(L / E)) void k_z_r2c(const T *__restrict__ src, V2<T> *__restrict__ dst,
                                                         long nlines, const V2<T> *__restrict__ twg, T scale,
                                                         int rev) {
    using C = V2<T>;
    constexpr int TPL = L / E;
    constexpr int NT = LPW * TPL;
    constexpr int LL = lds_line_len<L>();
    constexpr int NZH = L + 1;
    __shared__ C lds[LPW * LL];
    __shared__ C tw[2 * L];
    const int tid = threadIdx.x;
    const int ln = tid / TPL;
    const int jt = tid % TPL;
    const long l = (long)sweep_tile(blockIdx.x, gridDim.x, rev) * LPW + ln;
    const bool valid = l < nlines;
    const C *s2 = reinterpret_cast<const C *>(src) + l * L;
    C v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = valid ? s2[jt + i * TPL] : mk<T>(0, 0);
    load_twiddles<T>(tw, twg, 2 * L, tid, NT);
    __syncthreads();
    C *d = lds + ln * LL;
    line_fft<T, L, E, 1, 2>(v, d, jt, tw);
    C zm[E];
    mirror<T, L, E>(v, zm, jt);
    if (valid) {
        C *o = dst + l * NZH;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int k = jt + i * TPL;
            const C zk = v[i];
            const C a = cadd(zk, cconj(zm[i]));
            const C b = cmul(tw[k], csub(zk, cconj(zm[i])));
            C x;
            x.x = (T)0.5 * (a.x + b.y) * scale;
            x.y = (T)0.5 * (a.y - b.x) * scale;
            o[k] = x;
        }
        if (jt == 0) o[L] = mk<T>((v[0].x - v[0].y) * scale, (T)0);
    }
}

template <typename T, int L, int E, int LPW>
__global__ __launch_bounds__(LPW *(L / E)) void k_z_c2r(const V2<T> *__restrict__ src, T *__restrict__ dst,
                                                         long nlines, const V2<T> *__restrict__ twg, int rev) {
    using C = V2<T>;
    constexpr int TPL = L / E;
    constexpr int NT = LPW * TPL;
    constexpr int LL = lds_line_len<L>();
    constexpr int NZH = L + 1;
    __shared__ C lds[LPW * LL];
    __shared__ C tw[2 * L];
    const int tid = threadIdx.x;
    const int ln = tid / TPL;
    const int jt = tid % TPL;
    const long l = (long)sweep_tile(blockIdx.x, gridDim.x, rev) * LPW + ln;
    const bool valid = l < nlines;
    const C *s = src + (valid ? l : 0) * NZH;
    C v[E], xm[E];
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = valid ? s[jt + i * TPL] : mk<T>(0, 0);
    const C xl = (valid && jt == 0) ? s[L] : mk<T>(0, 0);  // Nyquist entry X[L]
    load_twiddles<T>(tw, twg, 2 * L, tid, NT);
    mirror<T, L, E>(v, xm, jt);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int k = jt + i * TPL;
        C xk = v[i];
        C xc = cconj(k == 0 ? xl : xm[i]);
        if (k == 0) {
            xk.y = 0;
            xc.y = 0;
        }
        const C a = cadd(xk, xc);
        const C b = cmul(cconj(tw[k]), csub(xk, xc));
        v[i] = mk<T>(a.x - b.y, -(a.y + b.x));  // conj(Z')
    }
    C *d = lds + ln * LL;
    line_fft<T, L, E, 1, 2>(v, d, jt, tw);
    if (valid) {
        C *o = reinterpret_cast<C *>(dst) + l * L;
#pragma unroll
        for (int i = 0; i < E; ++i) o[jt + i * TPL] = mk<T>(v[i].x, -v[i].y);
    }
}

template <typename T, int L, int E, int LPW>
void launch_z_r2c(const ZArgs &a, hipStream_t s) {
    constexpr int NT = LPW * (L / E);
    unsigned nb = cdiv(a.nlines, LPW);
    hipLaunchKernelGGL((k_z_r2c<T, L, E, LPW>), dim3(nb), dim3(NT), 0, s, (const T *)a.src, (V2<T> *)a.dst,
                       a.nlines, (const V2<T> *)a.tw, (T)a.scale, a.rev);
}

template <typename T, int L, int E, int LPW>
void launch_z_c2r(const ZArgs &a, hipStream_t s) {
    constexpr int NT = LPW * (L / E);
    unsigned nb = cdiv(a.nlines, LPW);
    hipLaunchKernelGGL((k_z_c2r<T, L, E, LPW>), dim3(nb), dim3(NT), 0, s, (const V2<T> *)a.src, (T *)a.dst,
                       a.nlines, (const V2<T> *)a.tw, a.rev);
}

// ---- tile-shape candidates ----------------------------------------------------------------------------
// Strided pass candidate (ce, cn): E = default_E(L) << ce points per thread, NT = 256 << cn
// threads, W = NT E / L columns; kept when W is a whole number and the LDS tile fits the 160 KB of a CU.
template <typename T> constexpr int strided_lds(int L, int W) { return (L * (W + 1) + L) * 2 * (int)sizeof(T); }
template <typename T> constexpr bool strided_cand_ok(int L, int ce, int cn) {
    int E = default_E(L) << ce;
    int NT = 256 << cn;
    if (E > L || !rplan_ok(L, E)) return false;
    if ((NT * E) % L != 0) return false;
    int W = NT * E / L;
    if (W < 1 || W * (L / E) != NT) return false;
    return strided_lds<T>(L, W) <= 163840;
}
// Z pass candidate (ce, cn): E = default_E(N/2) << ce, NT = 256 << cn threads (or one line).
template <typename T> constexpr bool z_cand_ok(int N, int ce, int cn) {
    int L = N / 2;
    int E = default_E(L) << ce;
    if (E > L || !rplan_ok(L, E)) return false;
    int TPL = L / E;
    int NT = 256 << cn;
    int LPW = NT / TPL;
    if (LPW < 1 || LPW * TPL != NT) return false;
    return (long)(LPW * (L + L / 32 + 1) + 2 * L) * 2 * (long)sizeof(T) <= 163840;
}

}  // namespace tk
