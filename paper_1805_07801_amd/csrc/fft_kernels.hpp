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
};
using StridedFn = void (*)(const StridedArgs &, hipStream_t);

struct StridedKernel {
    int L;
    tk_dtype dt;
    int W, E, nt, lds;
    StridedFn fn;
};

struct ZArgs {
    const void *src;
    void *dst;
    long nlines;
    const void *tw;  // W_N^j table, N = real line length
    double scale;    // r2c only
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

#define TK_FOR_EACH_LEN(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

// ---- strided complex pass ----------------------------------------------------------------------
template <int L, int E, int W> constexpr int strided_es() { return W + 1; }

__device__ __forceinline__ bool row_kept(int r, int L, int k) { return k < 0 || r <= k || r >= L - k; }

// One column tile: W columns x L points.  lds: L (W + 1) complex for the exchanges;
// tw: the W_L^j table already in LDS.  Contains barriers: every thread calls it.
template <typename T, int L, int E, int W>
__device__ __forceinline__ void strided_tile(const V2<T> *src, V2<T> *dst, long ncols, long CB, long SO, long SI,
                                             int inv, T scale, int kl, int ks, long tile, V2<T> *lds,
                                             const V2<T> *tw) {
    using C = V2<T>;
    constexpr int TPL = L / E;
    constexpr int ES = strided_es<L, E, W>();
    const int tid = threadIdx.x;
    const int col = tid % W;
    const int jt = tid / W;
    const long c = tile * W + col;
    const bool valid = c < ncols;
    const long base = valid ? (c / CB) * SO + (c % CB) : 0;
    C v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int r = jt + i * TPL;
        C x = (valid && row_kept(r, L, kl)) ? src[base + (long)r * SI] : mk<T>(0, 0);
        if (inv) x.y = -x.y;
        v[i] = x;
    }
    line_fft<T, L, E, ES>(v, lds + col, jt, tw);
    if (valid) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int r = jt + i * TPL;
            C x = v[i];
            if (inv) x.y = -x.y;
            x.x *= scale;
            x.y *= scale;
            if (row_kept(r, L, ks)) dst[base + (long)r * SI] = x;
        }
    }
}

template <typename T, int L, int E, int W> constexpr int strided_lds_elems() { return L * strided_es<L, E, W>(); }

template <typename T, int L, int E, int W>
__global__ __launch_bounds__(W *(L / E)) void k_strided(const V2<T> *src, V2<T> *dst, long ncols, long CB,
                                                         long SO, long SI, const V2<T> *__restrict__ twg,
                                                         int inv, T scale, int kl, int ks) {
    using C = V2<T>;
    constexpr int NT = W * (L / E);
    __shared__ C lds[strided_lds_elems<T, L, E, W>()];
    __shared__ C tw[L];
    load_twiddles<T>(tw, twg, L, threadIdx.x, NT);
    __syncthreads();
    strided_tile<T, L, E, W>(src, dst, ncols, CB, SO, SI, inv, scale, kl, ks, xcd_tile(blockIdx.x, gridDim.x), lds,
                             tw);
}

template <typename T, int L, int E, int W>
void launch_strided(const StridedArgs &a, hipStream_t s) {
    constexpr int NT = W * (L / E);
    unsigned nb = cdiv(a.ncols, W);
    hipLaunchKernelGGL((k_strided<T, L, E, W>), dim3(nb), dim3(NT), 0, s, (const V2<T> *)a.src, (V2<T> *)a.dst,
                       a.ncols, a.CB, a.SO, a.SI, (const V2<T> *)a.tw, a.inv, (T)a.scale, a.kl, a.ks);
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
                                                         long nlines, const V2<T> *__restrict__ twg, T scale) {
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
    const long l = (long)xcd_tile(blockIdx.x, gridDim.x) * LPW + ln;
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
                                                         long nlines, const V2<T> *__restrict__ twg) {
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
    const long l = (long)xcd_tile(blockIdx.x, gridDim.x) * LPW + ln;
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
                       a.nlines, (const V2<T> *)a.tw, (T)a.scale);
}

template <typename T, int L, int E, int LPW>
void launch_z_c2r(const ZArgs &a, hipStream_t s) {
    constexpr int NT = LPW * (L / E);
    unsigned nb = cdiv(a.nlines, LPW);
    hipLaunchKernelGGL((k_z_c2r<T, L, E, LPW>), dim3(nb), dim3(NT), 0, s, (const V2<T> *)a.src, (T *)a.dst,
                       a.nlines, (const V2<T> *)a.tw);
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
