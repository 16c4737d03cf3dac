// Pass kernels of the 3D transform (templates) and the launcher registry types.
//
// Z pass  (paper, Section "Parallelization Strategy", step 1): real lines of N points
//         along the contiguous z axis -> N/2+1 complex, as an N/2-point complex FFT of
//         the packed (even, odd) samples plus the real-FFT split; the inverse undoes it.
// Y and X passes (steps 3 and 5): complex transforms along a strided axis.  The layout
//         never changes (Appendix A's transpose-free scheme): a workgroup stages a tile
//         of W neighbouring columns x L points in LDS, so every global access is a run
//         of W consecutive complex values.
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

// ---- strided complex pass ----------------------------------------------------------------------
template <typename T, int L, int E, int W>
__global__ __launch_bounds__(W *(L / E)) void k_strided(const V2<T> *src, V2<T> *dst, long ncols, long CB,
                                                         long SO, long SI, const V2<T> *__restrict__ tw,
                                                         int inv, T scale) {
    using C = V2<T>;
    constexpr int TPL = L / E;
    constexpr int ES = W;
    __shared__ C lds[L * ES];
    const int tid = threadIdx.x;
    const int col = tid % W;
    const int jt = tid / W;
    const long c = (long)xcd_tile(blockIdx.x, gridDim.x) * W + col;
    const bool valid = c < ncols;
    const long base = valid ? (c / CB) * SO + (c % CB) : 0;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int row = jt + i * TPL;
        C v = valid ? src[base + row * SI] : mk<T>(0, 0);
        if (inv) v.y = -v.y;
        lds[row * ES + col] = v;
    }
    __syncthreads();
    line_fft<T, L, E, ES, 1>(lds + col, jt, tw);
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int row = jt + i * TPL;
        C v = lds[row * ES + col];
        if (inv) v.y = -v.y;
        v.x *= scale;
        v.y *= scale;
        if (valid) dst[base + row * SI] = v;
    }
}

template <typename T, int L, int E, int W>
void launch_strided(const StridedArgs &a, hipStream_t s) {
    constexpr int NT = W * (L / E);
    unsigned nb = cdiv(a.ncols, W);
    hipLaunchKernelGGL((k_strided<T, L, E, W>), dim3(nb), dim3(NT), 0, s, (const V2<T> *)a.src, (V2<T> *)a.dst,
                       a.ncols, a.CB, a.SO, a.SI, (const V2<T> *)a.tw, a.inv, (T)a.scale);
}

// ---- Z pass: real lines <-> half spectra ----------------------------------------------------------
// LDS line stride: L + 1 entries (room for the Nyquist value of the c2r input).
template <typename T, int L, int E, int LPW>
__global__ __launch_bounds__(LPW *(L / E)) void k_z_r2c(const T *__restrict__ src, V2<T> *__restrict__ dst,
                                                         long nlines, const V2<T> *__restrict__ tw, T scale) {
    using C = V2<T>;
    constexpr int TPL = L / E;
    constexpr int NT = LPW * TPL;
    constexpr int LS = L + 1;
    constexpr int NZH = L + 1;
    __shared__ C lds[LPW * LS];
    const int tid = threadIdx.x;
    const long l0 = (long)xcd_tile(blockIdx.x, gridDim.x) * LPW;
    const long avail = nlines - l0;
    const C *s2 = reinterpret_cast<const C *>(src) + l0 * L;
    for (int q = tid; q < LPW * L; q += NT) {
        const int ln = q / L;
        C v = (ln < avail) ? s2[q] : mk<T>(0, 0);
        lds[ln * LS + (q - ln * L)] = v;
    }
    __syncthreads();
    const int ln = tid / TPL;
    const int jt = tid % TPL;
    C *d = lds + ln * LS;
    line_fft<T, L, E, 1, 2>(d, jt, tw);
    // split: X[k] = 1/2 (Z[k] + conj Z[L-k]) - i/2 W_N^k (Z[k] - conj Z[L-k]),  X[L] = Re Z0 - Im Z0
    if (ln < avail) {
        C *o = dst + (l0 + ln) * NZH;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int k = jt + i * TPL;
            const C zk = d[k];
            const C zm = cconj(d[(L - k) % L]);
            const C a = cadd(zk, zm);
            const C b = cmul(tw[k], csub(zk, zm));
            C x;
            x.x = (T)0.5 * (a.x + b.y);
            x.y = (T)0.5 * (a.y - b.x);
            x.x *= scale;
            x.y *= scale;
            o[k] = x;
        }
        if (jt == 0) {
            const C z0 = d[0];
            o[L] = mk<T>((z0.x - z0.y) * scale, (T)0);
        }
    }
}

template <typename T, int L, int E, int LPW>
__global__ __launch_bounds__(LPW *(L / E)) void k_z_c2r(const V2<T> *__restrict__ src, T *__restrict__ dst,
                                                         long nlines, const V2<T> *__restrict__ tw) {
    using C = V2<T>;
    constexpr int TPL = L / E;
    constexpr int NT = LPW * TPL;
    constexpr int LS = L + 1;
    constexpr int NZH = L + 1;
    __shared__ C lds[LPW * LS];
    const int tid = threadIdx.x;
    const long l0 = (long)xcd_tile(blockIdx.x, gridDim.x) * LPW;
    const long avail = nlines - l0;
    const C *s = src + l0 * NZH;
    for (int q = tid; q < LPW * NZH; q += NT) {
        const int ln = q / NZH;
        C v = (ln < avail) ? s[q] : mk<T>(0, 0);
        lds[ln * LS + (q - ln * NZH)] = v;
    }
    __syncthreads();
    const int ln = tid / TPL;
    const int jt = tid % TPL;
    C *d = lds + ln * LS;
    // merge: Z'[k] = (X[k] + conj X[L-k]) + i conj(W_N^k) (X[k] - conj X[L-k]); only the real
    // parts of X[0] and X[L] enter.  The inverse DFT is done as conj(DFT(conj .)).
    C zr[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int k = jt + i * TPL;
        C xk = d[k];
        C xm = cconj(d[L - k]);
        if (k == 0) {
            xk.y = 0;
            xm.y = 0;
        }
        const C a = cadd(xk, xm);
        const C b = cmul(cconj(tw[k]), csub(xk, xm));
        C z;
        z.x = a.x - b.y;
        z.y = a.y + b.x;
        zr[i] = cconj(z);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < E; ++i) d[jt + i * TPL] = zr[i];
    __syncthreads();
    line_fft<T, L, E, 1, 2>(d, jt, tw);
    C *o = reinterpret_cast<C *>(dst) + l0 * L;
    for (int q = tid; q < LPW * L; q += NT) {
        const int l = q / L;
        if (l < avail) {
            C v = lds[l * LS + (q - l * L)];
            v.y = -v.y;
            o[q] = v;
        }
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
// Strided pass: W columns per workgroup, NT = W L / E threads.  Candidate c (0, 1, 2) uses
// W = Wb << c with Wb = max(4, 64 E / L), kept when NT <= 1024 and the tile fits 64 KB.
constexpr int strided_Wb(int L, int E) { return (64 * E / L) > 4 ? (64 * E / L) : 4; }
template <typename T> constexpr bool strided_ok(int L, int E, int W) {
    return W * (L / E) <= 1024 && W * (L / E) >= 64 && (long)L * W * 2 * sizeof(T) <= 65536;
}
// Z pass: LPW lines per workgroup so that NT = LPW L / E is 256 threads (or one line).
constexpr int z_LPW(int L, int E) { return (256 / (L / E)) > 1 ? (256 / (L / E)) : 1; }

}  // namespace tk
