// Sine / cosine transforms along a strided axis (the paper's free-slip bases, Section
// "Fast Fourier Transform": 2 sin(ks), 2 cos(ks); the SFF and SSF combinations).
//
// On an axis of N points x_j = pi (j + 1/2) / N the forward transform is the DCT-II /
// DST-II with 1/N (cosine: F_k = (1/N) sum_j f_j cos(k x_j), k = 0..N-1; sine: k = 1..N
// stored at index k - 1), the inverse the matching DCT-III / DST-III (f = F_0 + sum 2 F_k
// cos(k x) ; f = sum_{k<N} 2 F_k sin(k x) + F_N sin(N x)).  Each is one N-point complex FFT
// (Makhoul's even/odd reordering): forward, v_m = g_{2m}, v_{N-1-m} = g_{2m+1}, V = DFT(v),
// C_k = Re(w_k A_k) + i Re(w_k B_k) with A, B the transforms of the real and imaginary
// parts split from V_k and conj V_{N-k}, w_k = exp(-i pi k / 2N); inverse,
// V_k = conj(w_k) (X_k - i X_{N-k}), v = sum_k V_k exp(+2 pi i km/N), g from v by the same
// reordering.  The sine transforms are the cosine ones of (-1)^j g with the coefficient
// index reversed.  Complex data: every transform is real-linear, so real and imaginary parts
// go through together.
#include "fft_api.hpp"

namespace tk {

enum R2RKind : int { DCT_FWD = 0, DST_FWD = 1, DCT_INV = 2, DST_INV = 3 };

template <int L> __device__ __forceinline__ int makhoul_row(int m) { return m < L / 2 ? 2 * m : 2 * (L - 1 - m) + 1; }
template <int L> __device__ __forceinline__ int sine_row(int k) { return k == 0 ? L - 1 : L - 1 - k; }

template <typename T, int L, int E, int W>
__global__ __launch_bounds__(W *(L / E)) void k_r2r(const V2<T> *src, V2<T> *dst, long ncols, long CB, long SO,
                                                     long SI, const V2<T> *__restrict__ twg,
                                                     const V2<T> *__restrict__ twqg, int kind, T scale) {
    using C = V2<T>;
    constexpr int TPL = L / E;
    constexpr int NT = W * TPL;
    constexpr int ES = W + 1;
    __shared__ C lds[L * ES];
    __shared__ C tw[L];
    __shared__ C twq[L];
    const int tid = threadIdx.x;
    load_twiddles<T>(tw, twg, L, tid, NT);
    load_twiddles<T>(twq, twqg, L, tid, NT);  // exp(-i pi k / 2L), k < L
    const int col = tid % W;
    const int jt = tid / W;
    const long c = (long)xcd_tile(blockIdx.x, gridDim.x) * W + col;
    const bool valid = c < ncols;
    const long base = valid ? (c / CB) * SO + (c % CB) : 0;
    const bool sine = (kind & 1) != 0;
    C v[E];
    if (kind < 2) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int r = makhoul_row<L>(jt + i * TPL);
            C x = valid ? src[base + (long)r * SI] : mk<T>(0, 0);
            if (sine && (r & 1)) x = mk<T>(-x.x, -x.y);
            v[i] = x;
        }
        __syncthreads();
        line_fft<T, L, E, ES>(v, lds + col, jt, tw);
#pragma unroll
        for (int i = 0; i < E; ++i) lds[(jt + i * TPL) * ES + col] = v[i];
        __syncthreads();
        if (valid) {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int k = jt + i * TPL;
                const C vm = cconj(lds[((L - k) % L) * ES + col]);
                const C a = cscale(cadd(v[i], vm), (T)0.5);   // A_k
                const C d = csub(v[i], vm);                   // 2 i B_k
                const C b = mk<T>((T)0.5 * d.y, (T)-0.5 * d.x);  // B_k
                const C w = twq[k];
                C out = mk<T>(w.x * a.x - w.y * a.y, w.x * b.x - w.y * b.y);
                out = cscale(out, scale);
                const int row = sine ? sine_row<L>(k) : k;
                dst[base + (long)row * SI] = out;
            }
        }
    } else {
        C x[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int k = jt + i * TPL;
            const int row = sine ? sine_row<L>(k) : k;
            x[i] = valid ? src[base + (long)row * SI] : mk<T>(0, 0);
            lds[k * ES + col] = x[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int k = jt + i * TPL;
            const C xm = k == 0 ? mk<T>(0, 0) : lds[(L - k) * ES + col];
            const C t = mk<T>(x[i].x + xm.y, x[i].y - xm.x);  // X_k - i X_{L-k}
            const C w = cconj(twq[k]);
            const C V = cmul(w, t);
            v[i] = cconj(V);
        }
        __syncthreads();
        line_fft<T, L, E, ES>(v, lds + col, jt, tw);
        if (valid) {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int r = makhoul_row<L>(jt + i * TPL);
                C y = cconj(v[i]);
                if (sine && (r & 1)) y = mk<T>(-y.x, -y.y);
                dst[base + (long)r * SI] = cscale(y, scale);
            }
        }
    }
}

// Sine / cosine transforms along the contiguous z axis (the SSS family: every axis takes a
// sine or cosine basis and the data stay real).  Two real lines a, b of L points go through
// one L-point complex transform as the real and imaginary parts of z = a + i b: every step
// of the strided kernel above is real-linear, so its formulas hold unchanged with X = X^a
// + i X^b, and the two lines' coefficients come out as the real and imaginary parts.  The
// TPL = L / E threads of a line pair are lanes of one wavefront: the mirror value V_{L-k}
// comes from a lane shuffle and the exchanges need no workgroup barrier.
template <typename T, int L, int E, int LPW>
__global__ __launch_bounds__(LPW *(L / E)) void k_z_r2r(const T *__restrict__ src, T *__restrict__ dst, long npairs,
                                                         const V2<T> *__restrict__ twg, const V2<T> *__restrict__ twqg,
                                                         int kind, T scale) {
    using C = V2<T>;
    constexpr int TPL = L / E;
    constexpr int NT = LPW * TPL;
    constexpr int LL = lds_line_len<L>();
    __shared__ C lds[LPW * LL];
    __shared__ C tw[L];
    __shared__ C twq[L];
    const int tid = threadIdx.x;
    const int ln = tid / TPL;
    const int jt = tid % TPL;
    load_twiddles<T>(tw, twg, L, tid, NT);
    load_twiddles<T>(twq, twqg, L, tid, NT);  // exp(-i pi k / 2L), k < L
    const long p = (long)blockIdx.x * LPW + ln;
    const bool valid = p < npairs;
    const T *ga = src + (valid ? p : 0) * 2 * L;
    const T *gb = ga + L;
    const bool sine = (kind & 1) != 0;
    C *d = lds + ln * LL;
    C v[E];
    __syncthreads();
    if (kind < 2) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int r = makhoul_row<L>(jt + i * TPL);
            C x = mk<T>(ga[r], gb[r]);
            if (sine && (r & 1)) x = mk<T>(-x.x, -x.y);
            v[i] = x;
        }
        line_fft<T, L, E, 1>(v, d, jt, tw);
        C vm[E];
        mirror<T, L, E>(v, vm, jt);
        if (valid) {
            T *oa = dst + p * 2 * L;
            T *ob = oa + L;
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int k = jt + i * TPL;
                const C m = cconj(vm[i]);
                const C a = cscale(cadd(v[i], m), (T)0.5);      // A_k
                const C dd = csub(v[i], m);                      // 2 i B_k
                const C b = mk<T>((T)0.5 * dd.y, (T)-0.5 * dd.x);  // B_k
                const C w = twq[k];
                const int row = sine ? sine_row<L>(k) : k;
                oa[row] = (w.x * a.x - w.y * a.y) * scale;
                ob[row] = (w.x * b.x - w.y * b.y) * scale;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int k = jt + i * TPL;
            const int row = sine ? sine_row<L>(k) : k;
            const C x = mk<T>(ga[row], gb[row]);
            C xm = mk<T>(0, 0);
            if (k > 0) {
                const int rm = sine ? sine_row<L>(L - k) : L - k;
                xm = mk<T>(ga[rm], gb[rm]);
            }
            const C t = mk<T>(x.x + xm.y, x.y - xm.x);  // X_k - i X_{L-k}
            v[i] = cconj(cmul(cconj(twq[k]), t));
        }
        line_fft<T, L, E, 1>(v, d, jt, tw);
        if (valid) {
            T *oa = dst + p * 2 * L;
            T *ob = oa + L;
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int r = makhoul_row<L>(jt + i * TPL);
                C y = cconj(v[i]);
                if (sine && (r & 1)) y = mk<T>(-y.x, -y.y);
                oa[r] = y.x * scale;
                ob[r] = y.y * scale;
            }
        }
    }
}

// Points per thread of the z sine / cosine kernel: a line pair takes at most one wavefront.
constexpr int zr2r_E(int L) {
    int E = default_E(L);
    while (L / E > 64) E *= 2;
    return E;
}

template <typename T, int L> void add_z_r2r(std::vector<ZR2RKernel> &v) {
    constexpr int E = zr2r_E(L);
    constexpr int TPL = L / E;
    constexpr int LPW = TPL >= 256 ? 1 : 256 / TPL;
    v.push_back({L, sizeof(T) == 4 ? TK_F32 : TK_F64, [](const ZR2RArgs &a, hipStream_t s) {
                     hipLaunchKernelGGL((k_z_r2r<T, L, E, LPW>), dim3(cdiv(a.npairs, LPW)), dim3(LPW * TPL), 0, s,
                                        (const T *)a.src, (T *)a.dst, a.npairs, (const V2<T> *)a.tw,
                                        (const V2<T> *)a.twq, a.kind, (T)a.scale);
                 }});
}

const std::vector<ZR2RKernel> &z_r2r_kernels() {
    static std::vector<ZR2RKernel> K = [] {
        std::vector<ZR2RKernel> v;
#define TK_R(L) add_z_r2r<float, L>(v); add_z_r2r<double, L>(v);
        TK_FOR_EACH_LEN(TK_R)
#undef TK_R
        return v;
    }();
    return K;
}

// Tile of the strided sine / cosine kernel: at least 16 columns, so that every row access
// is a whole 128-byte line in FP32 (8-column tiles fetched each line in two halves at
// different times), within 1024 threads and the LDS; small lengths keep 512-thread tiles.
template <typename T> constexpr int r2r_E(int L) { return L / default_E(L) > 64 ? 2 * default_E(L) : default_E(L); }
template <typename T> constexpr int r2r_W(int L) {
    const int E = r2r_E<T>(L), tpl = L / E;
    int W = 512 / tpl > 16 ? 512 / tpl : 16;
    while (W > 1 && (W * tpl > 1024 || (L * (W + 1) + 2 * L) * 2 * (int)sizeof(T) > 160 * 1024)) W /= 2;
    return W;
}

template <typename T, int L> void add_r2r(std::vector<R2RKernel> &v) {
    constexpr int E = r2r_E<T>(L);
    constexpr int W = r2r_W<T>(L);
    static_assert(rplan_ok(L, E) && W >= 1 && W * (L / E) <= 1024, "tile shape");
    v.push_back({L, sizeof(T) == 4 ? TK_F32 : TK_F64, W, E, [](const R2RArgs &a, hipStream_t s) {
                     hipLaunchKernelGGL((k_r2r<T, L, E, W>), dim3(cdiv(a.ncols, W)), dim3(W * (L / E)), 0, s,
                                        (const V2<T> *)a.src, (V2<T> *)a.dst, a.ncols, a.CB, a.SO, a.SI,
                                        (const V2<T> *)a.tw, (const V2<T> *)a.twq, a.kind, (T)a.scale);
                 }});
}

const std::vector<R2RKernel> &r2r_kernels() {
    static std::vector<R2RKernel> K = [] {
        std::vector<R2RKernel> v;
#define TK_R(L) add_r2r<float, L>(v); add_r2r<double, L>(v);
        TK_FOR_EACH_LEN(TK_R)
#undef TK_R
        return v;
    }();
    return K;
}

}  // namespace tk
