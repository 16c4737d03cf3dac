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

template <typename T, int L> void add_r2r(std::vector<R2RKernel> &v) {
    constexpr int E = default_E(L);
    constexpr int W = (512 * E / L) > 0 ? 512 * E / L : 1;
    static_assert(W * (L / E) == 512 || L / E > 512, "tile shape");
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
