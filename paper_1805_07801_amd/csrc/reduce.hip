// FP64 reductions for Parseval checks.
#include "reduce.hpp"

namespace tk {

static constexpr int RB = 256;     // threads per block
static constexpr int RMAXB = 2048; // partial sums

template <typename T>
__global__ __launch_bounds__(RB) void k_sumsq_real(const T *__restrict__ x, long n, double *__restrict__ part) {
    __shared__ double sh[RB / 64];
    double acc = 0;
    for (long i = (long)blockIdx.x * RB + threadIdx.x; i < n; i += (long)gridDim.x * RB) {
        double v = (double)x[i];
        acc += v * v;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

template <typename T>
__global__ __launch_bounds__(RB) void k_sumsq_half(const V2<T> *__restrict__ X, long nlines, int nz,
                                                   double *__restrict__ part) {
    __shared__ double sh[RB / 64];
    const int nzh = nz / 2 + 1;
    const long n = nlines * nzh;
    double acc = 0;
    for (long i = (long)blockIdx.x * RB + threadIdx.x; i < n; i += (long)gridDim.x * RB) {
        const int kz = (int)(i % nzh);
        const double w = (kz == 0 || kz == nz / 2) ? 1.0 : 2.0;
        const V2<T> v = X[i];
        acc += w * ((double)v.x * v.x + (double)v.y * v.y);
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(RB) void k_sum_parts(const double *__restrict__ part, int np, double *__restrict__ out) {
    __shared__ double sh[RB / 64];
    double acc = 0;
    for (int i = threadIdx.x; i < np; i += RB) acc += part[i];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) out[0] = acc;
}

static tk_status finish(double *d, int nb, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(RB), 0, s, d, nb, d + RMAXB);
    TK_TRY(launch_check("sum parts"));
    TK_HIP_CHECK(hipMemcpyAsync(out, d + RMAXB, sizeof(double), hipMemcpyDeviceToHost, s));
    TK_HIP_CHECK(hipStreamSynchronize(s));
    return TK_OK;
}

static double *scratch(tk_status *st) {
    static thread_local double *buf = nullptr;
    static thread_local int dev = -1;
    int d = 0;
    hipGetDevice(&d);
    if (!buf || d != dev) {
        if (hipMalloc((void **)&buf, sizeof(double) * (RMAXB + 1)) != hipSuccess) {
            *st = fail(TK_ENOMEM, "reduction scratch allocation failed");
            buf = nullptr;
            return nullptr;
        }
        dev = d;
    }
    *st = TK_OK;
    return buf;
}

tk_status reduce_sumsq_real(const void *x, long n, tk_dtype dt, double *out, hipStream_t s) {
    tk_status st;
    double *d = scratch(&st);
    if (!d) return st;
    int nb = (int)std::min<long>(RMAXB, std::max<long>(1, (n + RB - 1) / RB));
    if (dt == TK_F32)
        hipLaunchKernelGGL(k_sumsq_real<float>, dim3(nb), dim3(RB), 0, s, (const float *)x, n, d);
    else
        hipLaunchKernelGGL(k_sumsq_real<double>, dim3(nb), dim3(RB), 0, s, (const double *)x, n, d);
    TK_TRY(launch_check("sumsq real"));
    return finish(d, nb, out, s);
}

tk_status reduce_sumsq_half(const void *X, long nlines, int nz, tk_dtype dt, double *out, hipStream_t s) {
    tk_status st;
    double *d = scratch(&st);
    if (!d) return st;
    long n = nlines * (nz / 2 + 1);
    int nb = (int)std::min<long>(RMAXB, std::max<long>(1, (n + RB - 1) / RB));
    if (dt == TK_F32)
        hipLaunchKernelGGL(k_sumsq_half<float>, dim3(nb), dim3(RB), 0, s, (const float2 *)X, nlines, nz, d);
    else
        hipLaunchKernelGGL(k_sumsq_half<double>, dim3(nb), dim3(RB), 0, s, (const double2 *)X, nlines, nz, d);
    TK_TRY(launch_check("sumsq half"));
    return finish(d, nb, out, s);
}

}  // namespace tk

namespace tk {

template <typename T>
__global__ __launch_bounds__(RB) void k_diff(const T *__restrict__ a, const T *__restrict__ b, long n,
                                             double *__restrict__ part) {
    __shared__ double sh[RB / 64];
    double num = 0, den = 0;
    for (long i = (long)blockIdx.x * RB + threadIdx.x; i < n; i += (long)gridDim.x * RB) {
        double x = (double)a[i], y = (double)b[i];
        num += (x - y) * (x - y);
        den += y * y;
    }
    num = block_sum(num, sh);
    den = block_sum(den, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = num;
        part[RMAXB / 2 + blockIdx.x] = den;
    }
}

tk_status reduce_diff(const void *a, const void *b, long n, tk_dtype dt, double *num, double *den, hipStream_t s) {
    tk_status st;
    double *d = scratch(&st);
    if (!d) return st;
    int nb = (int)std::min<long>(RMAXB / 2, std::max<long>(1, (n + RB - 1) / RB));
    if (dt == TK_F32)
        hipLaunchKernelGGL(k_diff<float>, dim3(nb), dim3(RB), 0, s, (const float *)a, (const float *)b, n, d);
    else
        hipLaunchKernelGGL(k_diff<double>, dim3(nb), dim3(RB), 0, s, (const double *)a, (const double *)b, n, d);
    TK_TRY(launch_check("diff"));
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(RB), 0, s, d, nb, d + RMAXB);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(RB), 0, s, d + RMAXB / 2, nb, d + RMAXB - 1);
    TK_TRY(launch_check("diff parts"));
    double h[2];
    TK_HIP_CHECK(hipMemcpyAsync(&h[0], d + RMAXB, sizeof(double), hipMemcpyDeviceToHost, s));
    TK_HIP_CHECK(hipMemcpyAsync(&h[1], d + RMAXB - 1, sizeof(double), hipMemcpyDeviceToHost, s));
    TK_HIP_CHECK(hipStreamSynchronize(s));
    *num = h[0];
    *den = h[1];
    return TK_OK;
}

// splitmix-style hash of (seed, i) mapped to [-1, 1)
__device__ __forceinline__ double hash_unit(unsigned seed, long i) {
    unsigned long long z = (unsigned long long)i * 0x9E3779B97F4A7C15ull + seed * 0xBF58476D1CE4E5B9ull + 1;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 4503599627370496.0) - 1.0;
}

template <typename T> __global__ void k_fill(T *__restrict__ x, long n, unsigned seed) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        x[i] = (T)hash_unit(seed, i);
}

tk_status fill_pattern(void *x, long n, tk_dtype dt, unsigned seed, hipStream_t s) {
    int nb = (int)std::min<long>(8192, std::max<long>(1, (n + 255) / 256));
    if (dt == TK_F32)
        hipLaunchKernelGGL(k_fill<float>, dim3(nb), dim3(256), 0, s, (float *)x, n, seed);
    else
        hipLaunchKernelGGL(k_fill<double>, dim3(nb), dim3(256), 0, s, (double *)x, n, seed);
    return launch_check("fill");
}

}  // namespace tk
