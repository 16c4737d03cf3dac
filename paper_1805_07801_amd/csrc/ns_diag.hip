// FP64 diagnostics of a spectral velocity state and the random initial field.
//
// Sums over the stored half spectrum carry w(kz) = 1 on kz = 0 and N/2, 2 elsewhere, so
// they equal full-spectrum sums.  Every per-mode term is formed in FP64 from the stored
// values; per-block partial sums are added in a fixed order (deterministic).
#include "ns_api.hpp"
#include "reduce.hpp"

namespace tk {

static constexpr int DB = 256;

// Shell of a mode: the integer s with (2s-1)^2 <= 4|k|^2 < (2s+1)^2 (s = 0 for k = 0).
__device__ __forceinline__ int shell_of(long k2) {
    int s = (int)floor(sqrt((double)k2));
    if (4 * k2 >= (long)(2 * s + 1) * (2 * s + 1)) ++s;
    if (s > 0 && 4 * k2 < (long)(2 * s - 1) * (2 * s - 1)) --s;
    return s;
}

// part layout per block: [0] energy, [1] enstrophy, [2] max |k.u^|/|k|, [3] max |u^|,
// [4..4+nshell) E(s)
template <typename T>
__global__ __launch_bounds__(DB) void k_diag(const V2<T> *__restrict__ u, int N, int nshell, double *__restrict__ part,
                                             int stride) {
    extern __shared__ double hist[];
    __shared__ double sh[DB / 64];
    for (int i = threadIdx.x; i < nshell; i += DB) hist[i] = 0;
    __syncthreads();
    const int NZH = N / 2 + 1;
    const long FS = (long)N * N * NZH;
    double e = 0, z = 0, dmax = 0, umx = 0;
    for (long m = (long)blockIdx.x * DB + threadIdx.x; m < FS; m += (long)gridDim.x * DB) {
        const int kz = (int)(m % NZH);
        const long xy = m / NZH;
        const int y = (int)(xy % N), x = (int)(xy / N);
        const int kx = x < N / 2 ? x : x - N, ky = y < N / 2 ? y : y - N;
        const double w = (kz == 0 || 2 * kz == N) ? 1.0 : 2.0;
        const V2<T> a = u[m], b = u[FS + m], c = u[2 * FS + m];
        const double uu = (double)a.x * a.x + (double)a.y * a.y + (double)b.x * b.x + (double)b.y * b.y +
                          (double)c.x * c.x + (double)c.y * c.y;
        const long k2 = (long)kx * kx + (long)ky * ky + (long)kz * kz;
        const double em = 0.5 * w * uu;
        e += em;
        z += em * (double)k2;
        umx = fmax(umx, uu);
        if (k2 > 0) {
            const double dr = kx * (double)a.x + ky * (double)b.x + kz * (double)c.x;
            const double di = kx * (double)a.y + ky * (double)b.y + kz * (double)c.y;
            dmax = fmax(dmax, (dr * dr + di * di) / (double)k2);
        }
        const int s = shell_of(k2);
        if (s < nshell && em != 0) atomicAdd(&hist[s], em);
    }
    e = block_sum(e, sh);
    z = block_sum(z, sh);
    dmax = block_max(dmax, sh);
    umx = block_max(umx, sh);
    __syncthreads();
    double *p = part + (long)blockIdx.x * stride;
    if (threadIdx.x == 0) {
        p[0] = e;
        p[1] = z;
        p[2] = dmax;
        p[3] = umx;
    }
    for (int i = threadIdx.x; i < nshell; i += DB) p[4 + i] = hist[i];
}

// Column-wise sum (max for entries 2 and 3) of nb partial rows: one workgroup per column,
// a fixed strided split over threads and a fixed tree (deterministic).
__global__ __launch_bounds__(DB) void k_diag_final(const double *__restrict__ part, int nb, int stride,
                                                   double *__restrict__ out) {
    __shared__ double sh[DB / 64];
    const int i = blockIdx.x;
    const bool mx = (i == 2 || i == 3);
    double acc = 0;
    for (int b = threadIdx.x; b < nb; b += DB) {
        const double v = part[(long)b * stride + i];
        acc = mx ? fmax(acc, v) : acc + v;
    }
    acc = mx ? block_max(acc, sh) : block_sum(acc, sh);
    if (threadIdx.x == 0) out[i] = acc;
}

tk_status ns_diag_run(const void *u, int N, tk_dtype dt, int nshell, double *dscratch, double *hout,
                      hipStream_t s) {
    const int nb = NS_DIAG_BLOCKS;
    const int stride = NS_DIAG_HEAD + nshell;
    double *part = dscratch;
    double *out = dscratch + (long)nb * stride;
    const size_t shm = sizeof(double) * (nshell > 0 ? nshell : 1);
    if (dt == TK_F32)
        hipLaunchKernelGGL(k_diag<float>, dim3(nb), dim3(DB), shm, s, (const float2 *)u, N, nshell, part, stride);
    else
        hipLaunchKernelGGL(k_diag<double>, dim3(nb), dim3(DB), shm, s, (const double2 *)u, N, nshell, part, stride);
    TK_TRY(launch_check("diagnostics"));
    hipLaunchKernelGGL(k_diag_final, dim3(stride), dim3(DB), 0, s, part, nb, stride, out);
    TK_TRY(launch_check("diagnostics final"));
    TK_HIP_CHECK(hipMemcpyAsync(hout, out, sizeof(double) * stride, hipMemcpyDeviceToHost, s));
    TK_HIP_CHECK(hipStreamSynchronize(s));
    return TK_OK;
}

// ---- initial field ---------------------------------------------------------------------------
// Projection, 2/3 mask and k = 0 removal in place on a fresh r2c of the noise.
template <typename T> __global__ void k_init_project(V2<T> *u, int N) {
    const int NZH = N / 2 + 1;
    const long FS = (long)N * N * NZH;
    const int K = (N - 1) / 3;
    for (long m = (long)blockIdx.x * blockDim.x + threadIdx.x; m < FS; m += (long)gridDim.x * blockDim.x) {
        const int kz = (int)(m % NZH);
        const long xy = m / NZH;
        const int y = (int)(xy % N), x = (int)(xy / N);
        const int kx = x < N / 2 ? x : x - N, ky = y < N / 2 ? y : y - N;
        V2<T> a = u[m], b = u[FS + m], c = u[2 * FS + m];
        const bool kept = abs(kx) <= K && abs(ky) <= K && kz <= K;
        const long k2 = (long)kx * kx + (long)ky * ky + (long)kz * kz;
        if (!kept || k2 == 0) {
            a.x = a.y = b.x = b.y = c.x = c.y = 0;
        } else {
            const T ik2 = (T)(1.0 / (double)k2);
            const T dr = kx * a.x + ky * b.x + kz * c.x, di = kx * a.y + ky * b.y + kz * c.y;
            a.x -= kx * dr * ik2; a.y -= kx * di * ik2;
            b.x -= ky * dr * ik2; b.y -= ky * di * ik2;
            c.x -= kz * dr * ik2; c.y -= kz * di * ik2;
        }
        u[m] = a;
        u[FS + m] = b;
        u[2 * FS + m] = c;
    }
}

// Multiply every mode by fac[shell(k)] (FP64 factors).
template <typename T> __global__ void k_scale_shells(V2<T> *u, int N, const double *__restrict__ fac, int nshell) {
    const int NZH = N / 2 + 1;
    const long FS = (long)N * N * NZH;
    for (long m = (long)blockIdx.x * blockDim.x + threadIdx.x; m < FS; m += (long)gridDim.x * blockDim.x) {
        const int kz = (int)(m % NZH);
        const long xy = m / NZH;
        const int y = (int)(xy % N), x = (int)(xy / N);
        const int kx = x < N / 2 ? x : x - N, ky = y < N / 2 ? y : y - N;
        const int s = shell_of((long)kx * kx + (long)ky * ky + (long)kz * kz);
        const double f = s < nshell ? fac[s] : 0.0;
        for (int c = 0; c < 3; ++c) {
            V2<T> a = u[c * FS + m];
            a.x = (T)(a.x * f);
            a.y = (T)(a.y * f);
            u[c * FS + m] = a;
        }
    }
}

tk_status ns_init_project(void *u, int N, tk_dtype dt, hipStream_t s) {
    const long FS = (long)N * N * (N / 2 + 1);
    const unsigned nb = (unsigned)std::min<long>(16384, cdiv(FS, 256));
    if (dt == TK_F32) hipLaunchKernelGGL(k_init_project<float>, dim3(nb), dim3(256), 0, s, (float2 *)u, N);
    else hipLaunchKernelGGL(k_init_project<double>, dim3(nb), dim3(256), 0, s, (double2 *)u, N);
    return launch_check("init project");
}

tk_status ns_scale_shells(void *u, int N, tk_dtype dt, const double *fac_dev, int nshell, hipStream_t s) {
    const long FS = (long)N * N * (N / 2 + 1);
    const unsigned nb = (unsigned)std::min<long>(16384, cdiv(FS, 256));
    if (dt == TK_F32)
        hipLaunchKernelGGL(k_scale_shells<float>, dim3(nb), dim3(256), 0, s, (float2 *)u, N, fac_dev, nshell);
    else
        hipLaunchKernelGGL(k_scale_shells<double>, dim3(nb), dim3(256), 0, s, (double2 *)u, N, fac_dev, nshell);
    return launch_check("scale shells");
}

}  // namespace tk
