// Energy transfer diagnostics: the shell transfer T(s) = sum_{k in s} w Re[u^* . N], whose
// running sum is the energy flux, and the giver/receiver shell-to-shell transfer
//   T_nm = - sum_{k in band n} w Re[u^* . F((u . grad) u^(m))],  u^(m) = u restricted to band m.
// (The paper lists energy flux and shell-to-shell transfer among the solver's functions.)
// All sums FP64, per-block histograms added in a fixed order.
#include <cmath>
#include <new>

#include "ns_api.hpp"
#include "reduce.hpp"

namespace tk {

static constexpr int XB = 256;

__device__ __forceinline__ int shell_of_k2(long k2) {
    int s = (int)floor(sqrt((double)k2));
    if (4 * k2 >= (long)(2 * s + 1) * (2 * s + 1)) ++s;
    if (s > 0 && 4 * k2 < (long)(2 * s - 1) * (2 * s - 1)) --s;
    return s;
}

// part[blk][b] = sum over the block's modes in bin b of sign * w Re(A^* . B); bins are
// band_of_shell[shell(k)] (or the shell itself when band_of_shell is null).
template <typename T>
__global__ __launch_bounds__(XB) void k_cross_bins(const V2<T> *__restrict__ A, const V2<T> *__restrict__ B, int N,
                                                   const int *__restrict__ band_of_shell, int nshell, int nbins,
                                                   double sign, double *__restrict__ part) {
    extern __shared__ double hist[];
    for (int i = threadIdx.x; i < nbins; i += XB) hist[i] = 0;
    __syncthreads();
    const int NZH = N / 2 + 1;
    const long FS = (long)N * N * NZH;
    for (long m = (long)blockIdx.x * XB + threadIdx.x; m < FS; m += (long)gridDim.x * XB) {
        const int kz = (int)(m % NZH);
        const long xy = m / NZH;
        const int y = (int)(xy % N), x = (int)(xy / N);
        const int kx = x < N / 2 ? x : x - N, ky = y < N / 2 ? y : y - N;
        const int s = shell_of_k2((long)kx * kx + (long)ky * ky + (long)kz * kz);
        if (s >= nshell) continue;
        const int b = band_of_shell ? band_of_shell[s] : s;
        if (b < 0 || b >= nbins) continue;
        const double w = (kz == 0 || 2 * kz == N) ? 1.0 : 2.0;
        double acc = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const V2<T> a = A[c * FS + m], bb = B[c * FS + m];
            acc += (double)a.x * bb.x + (double)a.y * bb.y;
        }
        if (acc != 0) atomicAdd(&hist[b], sign * w * acc);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += XB) part[(long)blockIdx.x * nbins + i] = hist[i];
}

__global__ __launch_bounds__(XB) void k_bins_final(const double *__restrict__ part, int nb, int nbins,
                                                   double *__restrict__ out) {
    __shared__ double sh[XB / 64];
    const int i = blockIdx.x;
    double acc = 0;
    for (int b = threadIdx.x; b < nb; b += XB) acc += part[(long)b * nbins + i];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) out[i] = acc;
}

// out = u on the modes of band m (and inside the 2/3 set), zero elsewhere.
template <typename T>
__global__ void k_band_pass(const V2<T> *__restrict__ u, V2<T> *__restrict__ o, int N, int K,
                            const int *__restrict__ band_of_shell, int nshell, int m) {
    const int NZH = N / 2 + 1;
    const long FS = (long)N * N * NZH;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < FS; q += (long)gridDim.x * blockDim.x) {
        const int kz = (int)(q % NZH);
        const long xy = q / NZH;
        const int y = (int)(xy % N), x = (int)(xy / N);
        const int kx = x < N / 2 ? x : x - N, ky = y < N / 2 ? y : y - N;
        const int s = shell_of_k2((long)kx * kx + (long)ky * ky + (long)kz * kz);
        const bool on = abs(kx) <= K && abs(ky) <= K && kz <= K && s < nshell && band_of_shell[s] == m;
        for (int c = 0; c < 3; ++c) o[c * FS + q] = on ? u[c * FS + q] : mk<T>(0, 0);
    }
}

// g[3 i + j] = i k_j v^_i (Nyquist derivative zero).
template <typename T> __global__ void k_grad9(const V2<T> *__restrict__ v, V2<T> *__restrict__ g, int N) {
    const int NZH = N / 2 + 1;
    const long FS = (long)N * N * NZH;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < FS; q += (long)gridDim.x * blockDim.x) {
        const int kz0 = (int)(q % NZH);
        const long xy = q / NZH;
        const int y = (int)(xy % N), x = (int)(xy / N);
        const int k[3] = {2 * x == N ? 0 : (x < N / 2 ? x : x - N), 2 * y == N ? 0 : (y < N / 2 ? y : y - N),
                          2 * kz0 == N ? 0 : kz0};
        for (int i = 0; i < 3; ++i) {
            const V2<T> a = v[i * FS + q];
            for (int j = 0; j < 3; ++j) g[(3 * i + j) * FS + q] = mk<T>(-a.y * k[j], a.x * k[j]);
        }
    }
}

// a_i = sum_j u_j g[3 i + j] (real space), M points.
template <typename T> __global__ void k_advect(const T *__restrict__ u, const T *__restrict__ g, T *__restrict__ a,
                                               long M) {
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < M; p += (long)gridDim.x * blockDim.x) {
        const T u0 = u[p], u1 = u[M + p], u2 = u[2 * M + p];
        for (int i = 0; i < 3; ++i)
            a[i * M + p] = u0 * g[(3 * i) * M + p] + u1 * g[(3 * i + 1) * M + p] + u2 * g[(3 * i + 2) * M + p];
    }
}

static unsigned eb(long n) { return (unsigned)std::min<long>(16384, std::max<long>(1, (n + 255) / 256)); }

static tk_status cross_bins(const void *A, const void *B, int N, tk_dtype dt, const int *bos_dev, int nshell,
                            int nbins, double sign, double *dscratch, double *hout, hipStream_t s) {
    const int nb = NS_DIAG_BLOCKS;
    double *part = dscratch;
    double *out = dscratch + (long)nb * nbins;
    const size_t shm = sizeof(double) * nbins;
    if (dt == TK_F32)
        hipLaunchKernelGGL(k_cross_bins<float>, dim3(nb), dim3(XB), shm, s, (const float2 *)A, (const float2 *)B, N,
                           bos_dev, nshell, nbins, sign, part);
    else
        hipLaunchKernelGGL(k_cross_bins<double>, dim3(nb), dim3(XB), shm, s, (const double2 *)A, (const double2 *)B,
                           N, bos_dev, nshell, nbins, sign, part);
    TK_TRY(launch_check("cross spectrum"));
    hipLaunchKernelGGL(k_bins_final, dim3(nbins), dim3(XB), 0, s, part, nb, nbins, out);
    TK_TRY(launch_check("cross spectrum final"));
    TK_HIP_CHECK(hipMemcpyAsync(hout, out, sizeof(double) * nbins, hipMemcpyDeviceToHost, s));
    TK_HIP_CHECK(hipStreamSynchronize(s));
    return TK_OK;
}

}  // namespace tk

using namespace tk;

extern "C" tk_status ns_energy_transfer(tk_ns_t p, const void *u, double *T, int nshell, void *stream) {
    if (!p || !u || !T) return fail(TK_EINVAL, "NULL argument");
    if (nshell < 1 || nshell > p->nshell) return fail(TK_EINVAL, "nshell must be in [1, %d]", p->nshell);
    hipStream_t s = (hipStream_t)stream;
    // N(u) into the stage buffer (its masked modes are zero and stay zero)
    P5Args a{};
    a.u = const_cast<void *>(u);
    a.out = p->ust;
    a.st = p->st;
    a.nu = p->cfg.nu;
    a.mode = NS_RHS;
    TK_TRY(ns_rhs_eval(p->g, u, p->w6, a, nullptr, nullptr, s));
    std::vector<double> h(nshell);
    TK_TRY(cross_bins(u, p->ust, p->g.n, p->cfg.dtype, nullptr, nshell, nshell, 1.0, p->dscratch, h.data(), s));
    for (int i = 0; i < nshell; ++i) T[i] = h[i];
    return TK_OK;
}

extern "C" tk_status ns_shell_to_shell(tk_ns_t p, const void *u, const int *band_of_shell, int nshell, int nbands,
                                       double *Tnm, void *stream) {
    if (!p || !u || !band_of_shell || !Tnm) return fail(TK_EINVAL, "NULL argument");
    if (nshell < 1 || nbands < 1 || nbands > 4096) return fail(TK_EINVAL, "bad band arguments");
    for (int i = 0; i < nshell; ++i)
        if (band_of_shell[i] >= nbands) return fail(TK_EINVAL, "band_of_shell[%d] >= nbands", i);
    hipStream_t s = (hipStream_t)stream;
    const NsGrid &g = p->g;
    const int n = g.n;
    const size_t esz = p->cfg.dtype == TK_F32 ? 4 : 8;
    const long FS = (long)n * n * (n / 2 + 1), M = (long)n * n * n;
    void *ur = nullptr, *gsp = nullptr, *gr = nullptr, *ar = nullptr, *ah = nullptr, *um = nullptr, *ws = nullptr;
    int *bos = nullptr;
    double *scr = nullptr;
    auto cleanup = [&]() {
        void *ps[] = {ur, gsp, gr, ar, ah, um, ws, bos, scr};
        for (void *q : ps)
            if (q) hipFree(q);
    };
    const size_t cb = 2 * esz * FS, rb = esz * M;
    if (hipMalloc(&ur, 3 * rb) != hipSuccess || hipMalloc(&gsp, 9 * cb) != hipSuccess ||
        hipMalloc(&gr, 9 * rb) != hipSuccess || hipMalloc(&ar, 3 * rb) != hipSuccess ||
        hipMalloc(&ah, 3 * cb) != hipSuccess || hipMalloc(&um, 3 * cb) != hipSuccess ||
        hipMalloc(&ws, 3 * cb) != hipSuccess || hipMalloc((void **)&bos, sizeof(int) * nshell) != hipSuccess ||
        hipMalloc((void **)&scr, sizeof(double) * (NS_DIAG_BLOCKS + 2) * (size_t)nbands) != hipSuccess) {
        cleanup();
        return fail(TK_ENOMEM, "shell-to-shell workspace allocation failed");
    }
    tk_status st = TK_OK;
    std::vector<double> col(nbands);
    do {
        if (hipMemcpyAsync(bos, band_of_shell, sizeof(int) * nshell, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(ws, u, 3 * cb, hipMemcpyDeviceToDevice, s) != hipSuccess) {
            st = fail(TK_EHIP, "upload failed");
            break;
        }
        // u in real space (from a copy: the X pass below runs in place)
        if ((st = fft_x_pass(g.ax, ws, ws, 3, 1, 1.0, s)) != TK_OK) break;
        if ((st = fft_y_pass(g.ax, ws, ws, 3, 1, s)) != TK_OK) break;
        if ((st = fft_z_c2r(g.ax, ws, ur, 3, s)) != TK_OK) break;
        for (int m = 0; m < nbands && st == TK_OK; ++m) {
            if (p->cfg.dtype == TK_F32) {
                hipLaunchKernelGGL(k_band_pass<float>, dim3(eb(FS)), dim3(256), 0, s, (const float2 *)u, (float2 *)um, n,
                                   g.K, bos, nshell, m);
                hipLaunchKernelGGL(k_grad9<float>, dim3(eb(FS)), dim3(256), 0, s, (const float2 *)um, (float2 *)gsp, n);
            } else {
                hipLaunchKernelGGL(k_band_pass<double>, dim3(eb(FS)), dim3(256), 0, s, (const double2 *)u, (double2 *)um,
                                   n, g.K, bos, nshell, m);
                hipLaunchKernelGGL(k_grad9<double>, dim3(eb(FS)), dim3(256), 0, s, (const double2 *)um, (double2 *)gsp,
                                   n);
            }
            if ((st = launch_check("band gradients")) != TK_OK) break;
            if ((st = fft_x_pass(g.ax, gsp, gsp, 9, 1, 1.0, s)) != TK_OK) break;
            if ((st = fft_y_pass(g.ax, gsp, gsp, 9, 1, s)) != TK_OK) break;
            if ((st = fft_z_c2r(g.ax, gsp, gr, 9, s)) != TK_OK) break;
            if (p->cfg.dtype == TK_F32)
                hipLaunchKernelGGL(k_advect<float>, dim3(eb(M)), dim3(256), 0, s, (const float *)ur, (const float *)gr,
                                   (float *)ar, M);
            else
                hipLaunchKernelGGL(k_advect<double>, dim3(eb(M)), dim3(256), 0, s, (const double *)ur,
                                   (const double *)gr, (double *)ar, M);
            if ((st = launch_check("advection")) != TK_OK) break;
            if ((st = fft_z_r2c(g.ax, ar, ah, 3, 1.0, s)) != TK_OK) break;
            if ((st = fft_y_pass(g.ax, ah, ah, 3, 0, s)) != TK_OK) break;
            if ((st = fft_x_pass(g.ax, ah, ah, 3, 0, 1.0 / (double)M, s)) != TK_OK) break;
            // receivers: -sum w Re(u^* . A) per band (u is zero outside the 2/3 set)
            if ((st = cross_bins(u, ah, n, p->cfg.dtype, bos, nshell, nbands, -1.0, scr, col.data(), s)) != TK_OK)
                break;
            for (int r = 0; r < nbands; ++r) Tnm[(long)r * nbands + m] = col[r];
        }
    } while (0);
    if (hipStreamSynchronize(s) != hipSuccess && st == TK_OK) st = fail(TK_EHIP, "synchronisation failed");
    cleanup();
    return st;
}
