// FP64 reductions (Parseval sums and the like).  Deterministic: per-block partial sums
// in a fixed tree order, then one block adds the partials in index order.
#pragma once

#include "common.hpp"

namespace tk {

// sum x_i^2 over n real values of dtype dt; result on the host.  Synchronises s.
tk_status reduce_sumsq_real(const void *x, long n, tk_dtype dt, double *out, hipStream_t s);
// sum_lines sum_kz w(kz) |X_kz|^2 over nlines half-spectrum lines of nz/2+1 values.
tk_status reduce_sumsq_half(const void *X, long nlines, int nz, tk_dtype dt, double *out, hipStream_t s);

// Block-wide sum of a double (all threads get the result); blockDim.x multiple of 64.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = 0;
    for (int i = 0; i < nw; ++i) r += sh[i];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = sh[0];
    for (int i = 1; i < nw; ++i) r = fmax(r, sh[i]);
    __syncthreads();
    return r;
}

}  // namespace tk

namespace tk {
// num = sum (a_i - b_i)^2, den = sum b_i^2 over n real values.  Synchronises s.
tk_status reduce_diff(const void *a, const void *b, long n, tk_dtype dt, double *num, double *den, hipStream_t s);
// Fill n real values with a deterministic pseudo-random pattern in [-1, 1).
tk_status fill_pattern(void *x, long n, tk_dtype dt, unsigned seed, hipStream_t s);
}  // namespace tk
