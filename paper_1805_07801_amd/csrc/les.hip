// Learned sub-grid closure for coarse LES: the pointwise network (forward, backward,
// Adam), the filtered-DNS training data, and the LES step that adds the closure's
// stress divergence to the pseudo-spectral right-hand side.
//
// Network: 9 filtered velocity gradients (divided by in_scale) -> 64 GELU -> 64 GELU ->
// 6 stress components (times out_scale); parameters are BF16, every product and sum is
// FP32.  Flat parameter order W1[64][9], b1[64], W2[64][64], b2[64], W3[6][64], b3[6].
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "ns_api.hpp"
#include "reduce.hpp"

namespace tk {

constexpr int NP = 5190;
constexpr int OW1 = 0, OB1 = 576, OW2 = 640, OB2 = 4736, OW3 = 4800, OB3 = 5184;

__device__ __forceinline__ float bf16_f32(uint16_t b) { return __uint_as_float((unsigned)b << 16); }
__device__ __forceinline__ uint16_t f32_bf16(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
// erf by the rational approximation of Abramowitz and Stegun, Handbook of Mathematical
// Functions, eq. 7.1.26 (absolute error <= 1.5e-7 on x >= 0, odd extension):
//   erf(x) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2),  t = 1 / (1 + p x).
// Branch-free (one reciprocal, one exponential), where the library erf takes two
// divergent ranges: the network's activations are its main vector-ALU cost.
// The GELU needs it at x / sqrt 2, through the normal tail Phi(-|x|) = erfc(|x| / sqrt 2) / 2:
// tail = t P(t) e / 2 with t = 1 / (1 + p |x| / sqrt 2) and e = exp(-x^2 / 2), the 1/2 and
// the 1/sqrt 2 folded into the constants.
__device__ __forceinline__ float normal_tail(float x, float &e) {
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, fabsf(x), 1.0f));
    float q = fmaf(0.5f * 1.061405429f, t, 0.5f * -1.453152027f);
    q = fmaf(q, t, 0.5f * 1.421413741f);
    q = fmaf(q, t, 0.5f * -0.284496736f);
    q = fmaf(q, t, 0.5f * 0.254829592f);
    e = __builtin_amdgcn_exp2f(-0.72134752044448170f * x * x);  // exp(-x^2 / 2)
    return q * t * e;
}
// GELU(x) = x Phi(x) = max(x, 0) - |x| Phi(-|x|): the small negative branch comes out of the
// tail directly instead of as the difference of two numbers near 1.
__device__ __forceinline__ float gelu(float x) {
    float e;
    const float tail = normal_tail(x, e);
    return fmaf(-fabsf(x), tail, fmaxf(x, 0.0f));
}
// GELU'(x) = Phi(x) + x phi(x), phi(x) = exp(-x^2 / 2) / sqrt(2 pi) with the tail's exponential.
__device__ __forceinline__ float gelu_grad(float x) {
    float e;
    const float tail = normal_tail(x, e);
    return (x >= 0.0f ? 1.0f - tail : tail) + x * e * 0.39894228040143268f;
}

// ---- forward ------------------------------------------------------------------------------------------

__device__ __forceinline__ void load_weights(float *w, const uint16_t *__restrict__ wb) {
    for (int i = threadIdx.x; i < NP; i += blockDim.x) w[i] = bf16_f32(wb[i]);
    __syncthreads();
}

// Forward on the matrix cores.  Each layer is a product D = W H of the weights (outputs x
// inputs) and the activations (inputs x points), taken 16 points at a time by one
// wavefront with v_mfma_f32_16x16x32_bf16.  The weights are BF16 parameters already; each
// FP32 activation is split into three BF16 terms, h = hi + mid + lo (split3: exact for
// |h| >= 2^-110), so every product w h_i is exact in FP32 and the sums run in FP32 on the
// FP32 accumulators:
// the FP32 arithmetic of the definition, in another order, at a quarter of the matrix
// cycles of the FP32 instruction.  Operand layouts on a wavefront, lane l = 16 kk + c
// (kk < 4, c < 16):
//   A (16 x 32): lane l holds 8 values of row c (its K slots);  B (32 x 16): the same K
//   slots of column c;  D (16 x 16): 4 values, D[4 kk + r][c], r < 4.
// Which K slot carries which input feature is free (the sum is order-free) as long as A
// and B agree, so a lane holds, for point c of the block, outputs 4 kk + r of each 16-row
// tile q (feature o = 16 q + 4 kk + r) and the next layer consumes them in place: K step s
// takes from lane l its outputs of tiles 2 s and 2 s + 1, slot j = 4 (q - 2 s) + r, and its A
// operand is the weight column of that same feature.  The 9 inputs take slots j < 3 of
// lanes kk < 3 (feature 3 kk + j).  The weights are per-lane constants, loaded once per
// wavefront; wavefronts walk the 16-point blocks.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
constexpr int MB = 256;

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma32(v4u a, v4u b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0,
                                                   0, 0);
}
// Two BF16 bit patterns in one register, element 2 p in the low half.
__device__ __forceinline__ unsigned pack_hi16(unsigned lo_elem, unsigned hi_elem) {
    return (lo_elem >> 16) | (hi_elem & 0xffff0000u);
}
// v[j] = hi[j] + mid[j] + lo[j]: truncating an FP32 value to its BF16 head leaves a remainder
// of at most 16 significant bits, and truncating that one leaves at most 8, which BF16 holds
// exactly while the remainders are normal numbers (|v| >= 2^-110); below that the third
// term drops less than 2^-133.
__device__ __forceinline__ void split3(const float (&v)[8], v4u &hi, v4u &mid, v4u &lo) {
    unsigned uh[8], um[8], ul[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        uh[j] = __float_as_uint(v[j]);
        const float r1 = v[j] - __uint_as_float(uh[j] & 0xffff0000u);
        um[j] = __float_as_uint(r1);
        ul[j] = __float_as_uint(r1 - __uint_as_float(um[j] & 0xffff0000u));
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        hi[p] = pack_hi16(uh[2 * p], uh[2 * p + 1]);
        mid[p] = pack_hi16(um[2 * p], um[2 * p + 1]);
        lo[p] = pack_hi16(ul[2 * p], ul[2 * p + 1]);
    }
}
// D += A (hi + mid + lo), the smallest terms first
__device__ __forceinline__ v4f mfma32x3(v4u a, const float (&v)[8], v4f d) {
    v4u hi, mid, lo;
    split3(v, hi, mid, lo);
    d = mfma32(a, lo, d);
    d = mfma32(a, mid, d);
    return mfma32(a, hi, d);
}

__global__ __launch_bounds__(MB) void k_mlp_fwd(const uint16_t *__restrict__ wb, const float *__restrict__ x9,
                                               float *__restrict__ y6, long M, float in_inv, float out_scale) {
    const int lane = threadIdx.x & 63;
    const int kk = lane >> 4, c = lane & 15;
    auto w = [&](int i) { return bf16_f32(wb[i]); };
    auto bits = [&](bool ok, int i) { return ok ? (unsigned)wb[i] << 16 : 0u; };
    // A operands as BF16 pairs: layer 1 [q], layer 2 [q][s], layer 3 [s]
    v4u a1[4], a2[4][2], a3[2];
    v4f b1[4], b2[4], b3;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int j0 = 2 * p, j1 = 2 * p + 1, f0 = 3 * kk + j0, f1 = 3 * kk + j1;
            a1[q][p] = pack_hi16(bits(j0 < 3 && f0 < 9, OW1 + (16 * q + c) * 9 + f0),
                                 bits(j1 < 3 && f1 < 9, OW1 + (16 * q + c) * 9 + f1));
        }
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int n0 = 16 * (2 * s + (2 * p >> 2)) + 4 * kk + (2 * p & 3);
                a2[q][s][p] = pack_hi16(bits(true, OW2 + (16 * q + c) * 64 + n0),
                                        bits(true, OW2 + (16 * q + c) * 64 + n0 + 1));
            }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            b1[q][r] = w(OB1 + 16 * q + 4 * kk + r);
            b2[q][r] = w(OB2 + 16 * q + 4 * kk + r);
        }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int n0 = 16 * (2 * s + (2 * p >> 2)) + 4 * kk + (2 * p & 3);
            a3[s][p] = pack_hi16(bits(c < 6, OW3 + c * 64 + n0), bits(c < 6, OW3 + c * 64 + n0 + 1));
        }
#pragma unroll
    for (int r = 0; r < 4; ++r) b3[r] = (4 * kk + r < 6) ? w(OB3 + 4 * kk + r) : 0.f;

    const long nblk = (M + 15) / 16;
    const long wv = (long)blockIdx.x * (MB / 64) + (threadIdx.x >> 6);
    const long nwv = (long)gridDim.x * (MB / 64);
    // inputs of a block, loaded from clamped addresses without a branch (M >= 1) so that the
    // loads stay in flight until layer1 uses them; values past the end are zeroed there
    auto load_x = [&](long blk, float (&xr)[3]) {
        const long p = blk * 16 + c;
        const long pc = p < M ? p : M - 1;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int f = 3 * kk + j;
            xr[j] = x9[(f < 9 ? f : 8) * M + pc];
        }
    };
    // layer 1 of a block: h[q][r] = gelu(a1 x + b1), outputs 16 q + 4 kk + r
    auto layer1 = [&](long blk, const float (&xr)[3], float (&h)[4][4]) {
        const bool inb = blk * 16 + c < M;
        float xv[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < 3; ++j) xv[j] = (inb && 3 * kk + j < 9) ? xr[j] * in_inv : 0.f;
        v4u xh, xm, xl;
        split3(xv, xh, xm, xl);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v4f d = mfma32(a1[q], xl, b1[q]);
            d = mfma32(a1[q], xm, d);
            d = mfma32(a1[q], xh, d);
#pragma unroll
            for (int r = 0; r < 4; ++r) h[q][r] = gelu(d[r]);
        }
    };
    // software pipeline: layer 1 of the wavefront's next block runs while this block's
    // layer 2 is on the matrix cores, and the loads run two blocks ahead
    float xn[3], h[4][4];
    load_x(wv, xn);
    layer1(wv, xn, h);
    load_x(wv + nwv, xn);
    for (long blk = wv; blk < nblk; blk += nwv) {
        v4f d2[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) d2[q] = b2[q];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const float hv[8] = {h[2 * s][0],     h[2 * s][1],     h[2 * s][2],     h[2 * s][3],
                                 h[2 * s + 1][0], h[2 * s + 1][1], h[2 * s + 1][2], h[2 * s + 1][3]};
            v4u hh, hm, hl;
            split3(hv, hh, hm, hl);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                d2[q] = mfma32(a2[q][s], hl, d2[q]);
                d2[q] = mfma32(a2[q][s], hm, d2[q]);
                d2[q] = mfma32(a2[q][s], hh, d2[q]);
            }
        }
        // the next block's layer 1 (inputs zero past the last block; nothing of it is stored)
        const float xc[3] = {xn[0], xn[1], xn[2]};
        load_x(blk + 2 * nwv, xn);
        layer1(blk + nwv, xc, h);
        v4f d3 = b3;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            float gv[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) gv[j] = gelu(d2[2 * s + (j >> 2)][j & 3]);
            d3 = mfma32x3(a3[s], gv, d3);
        }
        const long p = blk * 16 + c;
        if (p < M) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (4 * kk + r < 6) y6[(4 * kk + r) * M + p] = d3[r] * out_scale;
        }
    }
}

// ---- loss and backward on the matrix cores -----------------------------------------------------------
// One wavefront walks 16-point blocks as the forward does, and per block:
//   the forward, on the FP32 instruction (outputs in k_mlp_fwd's accumulator layout),
//   keeping gelu'(a1) and gelu'(a2) beside h1 and h2;
//   dy = 2 (y - t / out_scale) / (6 M) with loss += (y - t / out_scale)^2, or the given dy;
//   da2 = (W3^T dy) gelu'(a2) and da1 = (W2^T da2) gelu'(a1), products in the forward's
//   layout (the transposed weights are per-lane A operands too);
//   the weight gradients, sums over points: gW1 += da1 x^T, gW2 += da2 h1^T, gW3 += dy h2^T.
// In those the contraction runs over the block's 16 points, four per instruction, whereas
// the activations sit with one point per lane: the factors go through the wavefront's own
// LDS as [feature][point] tiles and come back with the points along the K slots.  A lane
// reads (feature 16 t + c, point 4 s + kk), so accumulator tile (t, t') holds, at lane
// (kk, c), gradient entries (16 t + 4 kk + r, 16 t' + c).  The bias gradients are per-lane
// sums of da1, da2 and dy, reduced over the 16 lanes of a point block at the end.  Every
// workgroup leaves one partial sum per parameter (its waves added in a fixed order).
constexpr int TS = 20;  // row stride of the LDS tiles: at most two lanes of a wavefront per bank
constexpr int WT = (4 * 64 + 2 * 16) * TS;

__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

__global__ __launch_bounds__(MB) void k_mlp_bwd(const uint16_t *__restrict__ wb, const float *__restrict__ x9,
                                               const float *__restrict__ t6, const float *__restrict__ dy6, long M,
                                               float in_inv, float out_inv, float *__restrict__ part,
                                               double *__restrict__ lpart) {
    constexpr int NW = MB / 64;
    __shared__ float tiles[NW * WT];
    // W2 as the A operands of layer 2 (forward) and of W2^T da2 (backward), four steps r
    // per lane in one 16-byte read: [q][qi][lane][r]
    __shared__ float4 sW2[16 * 64], sW2t[16 * 64];
    __shared__ double sh[NW];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int kk = lane >> 4, c = lane & 15;
    float *sH1 = tiles + wid * WT, *sH2 = sH1 + 64 * TS, *sD1 = sH2 + 64 * TS, *sD2 = sD1 + 64 * TS;
    float *sX = sD2 + 64 * TS, *sDY = sX + 16 * TS;
    auto w = [&](int i) { return bf16_f32(wb[i]); };
    // forward operands as in k_mlp_fwd (W2's from the LDS); backward ones:
    //   W3^T dy, step s:       A[c][kk] = W3[4 s + kk][16 q + c] (outputs 6, 7 zero)
    //   W2^T da2, step (qi, r): A[c][kk] = W2[16 qi + 4 kk + r][16 q + c]
    for (int e = threadIdx.x; e < 16 * 64; e += MB) {
        const int q = e >> 8, qi = (e >> 6) & 3, l = e & 63, lk = l >> 4, lc = l & 15;
        float4 f, g;
        f.x = w(OW2 + (16 * q + lc) * 64 + 16 * qi + 4 * lk + 0);
        f.y = w(OW2 + (16 * q + lc) * 64 + 16 * qi + 4 * lk + 1);
        f.z = w(OW2 + (16 * q + lc) * 64 + 16 * qi + 4 * lk + 2);
        f.w = w(OW2 + (16 * q + lc) * 64 + 16 * qi + 4 * lk + 3);
        g.x = w(OW2 + (16 * qi + 4 * lk + 0) * 64 + 16 * q + lc);
        g.y = w(OW2 + (16 * qi + 4 * lk + 1) * 64 + 16 * q + lc);
        g.z = w(OW2 + (16 * qi + 4 * lk + 2) * 64 + 16 * q + lc);
        g.w = w(OW2 + (16 * qi + 4 * lk + 3) * 64 + 16 * q + lc);
        sW2[e] = f;
        sW2t[e] = g;
    }
    __syncthreads();
    float a1[4][3], a3[16], a3t[4][2];
    v4f b1[4], b2[4], b3;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int t = 0; t < 3; ++t) a1[q][t] = (4 * t + kk < 9) ? w(OW1 + (16 * q + c) * 9 + 4 * t + kk) : 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            b1[q][r] = w(OB1 + 16 * q + 4 * kk + r);
            b2[q][r] = w(OB2 + 16 * q + 4 * kk + r);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) a3t[q][s] = (4 * s + kk < 6) ? w(OW3 + (4 * s + kk) * 64 + 16 * q + c) : 0.f;
    }
#pragma unroll
    for (int qi = 0; qi < 4; ++qi)
#pragma unroll
        for (int r = 0; r < 4; ++r) a3[4 * qi + r] = c < 6 ? w(OW3 + c * 64 + 16 * qi + 4 * kk + r) : 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) b3[r] = (4 * kk + r < 6) ? w(OB3 + 4 * kk + r) : 0.f;
    // rows 12..15 of the input tile and 8..15 of the output-gradient tile stay zero
    for (int i = lane; i < 32 * TS; i += 64) sX[i] = 0.f;

    const v4f z4 = {0.f, 0.f, 0.f, 0.f};
    v4f gw1[4], gw2[4][4], gw3[4];
    float gb1[4][4], gb2[4][4], gb3[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        gw1[q] = z4;
        gw3[q] = z4;
        gb3[q] = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            gw2[q][r] = z4;
            gb1[q][r] = 0.f;
            gb2[q][r] = 0.f;
        }
    }
    double lacc = 0;
    const float dscale = 2.0f / (6.0f * (float)M);
    const long nblk = (M + 15) / 16;
    const long wv = (long)blockIdx.x * NW + wid;
    const long nwv = (long)gridDim.x * NW;
    // a block's inputs and targets (or given output gradients): lane (kk, c) takes input
    // features 4 t + kk and outputs 4 kk + r of point c
    auto load = [&](long blk, float (&xv)[3], float (&tv)[4]) {
        const long p = blk * 16 + c;
        const bool in = blk < nblk && p < M;
#pragma unroll
        for (int t = 0; t < 3; ++t) xv[t] = (in && 4 * t + kk < 9) ? x9[(4 * t + kk) * M + p] * in_inv : 0.f;
        const float *src = t6 ? t6 : dy6;
#pragma unroll
        for (int r = 0; r < 4; ++r) tv[r] = (in && 4 * kk + r < 6) ? src[(4 * kk + r) * M + p] : 0.f;
    };
    float xn[3], tn[4];
    load(wv, xn, tn);
    for (long blk = wv; blk < nblk; blk += nwv) {
        const bool in = blk * 16 + c < M;
        float xv[3] = {xn[0], xn[1], xn[2]};
        float tv[4] = {tn[0], tn[1], tn[2], tn[3]};
        load(blk + nwv, xn, tn);  // the next block's, in flight during this one
        // forward
        v4f d1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            d1[q] = b1[q];
#pragma unroll
            for (int t = 0; t < 3; ++t) d1[q] = mfma4(a1[q][t], xv[t], d1[q]);
        }
        float h1[4][4], g1[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                h1[q][r] = gelu(d1[q][r]);
                g1[q][r] = gelu_grad(d1[q][r]);
            }
        v4f d2[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            d2[q] = b2[q];
#pragma unroll
            for (int qi = 0; qi < 4; ++qi) {
                const float4 a = sW2[(4 * q + qi) * 64 + lane];
                d2[q] = mfma4(a.x, h1[qi][0], d2[q]);
                d2[q] = mfma4(a.y, h1[qi][1], d2[q]);
                d2[q] = mfma4(a.z, h1[qi][2], d2[q]);
                d2[q] = mfma4(a.w, h1[qi][3], d2[q]);
            }
        }
        float h2[4][4], g2[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                h2[q][r] = gelu(d2[q][r]);
                g2[q][r] = gelu_grad(d2[q][r]);
            }
        v4f d3q[4];
#pragma unroll
        for (int qi = 0; qi < 4; ++qi) {
            d3q[qi] = qi == 0 ? b3 : z4;
#pragma unroll
            for (int r = 0; r < 4; ++r) d3q[qi] = mfma4(a3[4 * qi + r], h2[qi][r], d3q[qi]);
        }
        const v4f d3 = (d3q[0] + d3q[1]) + (d3q[2] + d3q[3]);
        float dyv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float g = 0.f;
            if (in && 4 * kk + r < 6) {
                if (t6) {
                    const float d = d3[r] - tv[r] * out_inv;
                    lacc += (double)d * d;
                    g = d * dscale;
                } else {
                    g = tv[r];
                }
            }
            dyv[r] = g;
            gb3[r] += g;
        }
        // the block's tiles as [feature][point]
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                sH1[(16 * q + 4 * kk + r) * TS + c] = h1[q][r];
                sH2[(16 * q + 4 * kk + r) * TS + c] = h2[q][r];
            }
#pragma unroll
        for (int t = 0; t < 3; ++t) sX[(4 * t + kk) * TS + c] = xv[t];
        if (kk < 2) {
#pragma unroll
            for (int r = 0; r < 4; ++r) sDY[(4 * kk + r) * TS + c] = dyv[r];
        }
        wave_lds_sync();
        // da2 = (W3^T dy) gelu'(a2); da1 = (W2^T da2) gelu'(a1)
        const float bdy0 = sDY[kk * TS + c], bdy1 = sDY[(4 + kk) * TS + c];
        float da2[4][4], da1[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v4f e = mfma4(a3t[q][0], bdy0, z4);
            e = mfma4(a3t[q][1], bdy1, e);
#pragma unroll
            for (int r = 0; r < 4; ++r) da2[q][r] = e[r] * g2[q][r];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v4f e = z4;
#pragma unroll
            for (int qi = 0; qi < 4; ++qi) {
                const float4 a = sW2t[(4 * q + qi) * 64 + lane];
                e = mfma4(a.x, da2[qi][0], e);
                e = mfma4(a.y, da2[qi][1], e);
                e = mfma4(a.z, da2[qi][2], e);
                e = mfma4(a.w, da2[qi][3], e);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) da1[q][r] = e[r] * g1[q][r];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                gb1[q][r] += da1[q][r];
                gb2[q][r] += da2[q][r];
                sD1[(16 * q + 4 * kk + r) * TS + c] = da1[q][r];
                sD2[(16 * q + 4 * kk + r) * TS + c] = da2[q][r];
            }
        wave_lds_sync();
        // weight gradients: the block's points as the contraction, four per step
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int pc = 4 * s + kk;
            const float xb = sX[c * TS + pc];
            const float ya = sDY[c * TS + pc];
            float h1b[4], h2b[4], d1a[4], d2a[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                h1b[t] = sH1[(16 * t + c) * TS + pc];
                h2b[t] = sH2[(16 * t + c) * TS + pc];
                d1a[t] = sD1[(16 * t + c) * TS + pc];
                d2a[t] = sD2[(16 * t + c) * TS + pc];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                gw1[t] = mfma4(d1a[t], xb, gw1[t]);
                gw3[t] = mfma4(ya, h2b[t], gw3[t]);
#pragma unroll
                for (int t2 = 0; t2 < 4; ++t2) gw2[t][t2] = mfma4(d2a[t], h1b[t2], gw2[t][t2]);
            }
        }
        wave_lds_sync();  // this block's tile reads are done before the next block writes
    }
    // bias gradients: sums over the 16 lanes of each point block
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                gb1[q][r] += __shfl_xor(gb1[q][r], o, 64);
                gb2[q][r] += __shfl_xor(gb2[q][r], o, 64);
            }
            gb3[q] += __shfl_xor(gb3[q], o, 64);
        }
    }
    // the workgroup's partial sums: wave 0 writes, waves 1.. add in order
    float *red = tiles;
    __syncthreads();
    for (int v = 0; v < NW; ++v) {
        if (wid == v) {
            auto put = [&](int j, float x) { red[j] = v == 0 ? x : red[j] + x; };
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int o = 16 * t + 4 * kk + r;
#pragma unroll
                    for (int t2 = 0; t2 < 4; ++t2) put(OW2 + o * 64 + 16 * t2 + c, gw2[t][t2][r]);
                    if (c < 9) put(OW1 + o * 9 + c, gw1[t][r]);
                    if (4 * kk + r < 6) put(OW3 + (4 * kk + r) * 64 + 16 * t + c, gw3[t][r]);
                    if (c == 0) {
                        put(OB1 + o, gb1[t][r]);
                        put(OB2 + o, gb2[t][r]);
                    }
                }
            if (c == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (4 * kk + r < 6) put(OB3 + 4 * kk + r, gb3[r]);
            }
        }
        __syncthreads();
    }
    for (int j = threadIdx.x; j < NP; j += MB) part[(long)blockIdx.x * NP + j] = red[j];
    if (t6) {
        lacc = block_sum(lacc, sh);
        if (threadIdx.x == 0) lpart[blockIdx.x] = lacc;
    }
}

// Fixed-order FP64 sum of the workgroups' partials: 16 parameters per workgroup, sixteen
// interleaved runs over the partials, added in a fixed order.
constexpr int SUM_J = 16, SUM_G = 16;
__global__ __launch_bounds__(SUM_J * SUM_G) void k_mlp_bwd_sum(const float *__restrict__ part, int npart,
                                                               float *__restrict__ grad) {
    __shared__ double sh[SUM_G][SUM_J];
    const int jl = threadIdx.x % SUM_J, sg = threadIdx.x / SUM_J;
    const int j = blockIdx.x * SUM_J + jl;
    double a = 0;
    if (j < NP)
        for (int s = sg; s < npart; s += SUM_G) a += (double)part[(long)s * NP + j];
    sh[sg][jl] = a;
    __syncthreads();
    if (sg == 0 && j < NP) {
        double r = sh[0][jl];
        for (int g = 1; g < SUM_G; ++g) r += sh[g][jl];
        grad[j] = (float)r;
    }
}

// ---- Adam (Kingma & Ba) ---------------------------------------------------------------------------
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, uint16_t *__restrict__ wb, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < NP) {
        const float gj = g[j];
        const float mj = b1 * m[j] + (1.f - b1) * gj;
        const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
        m[j] = mj;
        v[j] = vj;
        const float wj = w[j] - lr * (mj / c1) / (sqrtf(vj / c2) + eps);
        w[j] = wj;
        wb[j] = f32_bf16(wj);
    }
}

__global__ void k_to_bf16(const float *__restrict__ w, uint16_t *__restrict__ wb, int n) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) wb[j] = f32_bf16(w[j]);
}

__global__ void k_count_nonfinite(const uint16_t *__restrict__ wb, int n, int *__restrict__ cnt) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n && (wb[j] & 0x7f80u) == 0x7f80u) atomicAdd(cnt, 1);
}

// ---- spectral helpers ---------------------------------------------------------------------------------
// g[3 i + j] = i k_j u^_i (Nyquist derivative taken as zero), 9 fields in the state layout.
// Only modes with |kx|, |ky|, kz <= K are read (the others are zero in a 2/3-masked state,
// and the solver's stage buffers leave them unwritten); u has rows of `rowlen` complex
// values per (x, y): N/2+1 for a state, the transit length for a stage buffer.
__global__ void k_grad_spec(const float2 *__restrict__ u, float2 *__restrict__ g, int N, int K, int rowlen) {
    const int NZH = N / 2 + 1;
    const long FS = (long)N * N * NZH;
    const long FSu = (long)N * N * rowlen;
    for (long m = (long)blockIdx.x * blockDim.x + threadIdx.x; m < FS; m += (long)gridDim.x * blockDim.x) {
        const int kz0 = (int)(m % NZH);
        const long xy = m / NZH;
        const int y = (int)(xy % N), x = (int)(xy / N);
        const int k[3] = {2 * x == N ? 0 : (x < N / 2 ? x : x - N), 2 * y == N ? 0 : (y < N / 2 ? y : y - N),
                          2 * kz0 == N ? 0 : kz0};
        const bool kept = abs(x < N / 2 ? x : x - N) <= K && abs(y < N / 2 ? y : y - N) <= K && kz0 <= K;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float2 a = kept ? u[i * FSu + xy * rowlen + kz0] : make_float2(0.f, 0.f);
#pragma unroll
            for (int j = 0; j < 3; ++j) g[(3 * i + j) * FS + m] = make_float2(-a.y * k[j], a.x * k[j]);
        }
    }
}

// add3_i = -i sum_j k_j tau^_ij, tau components (xx, yy, zz, xy, xz, yz).
__global__ void k_sgs_div(const float2 *__restrict__ th, float2 *__restrict__ add3, int N) {
    const int NZH = N / 2 + 1;
    const long FS = (long)N * N * NZH;
    for (long m = (long)blockIdx.x * blockDim.x + threadIdx.x; m < FS; m += (long)gridDim.x * blockDim.x) {
        const int kz0 = (int)(m % NZH);
        const long xy = m / NZH;
        const int y = (int)(xy % N), x = (int)(xy / N);
        const float k0 = 2 * x == N ? 0 : (x < N / 2 ? x : x - N), k1 = 2 * y == N ? 0 : (y < N / 2 ? y : y - N),
                    k2 = 2 * kz0 == N ? 0 : kz0;
        const float2 xx = th[m], yy = th[FS + m], zz = th[2 * FS + m], xy_ = th[3 * FS + m], xz = th[4 * FS + m],
                     yz = th[5 * FS + m];
        const float2 s0 = make_float2(k0 * xx.x + k1 * xy_.x + k2 * xz.x, k0 * xx.y + k1 * xy_.y + k2 * xz.y);
        const float2 s1 = make_float2(k0 * xy_.x + k1 * yy.x + k2 * yz.x, k0 * xy_.y + k1 * yy.y + k2 * yz.y);
        const float2 s2 = make_float2(k0 * xz.x + k1 * yz.x + k2 * zz.x, k0 * xz.y + k1 * yz.y + k2 * zz.y);
        // -i s = (s.y, -s.x)
        add3[m] = make_float2(s0.y, -s0.x);
        add3[FS + m] = make_float2(s1.y, -s1.x);
        add3[2 * FS + m] = make_float2(s2.y, -s2.x);
    }
}

// Box filter by truncation: modes |kx|, |ky|, kz <= kc of an n1 half spectrum onto an n2
// half spectrum (zero elsewhere), nf fields.
__global__ void k_truncate(const float2 *__restrict__ src, int n1, float2 *__restrict__ dst, int n2, int kc,
                           int nf) {
    const int h1 = n1 / 2 + 1, h2 = n2 / 2 + 1;
    const long F2 = (long)n2 * n2 * h2, F1 = (long)n1 * n1 * h1;
    for (long m = (long)blockIdx.x * blockDim.x + threadIdx.x; m < F2 * nf; m += (long)gridDim.x * blockDim.x) {
        const int f = (int)(m / F2);
        const long r = m % F2;
        const int kz = (int)(r % h2);
        const long xy = r / h2;
        const int y = (int)(xy % n2), x = (int)(xy / n2);
        const int kx = x < n2 / 2 ? x : x - n2, ky = y < n2 / 2 ? y : y - n2;
        float2 v = make_float2(0.f, 0.f);
        if (abs(kx) <= kc && abs(ky) <= kc && kz <= kc) {
            const int sx = kx < 0 ? kx + n1 : kx, sy = ky < 0 ? ky + n1 : ky;
            v = src[f * F1 + ((long)sx * n1 + sy) * h1 + kz];
        }
        dst[m] = v;
    }
}

__global__ void k_mul(const float *__restrict__ a, const float *__restrict__ b, float *__restrict__ o, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        o[i] = a[i] * b[i];
}

// a -= b on the modes |kx|, |ky|, kz <= kc of an n-grid half spectrum (one field).
__global__ void k_sub_kept(const float2 *__restrict__ b, float2 *__restrict__ a, int n, int kc) {
    const int h = n / 2 + 1;
    const long F = (long)n * n * h;
    for (long m = (long)blockIdx.x * blockDim.x + threadIdx.x; m < F; m += (long)gridDim.x * blockDim.x) {
        const int kz = (int)(m % h);
        const long xy = m / h;
        const int y = (int)(xy % n), x = (int)(xy / n);
        const int kx = x < n / 2 ? x : x - n, ky = y < n / 2 ? y : y - n;
        if (abs(kx) <= kc && abs(ky) <= kc && kz <= kc) {
            const float2 u = a[m], v = b[m];
            a[m] = make_float2(u.x - v.x, u.y - v.y);
        }
    }
}

static unsigned ew_blocks(long n) { return (unsigned)std::min<long>(16384, std::max<long>(1, (n + 255) / 256)); }

// ---- backward scratch (grow-only, per process) ---------------------------------------------------------
struct BwdScratch {
    std::mutex mu;  // guards the allocation; the buffers themselves are shared (see tk.h)
    float *part = nullptr;
    double *lpart = nullptr;
    int dev = -1;
};
static BwdScratch g_bwd;
constexpr int BWD_MAXG = 1024;  // at most this many workgroups leave partial sums

static tk_status bwd_scratch(float **part, double **lpart) {
    int dev = 0;
    TK_HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_bwd.mu);
    if (!g_bwd.part || dev != g_bwd.dev) {
        if (g_bwd.part) hipFree(g_bwd.part);
        if (g_bwd.lpart) hipFree(g_bwd.lpart);
        g_bwd.part = nullptr;
        g_bwd.lpart = nullptr;
        if (hipMalloc((void **)&g_bwd.part, sizeof(float) * (size_t)NP * BWD_MAXG) != hipSuccess ||
            hipMalloc((void **)&g_bwd.lpart, sizeof(double) * BWD_MAXG) != hipSuccess)
            return fail(TK_ENOMEM, "network backward scratch allocation failed");
        g_bwd.dev = dev;
    }
    *part = g_bwd.part;
    *lpart = g_bwd.lpart;
    return TK_OK;
}

static tk_status mlp_check(const tk_mlp *w) {
    if (!w || !w->w) return fail(TK_EINVAL, "network weights are NULL");
    if (!(w->in_scale > 0) || !(w->out_scale > 0) || !std::isfinite(w->in_scale) || !std::isfinite(w->out_scale))
        return fail(TK_EINVAL, "network scales must be finite and > 0");
    return TK_OK;
}

tk_status mlp_forward_run(const tk_mlp *w, const float *x9, float *y6, long M, hipStream_t s) {
    if (M <= 0) return TK_OK;  // the kernel's clamped loads need one point
    // as many workgroups as are resident (each wavefront walks 16-point blocks), no more
    // than there are blocks
    const long nblk = (M + 15) / 16;
    const long G = std::min<long>(resident_groups(reinterpret_cast<const void *>(&k_mlp_fwd), MB),
                                  std::max<long>(1, (nblk + MB / 64 - 1) / (MB / 64)));
    hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)G), dim3(MB), 0, s, (const uint16_t *)w->w, x9, y6, M,
                       1.0f / w->in_scale, w->out_scale);
    return launch_check("network forward");
}

static tk_status mlp_backward_run(const tk_mlp *w, const float *x9, const float *t6, const float *dy6, long M,
                                  float *grad, double *loss, hipStream_t s) {
    float *part;
    double *lpart;
    TK_TRY(bwd_scratch(&part, &lpart));
    // as many workgroups as are resident (each wavefront walks 16-point blocks), no more
    // than there are blocks
    const long nblk = (M + 15) / 16;
    const int G = (int)std::min<long>(std::min<long>(resident_groups(reinterpret_cast<const void *>(&k_mlp_bwd), MB),
                                                     BWD_MAXG),
                                      std::max<long>(1, (nblk + MB / 64 - 1) / (MB / 64)));
    hipLaunchKernelGGL(k_mlp_bwd, dim3(G), dim3(MB), 0, s, w->w, x9, t6, dy6, M, 1.0f / w->in_scale,
                       1.0f / w->out_scale, part, lpart);
    TK_TRY(launch_check("network backward"));
    hipLaunchKernelGGL(k_mlp_bwd_sum, dim3(cdiv(NP, SUM_J)), dim3(SUM_J * SUM_G), 0, s, part, G, grad);
    TK_TRY(launch_check("network backward (sum)"));
    if (loss) {
        std::vector<double> h(G);
        TK_HIP_CHECK(hipMemcpyAsync(h.data(), lpart, sizeof(double) * G, hipMemcpyDeviceToHost, s));
        TK_HIP_CHECK(hipStreamSynchronize(s));
        double a = 0;
        for (double v : h) a += v;
        *loss = a / (6.0 * (double)M);
    }
    return TK_OK;
}

// ---- LES workspace and one closure evaluation --------------------------------------------------------
void les_work_free(LesWork &w) {
    void *ps[] = {w.gsp, w.greal, w.tau, w.tauh, w.add3, w.backup};
    for (void *p : ps)
        if (p) hipFree(p);
    w = LesWork{};
}

static tk_status les_work_alloc(tk_ns_t p) {
    LesWork &w = p->les;
    if (w.gsp) return TK_OK;
    const int n = p->g.n;
    const size_t fb = p->fbytes;
    const size_t rb = sizeof(float) * (size_t)n * n * n;
    if (hipMalloc(&w.gsp, 9 * fb) != hipSuccess || hipMalloc((void **)&w.greal, 9 * rb) != hipSuccess ||
        hipMalloc((void **)&w.tau, 6 * rb) != hipSuccess || hipMalloc(&w.tauh, 6 * fb) != hipSuccess ||
        hipMalloc(&w.add3, 3 * fb) != hipSuccess || hipMalloc(&w.backup, 3 * fb) != hipSuccess) {
        les_work_free(w);
        return fail(TK_ENOMEM, "LES workspace allocation failed");
    }
    return TK_OK;
}

// add3 = -i k_j tau^_ij with tau = out_scale f(grad(u) / in_scale) evaluated on the grid;
// u_transit: u is the stage buffer (transit layout) rather than the state.
static tk_status les_closure(tk_ns_t p, const tk_mlp *w, const void *u, int u_transit, hipStream_t s) {
    const NsGrid &g = p->g;
    const int n = g.n;
    const long FS = (long)n * n * (n / 2 + 1);
    const long M = (long)n * n * n;
    LesWork &L = p->les;
    hipLaunchKernelGGL(k_grad_spec, dim3(ew_blocks(FS)), dim3(256), 0, s, (const float2 *)u, (float2 *)L.gsp, n, g.K,
                       u_transit ? g.KZP : n / 2 + 1);
    TK_TRY(launch_check("gradient spectra"));
    TK_TRY(fft_x_pass(g.ax, L.gsp, L.gsp, 9, 1, 1.0, s));
    TK_TRY(fft_y_pass(g.ax, L.gsp, L.gsp, 9, 1, s));
    TK_TRY(fft_z_c2r(g.ax, L.gsp, L.greal, 9, s));
    TK_TRY(mlp_forward_run(w, L.greal, L.tau, M, s));
    TK_TRY(fft_z_r2c(g.ax, L.tau, L.tauh, 6, 1.0, s));
    TK_TRY(fft_y_pass(g.ax, L.tauh, L.tauh, 6, 0, s));
    TK_TRY(fft_x_pass(g.ax, L.tauh, L.tauh, 6, 0, 1.0 / (double)M, s));
    hipLaunchKernelGGL(k_sgs_div, dim3(ew_blocks(FS)), dim3(256), 0, s, (const float2 *)L.tauh, (float2 *)L.add3, n);
    return launch_check("stress divergence");
}

static tk_status les_steps(tk_ns_t p, const tk_mlp *w, void *u, int nsteps, hipStream_t s) {
    const NsGrid &g = p->g;
    P5Args a{};
    a.u = u;
    a.aux = p->aux;
    a.ust = p->ust;
    a.st = p->st;
    a.nu = p->cfg.nu;
    for (int k = 0; k < nsteps; ++k) {
        if (w) TK_TRY(les_closure(p, w, u, 0, s));
        a.add3 = w ? p->les.add3 : nullptr;
        a.mode = RK2_S1;
        TK_TRY(ns_rhs_eval(g, u, p->w6, a, p->umax_part, p->st, s));
        if (w) TK_TRY(les_closure(p, w, p->ust, 1, s));
        a.mode = RK2_S2;
        TK_TRY(ns_rhs_eval(g, p->ust, p->w6, a, nullptr, nullptr, s, 1));
    }
    return TK_OK;
}

}  // namespace tk

using namespace tk;

extern "C" tk_status sgs_mlp_forward(const tk_mlp *w, const float *x9, float *y6, long M, void *stream) {
    TK_TRY(mlp_check(w));
    if (!x9 || !y6 || M < 0) return fail(TK_EINVAL, "bad arguments");
    if (M == 0) return TK_OK;
    return mlp_forward_run(w, x9, y6, M, (hipStream_t)stream);
}

extern "C" tk_status sgs_mlp_backward(const tk_mlp *w, const float *x9, const float *dy6, long M, float *grad,
                                      void *stream) {
    TK_TRY(mlp_check(w));
    if (!x9 || !dy6 || !grad || M <= 0) return fail(TK_EINVAL, "bad arguments");
    return mlp_backward_run(w, x9, nullptr, dy6, M, grad, nullptr, (hipStream_t)stream);
}

extern "C" tk_status sgs_mlp_loss_grad(const tk_mlp *w, const float *x9, const float *t6, long M, float *grad,
                                       double *loss, void *stream) {
    TK_TRY(mlp_check(w));
    if (!x9 || !t6 || !grad || M <= 0) return fail(TK_EINVAL, "bad arguments");
    return mlp_backward_run(w, x9, t6, nullptr, M, grad, loss, (hipStream_t)stream);
}

extern "C" tk_status sgs_adam_step(tk_adam *opt, const float *grad, uint16_t *w_bf16, void *stream) {
    if (!opt || !opt->w || !opt->m || !opt->v || !grad || !w_bf16) return fail(TK_EINVAL, "NULL argument");
    if (!(opt->lr > 0) || !(opt->beta1 >= 0 && opt->beta1 < 1) || !(opt->beta2 >= 0 && opt->beta2 < 1))
        return fail(TK_EINVAL, "bad Adam hyper-parameters");
    opt->step += 1;
    const float c1 = (float)(1.0 - std::pow((double)opt->beta1, opt->step));
    const float c2 = (float)(1.0 - std::pow((double)opt->beta2, opt->step));
    hipLaunchKernelGGL(k_adam, dim3(cdiv(NP, 256)), dim3(256), 0, (hipStream_t)stream, opt->w, opt->m, opt->v, grad,
                       w_bf16, opt->lr, opt->beta1, opt->beta2, opt->eps, c1, c2);
    return launch_check("adam");
}

extern "C" tk_status sgs_weights_to_bf16(const float *w, uint16_t *w_bf16, int n, void *stream) {
    if (!w || !w_bf16 || n < 0) return fail(TK_EINVAL, "bad arguments");
    if (n == 0) return TK_OK;
    hipLaunchKernelGGL(k_to_bf16, dim3(cdiv(n, 256)), dim3(256), 0, (hipStream_t)stream, w, w_bf16, n);
    return launch_check("to bf16");
}

extern "C" tk_status les_step(tk_ns_t p, const tk_mlp *w, void *u, double dt, int nsteps, double *t_inout,
                              int *fallback, void *stream) {
    if (!p || !u) return fail(TK_EINVAL, "NULL argument");
    if (nsteps < 0) return fail(TK_EINVAL, "nsteps must be >= 0");
    if (p->cfg.dtype != TK_F32 || p->cfg.scheme != 0) return fail(TK_EUNSUPPORTED, "LES runs FP32 IF-RK2");
    if (p->cfg.cfl <= 0 && !(dt > 0 && std::isfinite(dt))) return fail(TK_EINVAL, "dt must be > 0 without CFL");
    hipStream_t s = (hipStream_t)stream;
    int fb = 0;
    const tk_mlp *model = w;
    if (model) {
        TK_TRY(mlp_check(model));
        // weights that are not finite: plain DNS right-hand side
        int *cnt = (int *)p->dscratch;
        TK_HIP_CHECK(hipMemsetAsync(cnt, 0, sizeof(int), s));
        hipLaunchKernelGGL(k_count_nonfinite, dim3(cdiv(NP, 256)), dim3(256), 0, s, model->w, NP, cnt);
        TK_TRY(launch_check("weight check"));
        int h = 0;
        TK_HIP_CHECK(hipMemcpyAsync(&h, cnt, sizeof(int), hipMemcpyDeviceToHost, s));
        TK_HIP_CHECK(hipStreamSynchronize(s));
        if (h) {
            model = nullptr;
            fb = 1;
        }
    }
    TK_TRY(les_work_alloc(p));
    NsState &h0 = p->hstage;
    h0 = NsState{};
    h0.t = t_inout ? *t_inout : 0.0;
    h0.hfix = dt > 0 ? dt : 0.0;
    h0.cfl_dx = p->cfg.cfl > 0 ? p->cfg.cfl * 2.0 * M_PI / p->cfg.n : 0.0;
    h0.h = h0.hfix;
    TK_HIP_CHECK(hipMemcpyAsync(p->st, &h0, sizeof(h0), hipMemcpyHostToDevice, s));
    TK_HIP_CHECK(hipMemcpyAsync(p->les.backup, u, 3 * p->fbytes, hipMemcpyDeviceToDevice, s));
    TK_TRY(les_steps(p, model, u, nsteps, s));
    if (model) {
        // a state that left the finite numbers: redo the steps with the plain right-hand side
        std::vector<double> hd(NS_DIAG_HEAD + p->nshell);
        TK_TRY(ns_diag_run(u, p->g.n, TK_F32, p->nshell, p->dscratch, hd.data(), s));
        if (!std::isfinite(hd[0])) {
            fb = 2;
            TK_HIP_CHECK(hipMemcpyAsync(u, p->les.backup, 3 * p->fbytes, hipMemcpyDeviceToDevice, s));
            TK_HIP_CHECK(hipMemcpyAsync(p->st, &h0, sizeof(h0), hipMemcpyHostToDevice, s));
            TK_TRY(les_steps(p, nullptr, u, nsteps, s));
        }
    }
    NsState hf{};
    TK_HIP_CHECK(hipMemcpyAsync(&hf, p->st, sizeof(hf), hipMemcpyDeviceToHost, s));
    TK_HIP_CHECK(hipStreamSynchronize(s));
    if (t_inout) *t_inout = hf.t;
    p->last_dt = hf.h;
    if (fallback) *fallback = fb;
    return TK_OK;
}

// Filtered-DNS training data (see tk.h).
extern "C" tk_status les_filter_dns(const void *uhat_dns, int n_dns, int n_les, int kc, float *grad9, float *tau6,
                                    void *ubar_hat, void *stream) {
    if (!uhat_dns || !grad9 || !tau6) return fail(TK_EINVAL, "NULL argument");
    if (!supported_len(n_dns) || !supported_len(n_les) || n_les > n_dns)
        return fail(TK_EUNSUPPORTED, "grids %d -> %d not supported", n_dns, n_les);
    if (kc < 0 || 3 * kc >= n_les) return fail(TK_EINVAL, "cutoff kc=%d must satisfy 3 kc < n_les", kc);
    hipStream_t s = (hipStream_t)stream;
    FftAxes A, B;
    TK_TRY(axes_init(&A, n_dns, n_dns, n_dns, TK_F32, true));
    TK_TRY(axes_init(&B, n_les, n_les, n_les, TK_F32, true));
    const long FD = (long)n_dns * n_dns * (n_dns / 2 + 1), FL = (long)n_les * n_les * (n_les / 2 + 1);
    const long MD = (long)n_dns * n_dns * n_dns, ML = (long)n_les * n_les * n_les;
    void *ud = nullptr, *cd = nullptr, *wsd = nullptr, *prod = nullptr, *ubh = nullptr, *gl = nullptr, *gsp = nullptr,
         *ubr = nullptr, *guu = nullptr;
    auto cleanup = [&]() {
        void *ps[] = {ud, cd, wsd, prod, ubh, gl, gsp, ubr, guu};
        for (void *q : ps)
            if (q) hipFree(q);
    };
#define TK_ALLOC(ptr, bytes)                                                     \
    if (hipMalloc(&ptr, bytes) != hipSuccess) {                                  \
        cleanup();                                                               \
        return fail(TK_ENOMEM, "filter workspace allocation failed");            \
    }
    TK_ALLOC(ud, sizeof(float) * 3 * MD);          // u on the DNS grid
    TK_ALLOC(cd, sizeof(float2) * FD);             // one DNS spectral field
    TK_ALLOC(wsd, sizeof(float2) * FD);            // c2r workspace
    TK_ALLOC(prod, sizeof(float) * MD);            // one product field
    TK_ALLOC(ubh, sizeof(float2) * 3 * FL);        // filtered velocity spectrum
    TK_ALLOC(gl, sizeof(float2) * 6 * FL);         // filtered products spectrum
    TK_ALLOC(gsp, sizeof(float2) * 9 * FL);        // gradient spectra
    TK_ALLOC(ubr, sizeof(float) * 3 * ML);         // filtered velocity, real
    TK_ALLOC(guu, sizeof(float) * ML);             // one coarse product, real
#undef TK_ALLOC
    tk_status st = TK_OK;
    const int pi[6] = {0, 1, 2, 0, 0, 1}, pj[6] = {0, 1, 2, 1, 2, 2};
    do {
        // u on the DNS grid (input preserved: inverse through a workspace copy)
        for (int c = 0; c < 3 && st == TK_OK; ++c) {
            st = fft_x_pass(A, (const float2 *)uhat_dns + c * FD, wsd, 1, 1, 1.0, s);
            if (st == TK_OK) st = fft_y_pass(A, wsd, wsd, 1, 1, s);
            if (st == TK_OK) st = fft_z_c2r(A, wsd, (float *)ud + c * MD, 1, s);
        }
        if (st != TK_OK) break;
        // G(u_i u_j): product on the DNS grid, r2c, truncation onto the coarse grid
        for (int q = 0; q < 6 && st == TK_OK; ++q) {
            hipLaunchKernelGGL(k_mul, dim3(ew_blocks(MD)), dim3(256), 0, s, (const float *)ud + pi[q] * MD,
                               (const float *)ud + pj[q] * MD, (float *)prod, MD);
            st = launch_check("product");
            if (st == TK_OK) st = fft_z_r2c(A, prod, cd, 1, 1.0, s);
            if (st == TK_OK) st = fft_y_pass(A, cd, cd, 1, 0, s);
            if (st == TK_OK) st = fft_x_pass(A, cd, cd, 1, 0, 1.0 / (double)MD, s);
            if (st == TK_OK) {
                hipLaunchKernelGGL(k_truncate, dim3(ew_blocks(FL)), dim3(256), 0, s, (const float2 *)cd, n_dns,
                                   (float2 *)gl + q * FL, n_les, kc, 1);
                st = launch_check("truncate");
            }
        }
        if (st != TK_OK) break;
        // filtered velocity and its gradients on the coarse grid
        hipLaunchKernelGGL(k_truncate, dim3(ew_blocks(3 * FL)), dim3(256), 0, s, (const float2 *)uhat_dns, n_dns,
                           (float2 *)ubh, n_les, kc, 3);
        if ((st = launch_check("truncate u")) != TK_OK) break;
        if (ubar_hat) TK_HIP_CHECK(hipMemcpyAsync(ubar_hat, ubh, sizeof(float2) * 3 * FL, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_grad_spec, dim3(ew_blocks(FL)), dim3(256), 0, s, (const float2 *)ubh, (float2 *)gsp,
                           n_les, kc, n_les / 2 + 1);
        if ((st = launch_check("gradient spectra")) != TK_OK) break;
        if ((st = fft_x_pass(B, gsp, gsp, 9, 1, 1.0, s)) != TK_OK) break;
        if ((st = fft_y_pass(B, gsp, gsp, 9, 1, s)) != TK_OK) break;
        if ((st = fft_z_c2r(B, gsp, grad9, 9, s)) != TK_OK) break;
        // tau = G(u_i u_j) - G(ubar_i ubar_j): ubar in real space on the coarse grid, its
        // products (kept modes exact there by the 2/3 rule) subtracted in spectral space
        if ((st = fft_x_pass(B, ubh, ubh, 3, 1, 1.0, s)) != TK_OK) break;
        if ((st = fft_y_pass(B, ubh, ubh, 3, 1, s)) != TK_OK) break;
        if ((st = fft_z_c2r(B, ubh, ubr, 3, s)) != TK_OK) break;
        for (int q = 0; q < 6 && st == TK_OK; ++q) {
            float *pr = (float *)guu;  // coarse real product
            float2 *pc = (float2 *)gsp;  // coarse spectral product
            hipLaunchKernelGGL(k_mul, dim3(ew_blocks(ML)), dim3(256), 0, s, (const float *)ubr + pi[q] * ML,
                               (const float *)ubr + pj[q] * ML, pr, ML);
            st = launch_check("coarse product");
            if (st == TK_OK) st = fft_z_r2c(B, pr, pc, 1, 1.0, s);
            if (st == TK_OK) st = fft_y_pass(B, pc, pc, 1, 0, s);
            if (st == TK_OK) st = fft_x_pass(B, pc, pc, 1, 0, 1.0 / (double)ML, s);
            if (st == TK_OK) {
                hipLaunchKernelGGL(k_sub_kept, dim3(ew_blocks(FL)), dim3(256), 0, s, (const float2 *)pc,
                                   (float2 *)gl + q * FL, n_les, kc);
                st = launch_check("subtract resolved product");
            }
        }
        if (st != TK_OK) break;
        if ((st = fft_x_pass(B, gl, gl, 6, 1, 1.0, s)) != TK_OK) break;
        if ((st = fft_y_pass(B, gl, gl, 6, 1, s)) != TK_OK) break;
        st = fft_z_c2r(B, gl, tau6, 6, s);
    } while (0);
    if (st == TK_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(TK_EHIP, "filter synchronisation failed");
    cleanup();
    return st;
}
