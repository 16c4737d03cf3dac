// Kernels of the pseudo-spectral Navier-Stokes right-hand side and the integrating-factor
// Runge-Kutta updates (paper, Section "Spectral Solver": eq:NSk with eq:continuity2,
// nonlinear term pseudo-spectral, 2/3-rule dealiasing).
//
// One right-hand side is five passes over HBM:
//   P1  X-inverse with the curl formed on load: u^ (3 fields) -> u^, omega^ = i k x u^
//       (6 fields), transformed along x.
//   P2  Y-inverse on the 6 fields (the generic strided kernel with row masks).
//   P3  Z fused per line: 6 c2r -> c = u x omega (and max |u|_1 for the CFL step) ->
//       3 r2c.  The real-space fields never reach HBM.
//   P4  Y-forward on the 3 fields (generic strided kernel).
//   P5  X-forward with the epilogue: 1/N^3, 2/3 mask, projection P = I - k k^T/|k|^2,
//       then the integrating-factor Runge-Kutta stage combine.
// Every pass touches only what the 2/3 rule keeps: with K = (N-1)/3 a mode survives iff
// |kx|, |ky| <= K and kz <= K; columns and rows that only ever hold masked modes are
// neither read nor written (their values are exact zeros in the unpruned computation).
#pragma once

#include "fft_kernels.hpp"

namespace tk {

// Stage-combine modes of P5.  h and the factors E = exp(-nu |k|^2 h), E2 = exp(-nu|k|^2 h/2)
// come from the device step state; N is the projected, masked nonlinear term.  The
// accumulator aux carries every term of the new state except the last stage's, so the
// last stage does not read u:
//   RK2:  u' = E u + h/2 (E N1 + N2)
//   RK4:  u' = E u + h/6 (E N1 + 2 E2 N2 + 2 E2 N3 + N4)
enum NsMode : int {
    NS_RHS = 0,   // out = N
    RK2_S1 = 1,   // aux = E (u + h/2 N) ;  ust = E (u + h N)
    RK2_S2 = 2,   // u = aux + h/2 N
    RK4_S1 = 3,   // aux = E (u + h/6 N) ;  ust = E2 (u + h/2 N)
    RK4_S2 = 4,   // aux += h/3 E2 N ;      ust = E2 u + h/2 N
    RK4_S3 = 5,   // aux += h/3 E2 N ;      ust = E u + h E2 N
    RK4_S4 = 6    // u = aux + h/6 N
};

// Device step state.
struct NsState {
    double h;        // current step size
    double t;        // time (advanced by h at the start of each step)
    unsigned umax;   // max over grid of |ux| + |uy| + |uz| (float bits): the ensemble's CFL step
    unsigned pad;
    double cfl_dx;   // cfl * 2 pi / N (0: fixed step)
    double hfix;     // fixed step size
};

__device__ __forceinline__ int wave_k(int r, int L) { return r < L / 2 ? r : r - L; }
// Odd (first-derivative) wavenumber: Nyquist taken as zero.
__device__ __forceinline__ int deriv_k(int r, int L) { return (2 * r == L) ? 0 : wave_k(r, L); }

// Column cc of the kept (ky, kz) set: kyi = cc / KZC, kz = cc % KZC; ky index kyi for
// kyi <= K, else kyi + N - 2K - 1 (the negative wavenumbers).  Returns the offset of the
// column inside one field plane row (ky_row * NZH + kz) and the two wavenumbers.
__device__ __forceinline__ long kept_col(long cc, int N, int K, int KZC, int NZH, int *ky, int *kz) {
    int kyi = (int)(cc / KZC);
    *kz = (int)(cc - (long)kyi * KZC);
    int row = kyi <= K ? kyi : kyi + N - 2 * K - 1;
    *ky = wave_k(row, N);
    return (long)row * NZH + *kz;
}

// Transit layout of the workspace fields P1 writes and P2..P5 pass along: only the kz
// columns the 2/3 rule keeps, padded to whole 128-byte lines, KZP = min(roundup(K + 1,
// 16), N/2 + 1) complex values per (x, y) row, so every row segment a pass touches is
// line-aligned (the full N/2+1 rows left partial lines at both ends of each kept run,
// +5..19% HBM traffic by the counters).  Field f, x, y, kz at ((f N + x) N + y) KZP + kz.
// The padding columns carry values no pass depends on.
template <int N> constexpr int ns_kzp() {
    const int kzc = (N - 1) / 3 + 1;
    const int p = (kzc + 15) / 16 * 16;
    return p < N / 2 + 1 ? p : N / 2 + 1;
}

// ---- P1: X-inverse with curl on load -------------------------------------------------------------
// RBC = true: a fourth input field (temperature) is passed through as a seventh output.
// ka scales the wavenumbers of the curl (2 pi / box side).

// Column of a P1 tile for thread (col, jt) = (tid % W, tid / W): column (ky, kz) of the
// kept ky rows and the KZP transit columns; its input point i of field f at element
// f FSi + i TPL RSi (uniform) + lo / sizeof(C), where the input has rows of NZH (the
// state) or, with cin, of KZP (a stage buffer in the transit layout); its output point at
// f FSc + i TPL RSc + lo2 / sizeof(C) of the transit fields.
struct P1Col {
    int ky, kz;
    unsigned lo, lo2;
    bool valid;
};

template <typename T, int L, int E, int W>
__device__ __forceinline__ P1Col ns_p1_col(long tile, int K, int cin) {
    constexpr int N = L;
    constexpr int NZH = N / 2 + 1;
    constexpr int KZP = ns_kzp<N>();
    const long rowi = cin ? KZP : NZH;
    const long RSi = (long)N * rowi;
    constexpr long RSc = (long)N * KZP;
    const int col = threadIdx.x % W;
    const int jt = threadIdx.x / W;
    const long ncols = (long)(2 * K + 1) * KZP;
    const long cc = tile * W + col;
    P1Col c;
    c.valid = cc < ncols;
    c.ky = c.kz = 0;
    long row = 0;
    if (c.valid) {
        const long kyi = cc / KZP;
        c.kz = (int)(cc - kyi * KZP);
        row = kyi <= K ? kyi : kyi + N - 2 * K - 1;
        c.ky = wave_k((int)row, N);
    }
    c.lo = (unsigned)((row * rowi + c.kz + (long)jt * RSi) * (long)sizeof(V2<T>));
    c.lo2 = (unsigned)((row * KZP + c.kz + (long)jt * RSc) * (long)sizeof(V2<T>));
    return c;
}

// The kept x rows of the tile's 3 (RBC: 4) input fields (rows of NZH, or KZP with cin).
template <typename T, int L, int E, int W, bool RBC>
__device__ __forceinline__ void ns_p1_load(const V2<T> *__restrict__ u, const P1Col &c, int K, int cin,
                                           V2<T> (&a0)[E], V2<T> (&a1)[E], V2<T> (&a2)[E],
                                           V2<T> (&a3)[RBC ? E : 1]) {
    constexpr int N = L;
    constexpr int TPL = L / E;
    const long rowi = cin ? ns_kzp<N>() : N / 2 + 1;
    const long FS = (long)N * N * rowi;
    const long RS = (long)N * rowi;
    const int jt = threadIdx.x / W;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const bool ld = c.valid && row_kept(jt + i * TPL, L, K);
        const long ro = (long)(i * TPL) * RS;
        a0[i] = ld ? *at_bytes(u + ro, c.lo) : mk<T>(0, 0);
        a1[i] = ld ? *at_bytes(u + FS + ro, c.lo) : mk<T>(0, 0);
        a2[i] = ld ? *at_bytes(u + 2 * FS + ro, c.lo) : mk<T>(0, 0);
        if constexpr (RBC) a3[i] = ld ? *at_bytes(u + 3 * FS + ro, c.lo) : mk<T>(0, 0);
    }
}

// u^ and omega^ = i k x u^ (and theta^) transformed along x, stored to w6.  ky and kz are
// constant along an x line and the transform is linear, so with U = F(u) (F the inverse
// transform along x) only the kx terms need lines of their own:
//   omega_x = i ky U_z - i kz U_y,  omega_y = i kz U_x - F(i kx u_z),  omega_z = F(i kx u_y) - i ky U_x,
// five line transforms for the six outputs.  Steps: 0 U_x (kept), 1 F(i kx u_y), 2 F(i kx
// u_z), 3 U_y (-i kz U_y kept), 4 U_z, 5 (RBC) theta.
template <typename T, int L, int E, int W, bool RBC>
__device__ __forceinline__ void ns_p1_body(const V2<T> (&a0)[E], const V2<T> (&a1)[E], const V2<T> (&a2)[E],
                                           const V2<T> (&a3)[RBC ? E : 1], V2<T> *__restrict__ w6, const P1Col &c,
                                           V2<T> *lds, const V2<T> *tw, T ka) {
    using C = V2<T>;
    constexpr int N = L;
    constexpr int TPL = L / E;
    constexpr int ES = W + 1;
    constexpr long FSc = (long)N * N * ns_kzp<N>();
    constexpr long RSc = (long)N * ns_kzp<N>();
    const int col = threadIdx.x % W;
    const int jt = threadIdx.x / W;
    const T kyd = ka * (T)c.ky, kzd = ka * (T)((2 * c.kz == N) ? 0 : c.kz);
    auto store = [&](int f, const C(&y)[E]) {
        if (c.valid) {
#pragma unroll
            for (int i = 0; i < E; ++i) *at_bytes(w6 + f * FSc + (long)(i * TPL) * RSc, c.lo2) = y[i];
        }
    };
    // one line transform of the inputs selected by `in`, conjugated back
    auto xform = [&](C(&v)[E], auto in) {
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = cconj(in(i, ka * (T)deriv_k(jt + i * TPL, N)));
        line_fft<T, L, E, ES, 1, 0, true>(v, lds + col, jt, tw);
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = cconj(v[i]);
    };
    C ux[E], v[E];
    xform(ux, [&](int i, T) { return a0[i]; });
    store(0, ux);
    xform(v, [&](int i, T kx) { return cmul_pi(cscale(a1[i], kx)); });
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = csub(v[i], cmul_pi(cscale(ux[i], kyd)));
    store(5, v);
    xform(v, [&](int i, T kx) { return cmul_pi(cscale(a2[i], kx)); });
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = csub(cmul_pi(cscale(ux[i], kzd)), v[i]);
    store(4, v);
    C wx[E];
    xform(v, [&](int i, T) { return a1[i]; });
    store(1, v);
#pragma unroll
    for (int i = 0; i < E; ++i) wx[i] = cmul_pi(cscale(v[i], -kzd));
    xform(v, [&](int i, T) { return a2[i]; });
    store(2, v);
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = cadd(wx[i], cmul_pi(cscale(v[i], kyd)));
    store(3, v);
    if constexpr (RBC) {
        xform(v, [&](int i, T) { return a3[i]; });
        store(6, v);
    }
}

// cin: the input u is a stage buffer in the transit layout (rows of KZP) instead of a
// state with rows of N/2+1.
template <typename T, int L, int E, int W, bool RBC = false>
__device__ __forceinline__ void ns_p1_tile(const V2<T> *__restrict__ u, V2<T> *__restrict__ w6, int K, int cin,
                                           long tile, V2<T> *lds, const V2<T> *tw, T ka = (T)1) {
    using C = V2<T>;
    const P1Col c = ns_p1_col<T, L, E, W>(tile, K, cin);
    C a0[E], a1[E], a2[E], a3[RBC ? E : 1];
    ns_p1_load<T, L, E, W, RBC>(u, c, K, cin, a0, a1, a2, a3);
    ns_p1_body<T, L, E, W, RBC>(a0, a1, a2, a3, w6, c, lds, tw, ka);
}

template <typename T, int L, int E, int W, bool RBC = false>
__global__ __launch_bounds__(W *(L / E)) void k_ns_p1(const V2<T> *__restrict__ u, V2<T> *__restrict__ w6, int K,
                                                       int cin, const V2<T> *__restrict__ twg, T ka) {
    using C = V2<T>;
    __shared__ C lds[L * (W + 1)];
    __shared__ C tw[L];
    load_twiddles<T>(tw, twg, L, threadIdx.x, W * (L / E));
    __syncthreads();
    ns_p1_tile<T, L, E, W, RBC>(u, w6, K, cin, xcd_tile(blockIdx.x, gridDim.x), lds, tw, ka);
}

// ---- P3: fused Z pass ------------------------------------------------------------------------------
// Lines l = x * N + y of the 6 transit fields in w6 (kz < KZC read, the rest taken as
// zero); outputs c = u x omega transformed back, kz < KZP, into fields 0..2 of w6 (in
// place: each workgroup reads all
// six fields of its lines before it writes).  lds: LPW lines of lds_line_len<L>().
// RBC = true: a seventh input (temperature theta) gives three more outputs q = u theta.
// CFL maximum of |u|_1 over the tile's samples: written to part[tile] (one value per
// workgroup, reduced by the step-size kernel), else folded into *umax with one atomic per
// workgroup; neither when both are null.
template <typename T, int L, int E, int LPW, bool RBC = false>
__device__ __forceinline__ void ns_p3_tile(V2<T> *w6, long nlines, int KZC, long tile, V2<T> *lds, const V2<T> *tw,
                                           unsigned *umax, float *part = nullptr) {
    using C = V2<T>;
    constexpr int N = 2 * L;
    constexpr int NZH = L + 1;
    constexpr int TPL = L / E;
    constexpr int LL = lds_line_len<L>();
    constexpr int KZP = ns_kzp<N>();          // transit row length
    constexpr long FS = (long)N * N * KZP;      // transit field stride
    const int tid = threadIdx.x;
    const int ln = tid / TPL;
    const int jt = tid % TPL;
    const long l = tile * LPW + ln;
    const bool valid = l < nlines;
    C *d = lds + ln * LL;
    // real-space samples, packed pairs (x[2n], x[2n+1]) at n = jt + i TPL: u is kept, the
    // three vorticity components are folded into c = u x omega as they arrive
    constexpr int NIN = RBC ? 7 : 6;
    constexpr int NOUT = RBC ? 6 : 3;
    C uu[3][E], c[NOUT][E];
    // the next field's samples are loaded before the current field is transformed, so the
    // loads overlap the transform (the exchange waits only on LDS traffic)
    // Unguarded loads: lanes of an invalid line read line 0 and store nothing; register
    // blocks wholly past the kept columns are zero without a load, and only the block that
    // straddles KZC compares (KZC is the 2/3 rule's (N - 1) / 3 + 1 for every caller).
    constexpr int KZC0 = (N - 1) / 3 + 1;
    auto load = [&](C(&x)[E], int f) {
        const C *s = w6 + f * FS + (valid ? l : 0) * KZP;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int k = jt + i * TPL;
            if (i * TPL >= KZC0) x[i] = mk<T>(0, 0);
            else if ((i + 1) * TPL <= KZC0) x[i] = s[k];
            else x[i] = k < KZC0 ? s[k] : mk<T>(0, 0);
        }
    };
    C nx[E];
    float umx = 0.f;  // lanes of invalid lines hold zeros
    load(nx, 0);
    // (twiddles held in registers for all nine transforms instead of the LDS table cost
    // occupancy and measured no faster at 512^3)
    auto split_tw = [&](int i) { return tw[jt + i * TPL]; };
    // the twiddles of the one stage that has a single butterfly per thread depend on the lane
    // alone: formed once, in registers, for all nine transforms
    constexpr int RS = lane_twiddle_stage<L, E>();
    C wr[E - 1];
    if constexpr (RS > 0) stage_twiddles<T, L, E, 2, RS>(jt, tw, wr);
    auto xform = [&](C(&v)[E]) { line_fft<T, L, E, 1, 2, 0, true, false, RS>(v, d, jt, tw, wr); };
    // The real-FFT merge and split pair X[k] with X[L - k], k = jt + p TPL: for jt > 0 the
    // partner sits in the mirror lane TPL - jt, register E - 1 - p, and lane 0 pairs register p
    // with its own register E - p (register 0 with the Nyquist mode, register E / 2 with
    // itself).  Both results of a pair come from the same sums, so each lane forms the pairs
    // of its registers p < E / 2 only: the merge hands the partner's result back through the
    // shuffle, the split stores it at column L - k.
    constexpr int H = E / 2;
    const int src = (tid & 63) - jt + ((TPL - jt) & (TPL - 1));
    auto shfl2 = [&](const C &x) {
        if constexpr (TPL > 1) {
            C q;
            q.x = __shfl(x.x, src, 64);
            q.y = __shfl(x.y, src, 64);
            return q;
        } else {
            return x;
        }
    };
#pragma unroll
    for (int f = 0; f < NIN; ++f) {
        C v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = nx[i];
        if (f + 1 < NIN) load(nx, f + 1);
        // c2r merge.  Register r holds X[jt + r TPL], zero on every lane when r TPL >= KZC0:
        // a pair whose own or partner register is such a register leaves those terms out at
        // compile time, and the shuffle that would fetch the zero with them.  X[L] (the
        // partner of lane 0's register 0) is a masked mode, and X[0] counts with its real part.
        // Pairs from the last to the first: pair p writes its own register p and register
        // E - 1 - p, which takes the mirror lane's partner result (lane 0: its own result of
        // pair p + 1, formed one step before; for p = E/2 - 1 its self-paired register E/2,
        // 2 X[L/2]).  No register is read after it is written, in any lane.
        const C xh = v[H];
        C hnext = mk<T>(0, 0);
#pragma unroll
        for (int p = H - 1; p >= 0; --p) {
            const bool xk_zero = p * TPL >= KZC0;
            const bool xc_zero = (E - 1 - p) * TPL >= KZC0;  // lane 0's partner E - p as well
            C xk = v[p];
            if (p == 0) xk.y = jt == 0 ? (T)0 : xk.y;
            C a, dd;
            if (xc_zero) {
                a = xk;
                dd = xk;
            } else {
                const C s = shfl2(v[E - 1 - p]);
                const C xp = jt != 0 ? s : (p == 0 ? mk<T>(0, 0) : v[(E - p) % E]);
                const C xc = cconj(xp);
                if (xk_zero) {
                    a = xc;
                    dd = mk<T>(-xc.x, -xc.y);
                } else {
                    a = cadd(xk, xc);
                    dd = csub(xk, xc);
                }
            }
            const C b = cmul(cconj(split_tw(p)), dd);
            const C hi = mk<T>(a.x + b.y, a.y - b.x);  // conj Z'[L - k]
            v[p] = mk<T>(a.x - b.y, -(a.y + b.x));     // conj Z'[k]
            const C m = shfl2(hi);
            const C own = p == H - 1 ? mk<T>(2 * xh.x, 2 * xh.y) : hnext;
            v[E - 1 - p] = jt != 0 ? m : own;
            hnext = hi;
        }
        xform(v);
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const C w = mk<T>(v[i].x, -v[i].y);
            if (f < 3) {
                uu[f][i] = w;
            } else if (f == 3) {  // omega_x: c_y += u_z w, c_z = -u_y w
                c[0][i] = mk<T>(0, 0);
                c[1][i] = mk<T>(uu[2][i].x * w.x, uu[2][i].y * w.y);
                c[2][i] = mk<T>(-uu[1][i].x * w.x, -uu[1][i].y * w.y);
            } else if (f == 4) {  // omega_y: c_x -= u_z w, c_z += u_x w
                c[0][i] = mk<T>(c[0][i].x - uu[2][i].x * w.x, c[0][i].y - uu[2][i].y * w.y);
                c[2][i] = mk<T>(c[2][i].x + uu[0][i].x * w.x, c[2][i].y + uu[0][i].y * w.y);
            } else if (f == 5) {  // omega_z: c_x += u_y w, c_y -= u_x w
                c[0][i] = mk<T>(c[0][i].x + uu[1][i].x * w.x, c[0][i].y + uu[1][i].y * w.y);
                c[1][i] = mk<T>(c[1][i].x - uu[0][i].x * w.x, c[1][i].y - uu[0][i].y * w.y);
            } else if constexpr (RBC) {  // theta: q_j = u_j theta
#pragma unroll
                for (int jj = 0; jj < 3; ++jj) c[3 + jj][i] = mk<T>(uu[jj][i].x * w.x, uu[jj][i].y * w.y);
            }
        }
        if (f == 2 && (umax || part)) {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const float s0 = (float)(fabs(uu[0][i].x) + fabs(uu[1][i].x) + fabs(uu[2][i].x));
                const float s1 = (float)(fabs(uu[0][i].y) + fabs(uu[1][i].y) + fabs(uu[2][i].y));
                umx = fmaxf(umx, fmaxf(s0, s1));
            }
        }
    }
    // forward r2c of the products (unscaled; P5 applies 1/N^3), kz < KZP (whole transit rows:
    // the padding values are never used); the pairs as in the merge
#pragma unroll
    for (int f = 0; f < NOUT; ++f) {
        C v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = c[f][i];
        xform(v);
        C *o = w6 + f * FS + l * KZP;
        const C zh = v[H];
#pragma unroll
        for (int p = 0; p < H; ++p) {
            const C s = shfl2(v[E - 1 - p]);
            const C zc = cconj(jt != 0 ? s : v[(E - p) % E]);  // Z[L - k] (lane 0, p = 0: Z[0])
            const C a = cadd(v[p], zc);
            const C b = cmul(split_tw(p), csub(v[p], zc));
            const int k = jt + p * TPL;
            if (valid) {
                if (k < KZP) o[k] = mk<T>((T)0.5 * (a.x + b.y), (T)0.5 * (a.y - b.x));  // X[k]
                // X[L - k]: column L - k >= (E - 1 - p) TPL + 1, stored only where it can be kept
                if ((E - 1 - p) * TPL + 1 < KZP && (jt != 0 || p != 0) && L - k < KZP)
                    o[L - k] = mk<T>((T)0.5 * (a.x - b.y), (T)-0.5 * (a.y + b.x));
            }
        }
        if (valid) {
            // lane 0's register H pairs with itself: X[L/2] = conj Z[L/2]
            if (jt == 0 && L / 2 < KZP) o[L / 2] = cconj(zh);
        }
    }
    if (umax || part) {
        __shared__ float wmax[16];
        for (int o = 32; o > 0; o >>= 1) umx = fmaxf(umx, __shfl_xor(umx, o, 64));
        if ((tid & 63) == 0) wmax[tid >> 6] = umx;
        __syncthreads();
        if (tid == 0) {
            float m = wmax[0];
            for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, wmax[w]);
            if (part) part[tile] = m;
            else atomicMax(umax, __float_as_uint(m));
        }
    }
}

template <typename T, int L, int E, int LPW, bool RBC = false>
__global__ __launch_bounds__(LPW *(L / E)) void k_ns_p3(V2<T> *w6, long nlines, int KZC,
                                                         const V2<T> *__restrict__ twg, float *part) {
    using C = V2<T>;
    __shared__ C lds[LPW * lds_line_len<L>()];
    __shared__ C tw[2 * L];
    load_twiddles<T>(tw, twg, 2 * L, threadIdx.x, LPW * (L / E));
    __syncthreads();
    // backwards over the lines: P2 ends at the last x planes and P4 starts at the first
    ns_p3_tile<T, L, E, LPW, RBC>(w6, nlines, KZC, sweep_tile(blockIdx.x, gridDim.x, 1), lds, tw, nullptr, part);
}

// ---- P5: X-forward with projection and the Runge-Kutta stage combine --------------------------------
struct P5Args {
    const void *c3;    // 3 fields after P4 (transit layout)
    const void *add3;  // optional extra term added before masking/projection (spectral, scaled), or null
    void *u;           // state (read; written by RK2_S2 / RK4_S4)
    void *aux;         // RK accumulator (transit layout): every term of the new state but the last stage's
    void *ust;         // stage input written by the first stages (transit layout)
    void *out;         // NS_RHS output
    const NsState *st;
    double nu;
    int mode;
};

// FUSE: the stage input (ust, or the new state) the combine forms is kept in registers and
// transformed on as the next right-hand side's P1 (the same columns, tile by tile) into the
// six transit fields at w6o, instead of going through the stage buffer: ust is neither
// written nor read back.  Not for NS_RHS.
template <typename T, int L, int E, int W, bool FUSE = false>
__device__ __forceinline__ void ns_p5_tile(const V2<T> *c3, const V2<T> *__restrict__ add3, V2<T> *u,
                                           V2<T> *aux, V2<T> *ust, V2<T> *out, const NsState *__restrict__ st,
                                           double nu, int mode, int K, int KZC, long tile, V2<T> *lds,
                                           const V2<T> *tw, V2<T> *w6o = nullptr) {
    using C = V2<T>;
    constexpr int N = L;
    constexpr int NZH = N / 2 + 1;
    constexpr int TPL = L / E;
    constexpr int ES = W + 1;
    constexpr long FS = (long)N * N * NZH;
    constexpr long RS = (long)N * NZH;
    const int tid = threadIdx.x;
    const int col = tid % W;
    const int jt = tid / W;
    // columns: the kept ky rows times the KZP transit columns (the padding columns, kz > K,
    // are masked modes: N = 0 there, so the stage buffers' rows are written whole)
    constexpr int KZP = ns_kzp<N>();
    constexpr long FSc = (long)N * N * KZP;
    constexpr long RSc = (long)N * KZP;
    const long ncols = (long)(2 * K + 1) * KZP;
    const long cc = tile * W + col;
    const bool valid = cc < ncols;
    int ky = 0, kz = 0;
    long row = 0;
    if (valid) {
        const long kyi = cc / KZP;
        kz = (int)(cc - kyi * KZP);
        row = kyi <= K ? kyi : kyi + N - 2 * K - 1;
        ky = wave_k((int)row, N);
    }
    const bool kz_kept = kz <= K;
    // point i of field f at element f FS + i TPL RS (uniform) + lo / sizeof(C) (per lane) in
    // the state-layout fields (u, add3, out); at f FSc + i TPL RSc + loc / sizeof(C) in the
    // transit-layout fields (c3, aux, ust)
    const unsigned lo = (unsigned)((row * NZH + kz + (long)jt * RS) * (long)sizeof(C));
    const unsigned loc = (unsigned)((row * KZP + kz + (long)jt * RSc) * (long)sizeof(C));
    // Unguarded loads: a lane past the last column addresses column 0 (row = kz = 0 above),
    // transforms it and stores nothing.  Without a select on the loaded values the first
    // transform waits for its own field's loads only, not for all three fields'.
    C cf[3][E];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
#pragma unroll
        for (int i = 0; i < E; ++i) cf[f][i] = *at_bytes(c3 + f * FSc + (long)(i * TPL) * RSc, loc);
    }
    // unrolled over the fields: a run-time field index into cf would put it in scratch
#pragma unroll
    for (int f = 0; f < 3; ++f) line_fft<T, L, E, ES>(cf[f], lds + col, jt, tw);
    if (valid) {
        const T scale = (T)(1.0 / ((double)N * N * N));
        const double h = st->h;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int r = jt + i * TPL;
            if (!row_kept(r, L, K)) {
                if constexpr (FUSE) {
#pragma unroll
                    for (int f = 0; f < 3; ++f) cf[f][i] = mk<T>(0, 0);
                }
                continue;
            }
            const int kx = wave_k(r, N);
            auto at = [&](auto *b, int f) { return at_bytes(b + f * FS + (long)(i * TPL) * RS, lo); };
            auto atc = [&](auto *b, int f) { return at_bytes(b + f * FSc + (long)(i * TPL) * RSc, loc); };
            C n0 = cscale(cf[0][i], scale), n1 = cscale(cf[1][i], scale), n2 = cscale(cf[2][i], scale);
            if (add3 && kz_kept) {
                n0 = cadd(n0, *at(add3, 0));
                n1 = cadd(n1, *at(add3, 1));
                n2 = cadd(n2, *at(add3, 2));
            }
            const T k2 = (T)(kx * kx + ky * ky + kz * kz);
            if (k2 > 0 && kz_kept) {
                const T ik2 = (T)1 / k2;
                const C kd = cadd(cadd(cscale(n0, (T)kx), cscale(n1, (T)ky)), cscale(n2, (T)kz));
                n0 = csub(n0, cscale(kd, (T)kx * ik2));
                n1 = csub(n1, cscale(kd, (T)ky * ik2));
                n2 = csub(n2, cscale(kd, (T)kz * ik2));
            } else {
                n0 = n1 = n2 = mk<T>(0, 0);
            }
            const C nn[3] = {n0, n1, n2};
            if (mode == NS_RHS) {
#pragma unroll
                for (int f = 0; f < 3; ++f) *at(out, f) = nn[f];
                continue;
            }
            const double a = nu * (double)k2 * h;
            T e1, e2;
            if constexpr (sizeof(T) == 4) {
                // FP32: one single-precision exponential (relative error ~1e-7), E = E2^2
                e2 = expf((float)(-0.5 * a));
                e1 = e2 * e2;
            } else {
                e1 = exp(-a);
                e2 = exp(-0.5 * a);
            }
            const T th = (T)h;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const C n = nn[f];
                C next;  // the next right-hand side's input
                switch (mode) {
                case RK2_S1: {
                    const C uu = *at(u, f);
                    *atc(aux, f) = cscale(cadd(uu, cscale(n, (T)0.5 * th)), e1);
                    next = cscale(cadd(uu, cscale(n, th)), e1);
                    break;
                }
                case RK2_S2:
                    next = cadd(*atc(aux, f), cscale(n, (T)0.5 * th));
                    *at(u, f) = next;
                    break;
                case RK4_S1: {
                    const C uu = *at(u, f);
                    *atc(aux, f) = cscale(cadd(uu, cscale(n, th / (T)6)), e1);
                    next = cscale(cadd(uu, cscale(n, (T)0.5 * th)), e2);
                    break;
                }
                case RK4_S2:
                    *atc(aux, f) = cadd(*atc(aux, f), cscale(n, th / (T)3 * e2));
                    next = cadd(cscale(*at(u, f), e2), cscale(n, (T)0.5 * th));
                    break;
                case RK4_S3:
                    *atc(aux, f) = cadd(*atc(aux, f), cscale(n, th / (T)3 * e2));
                    next = cadd(cscale(*at(u, f), e1), cscale(n, th * e2));
                    break;
                default:  // RK4_S4
                    next = cadd(*atc(aux, f), cscale(n, th / (T)6));
                    *at(u, f) = next;
                    break;
                }
                if constexpr (FUSE) cf[f][i] = next;
                else if (mode != RK2_S2 && mode != RK4_S4) *atc(ust, f) = next;
            }
        }
    }
    if constexpr (FUSE) {
        // the LDS is free again: the last exchange of the forward transforms ended with a
        // barrier after every thread's reads
        const P1Col c = ns_p1_col<T, L, E, W>(tile, K, 1);
        const C none[1] = {mk<T>(0, 0)};
        ns_p1_body<T, L, E, W, false>(cf[0], cf[1], cf[2], none, w6o, c, lds, tw, (T)1);
    }
}

template <typename T, int L, int E, int W>
__global__ __launch_bounds__(W *(L / E)) void k_ns_p5(const V2<T> *__restrict__ c3, const V2<T> *__restrict__ add3,
                                                       V2<T> *u, V2<T> *aux, V2<T> *ust, V2<T> *out,
                                                       const NsState *__restrict__ st, double nu, int mode, int K,
                                                       int KZC, const V2<T> *__restrict__ twg) {
    using C = V2<T>;
    __shared__ C lds[L * (W + 1)];
    __shared__ C tw[L];
    load_twiddles<T>(tw, twg, L, threadIdx.x, W * (L / E));
    __syncthreads();
    ns_p5_tile<T, L, E, W>(c3, add3, u, aux, ust, out, st, nu, mode, K, KZC, xcd_tile(blockIdx.x, gridDim.x), lds,
                           tw);
}

// P5 fused with the next right-hand side's P1: reads the products from w6 (fields 0..2)
// and writes the next six transit fields over them (each workgroup reads its columns
// whole before it writes them).
template <typename T, int L, int E, int W>
__global__ __launch_bounds__(W *(L / E)) void k_ns_p51(V2<T> *w6, const V2<T> *__restrict__ add3, V2<T> *u,
                                                        V2<T> *aux, const NsState *__restrict__ st, double nu,
                                                        int mode, int K, int KZC, const V2<T> *__restrict__ twg) {
    using C = V2<T>;
    __shared__ C lds[L * (W + 1)];
    __shared__ C tw[L];
    load_twiddles<T>(tw, twg, L, threadIdx.x, W * (L / E));
    __syncthreads();
    ns_p5_tile<T, L, E, W, true>(w6, add3, u, aux, nullptr, nullptr, st, nu, mode, K, KZC,
                                 xcd_tile(blockIdx.x, gridDim.x), lds, tw, w6);
}

// ---- P5 of the Boussinesq (RBC) right-hand side ----------------------------------------------------
// Fields in: c = u x omega (0..2) and q = u theta (3..5) after P4; stage input uin = (u, theta).
//   N_u = P M [c^ + theta^ z],   N_theta = M [-i a k . q^ + u_z^]
// then the IF-RK2 combine over 4 fields with exp(-nu_a |k|^2 h) for u and exp(-kappa_a |k|^2 h)
// for theta (nu_a, kappa_a already include a^2).  Modes: NS_RHS, RK2_S1, RK2_S2.
template <typename T, int L, int E, int W>
__device__ __forceinline__ void rbc_p5_tile(const V2<T> *__restrict__ c6, const V2<T> *__restrict__ uin, V2<T> *u,
                                            V2<T> *aux, V2<T> *ust, V2<T> *out, const NsState *__restrict__ st,
                                            double nu_a, double kap_a, T ka, int mode, int K, int KZC, long tile,
                                            V2<T> *lds, const V2<T> *tw) {
    using C = V2<T>;
    constexpr int N = L;
    constexpr int NZH = N / 2 + 1;
    constexpr int TPL = L / E;
    constexpr int ES = W + 1;
    constexpr long FS = (long)N * N * NZH;
    constexpr long RS = (long)N * NZH;
    const int tid = threadIdx.x;
    const int col = tid % W;
    const int jt = tid / W;
    const long ncols = (long)(2 * K + 1) * KZC;
    const long cc = tile * W + col;
    const bool valid = cc < ncols;
    int ky = 0, kz = 0;
    const long j = valid ? kept_col(cc, N, K, KZC, NZH, &ky, &kz) : 0;
    // point i of field f at element f FS + i TPL RS (uniform) + lo / sizeof(C) (per lane);
    // in the transit fields c6 at f FSc + i TPL RSc + loc / sizeof(C)
    constexpr int KZP = ns_kzp<N>();
    constexpr long FSc = (long)N * N * KZP;
    constexpr long RSc = (long)N * KZP;
    const unsigned lo = (unsigned)((j + (long)jt * RS) * (long)sizeof(C));
    const unsigned loc = (unsigned)(((j / NZH) * KZP + kz + (long)jt * RSc) * (long)sizeof(C));
    C cf[3][E], nt[E];
#pragma unroll
    for (int i = 0; i < E; ++i) nt[i] = mk<T>(0, 0);
#pragma unroll 1
    for (int f = 0; f < 6; ++f) {
        C v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = valid ? *at_bytes(c6 + f * FSc + (long)(i * TPL) * RSc, loc) : mk<T>(0, 0);
        line_fft<T, L, E, ES>(v, lds + col, jt, tw);
        if (f < 3) {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                if (f == 0) cf[0][i] = v[i];
                else if (f == 1) cf[1][i] = v[i];
                else cf[2][i] = v[i];
            }
        } else {
            // -i a k_f q^_f accumulated: (-i) (a k) (x + i y) = a k (y - i x)
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const T kf = ka * (T)(f == 3 ? deriv_k(jt + i * TPL, N) : (f == 4 ? ky : ((2 * kz == N) ? 0 : kz)));
                nt[i].x += kf * v[i].y;
                nt[i].y -= kf * v[i].x;
            }
        }
    }
    if (valid) {
        const T scale = (T)(1.0 / ((double)N * N * N));
        const double h = st->h;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int r = jt + i * TPL;
            if (!row_kept(r, L, K)) continue;
            const int kx = wave_k(r, N);
            auto at = [&](auto *b, int f) { return at_bytes(b + f * FS + (long)(i * TPL) * RS, lo); };
            const C th = *at(uin, 3);
            C n0 = cscale(cf[0][i], scale), n1 = cscale(cf[1][i], scale), n2 = cadd(cscale(cf[2][i], scale), th);
            const T k2 = (T)(kx * kx + ky * ky + kz * kz);
            if (k2 > 0) {
                const T ik2 = (T)1 / k2;
                const C kd = cadd(cadd(cscale(n0, (T)kx), cscale(n1, (T)ky)), cscale(n2, (T)kz));
                n0 = csub(n0, cscale(kd, (T)kx * ik2));
                n1 = csub(n1, cscale(kd, (T)ky * ik2));
                n2 = csub(n2, cscale(kd, (T)kz * ik2));
            } else {
                n0 = n1 = n2 = mk<T>(0, 0);
            }
            const C n3 = cadd(cscale(nt[i], scale), *at(uin, 2));
            const C nn[4] = {n0, n1, n2, n3};
            if (mode == NS_RHS) {
#pragma unroll
                for (int f = 0; f < 4; ++f) *at(out, f) = nn[f];
                continue;
            }
            T eu, et;
            if constexpr (sizeof(T) == 4) {
                eu = expf((float)(-nu_a * (double)k2 * h));
                et = expf((float)(-kap_a * (double)k2 * h));
            } else {
                eu = exp(-nu_a * (double)k2 * h);
                et = exp(-kap_a * (double)k2 * h);
            }
            const T th_ = (T)h;
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const T e = f < 3 ? eu : et;
                const C uu = *at(u, f);
                if (mode == RK2_S1) {
                    *at(aux, f) = nn[f];
                    *at(ust, f) = cscale(cadd(uu, cscale(nn[f], th_)), e);
                } else {
                    *at(u, f) = cadd(cscale(uu, e), cscale(cadd(cscale(*at(aux, f), e), nn[f]), (T)0.5 * th_));
                }
            }
        }
    }
}

template <typename T, int L, int E, int W>
__global__ __launch_bounds__(W *(L / E)) void k_rbc_p5(const V2<T> *__restrict__ c6, const V2<T> *__restrict__ uin,
                                                        V2<T> *u, V2<T> *aux, V2<T> *ust, V2<T> *out,
                                                        const NsState *__restrict__ st, double nu_a, double kap_a,
                                                        T ka, int mode, int K, int KZC, const V2<T> *__restrict__ twg) {
    using C = V2<T>;
    __shared__ C lds[L * (W + 1)];
    __shared__ C tw[L];
    load_twiddles<T>(tw, twg, L, threadIdx.x, W * (L / E));
    __syncthreads();
    rbc_p5_tile<T, L, E, W>(c6, uin, u, aux, ust, out, st, nu_a, kap_a, ka, mode, K, KZC,
                            xcd_tile(blockIdx.x, gridDim.x), lds, tw);
}

// ---- small kernels --------------------------------------------------------------------------------
// CFL step size from the maxima P3 recorded, one per workgroup (or the fixed step);
// advances t.  One workgroup of up to 1024 threads.
static __global__ void k_ns_set_h(NsState *st, const float *part, int nparts) {
    __shared__ float wmax[16];
    float m = 0.f;
    if (part)
        for (int i = threadIdx.x; i < nparts; i += blockDim.x) m = fmaxf(m, part[i]);
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, wmax[w]);
        m = fmaxf(m, wmax[0]);
        double h = st->hfix;
        if (st->cfl_dx > 0) {
            const double um = (double)m;
            h = um > 0 ? st->cfl_dx / um : st->hfix;
        }
        st->h = h;
        st->t += h;
    }
}

template <typename C> __global__ void k_zero(C *p, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        C z;
        z.x = 0;
        z.y = 0;
        p[i] = z;
    }
}

// ---- instantiation helpers --------------------------------------------------------------------------
// Tile shapes of P1 / P5 / the fused P5+P1: E = default_E(N) points per thread and W
// columns (16 for FP32, 8 for FP64, fewer if the workgroup would exceed its thread cap).
// They hold three fields per thread; a 1024-thread workgroup (4 waves per SIMD) leaves 128
// registers per thread, enough at E <= 8 in FP32 (about 112), so the cap is 1024 threads
// there and 512 otherwise.  The convection passes hold a fourth field and still fit
// (ns_rbc_W: 123 and 128 registers for its P1 and P5 at 512^3 in FP32; with 8-column tiles
// each 128-byte line was fetched in two halves).  P3 uses E = default_E(N/2) and 256 threads.
template <typename T> constexpr int ns_x_E(int N) { return default_E(N); }
template <typename T> constexpr int ns_x_cap(int N) { return (sizeof(T) == 4 && ns_x_E<T>(N) <= 8) ? 1024 : 512; }
template <typename T> constexpr int ns_x_W(int N) {
    int E = ns_x_E<T>(N);
    int W = sizeof(T) == 8 ? 8 : 16;
    while (W > 1 && W * (N / E) > ns_x_cap<T>(N)) W /= 2;
    while (W * (N / E) < 64) W *= 2;
    return W;
}
template <typename T> constexpr int ns_rbc_W(int N) { return ns_x_W<T>(N); }
constexpr int ns_z_LPW(int N) {
    int L = N / 2, E = default_E(L), TPL = L / E;
    return TPL >= 256 ? 1 : 256 / TPL;
}

// Tile-shape variants of P1, P3 and P5 (the autotuner picks one per grid size and dtype;
// variant 0 is the default above).  P1 / P5: a = W columns; P3: a = LPW lines.
// P1: cin = 1 when u is a stage buffer in the transit layout
using NsP1Fn = void (*)(const void *u, void *w6, int K, int cin, const void *tw, hipStream_t s);
using NsP3Fn = void (*)(void *w6, long nlines, int KZC, const void *tw, float *part, hipStream_t s);
using NsP5Fn = void (*)(const P5Args &a, int K, int KZC, const void *tw, hipStream_t s);
template <typename F> struct NsVar {
    int a, E, v;  // v: variant of one shape (0: the only one compiled)
    F fn;
};
constexpr int NS_MAXVAR = 6;

struct NsKernels {
    int N;
    tk_dtype dt;
    int np1 = 0, np3 = 0, np5 = 0, np51 = 0;
    NsVar<NsP1Fn> p1v[NS_MAXVAR];
    NsVar<NsP3Fn> p3v[NS_MAXVAR];
    NsVar<NsP5Fn> p5v[NS_MAXVAR];
    NsVar<NsP5Fn> p51v[NS_MAXVAR];  // P5 fused with the next P1 (a.c3 = the workspace, rewritten)
    // Boussinesq variants (default shapes): P1 with temperature (4 -> 7 fields), P3 (7 -> 6),
    // P5 (6 + state of 4)
    void (*p1r)(const void *u, void *w7, int K, int KZC, const void *tw, double ka, hipStream_t s);
    void (*p3r)(void *w7, long nlines, int KZC, const void *tw, float *part, hipStream_t s);
    void (*p5r)(const void *c6, const void *uin, void *u, void *aux, void *ust, void *out, const NsState *st,
                double nu_a, double kap_a, double ka, int mode, int K, int KZC, const void *tw, hipStream_t s);
};
const std::vector<NsKernels> &ns_kernels();

template <typename T, int N, int E, int W>
void launch_ns_p1(const void *u, void *w6, int K, int cin, const void *tw, hipStream_t s) {
    const long ncols = (long)(2 * K + 1) * ns_kzp<N>();
    hipLaunchKernelGGL((k_ns_p1<T, N, E, W>), dim3(cdiv(ncols, W)), dim3(W * (N / E)), 0, s, (const V2<T> *)u,
                       (V2<T> *)w6, K, cin, (const V2<T> *)tw, (T)1);
}
template <typename T, int L2, int E2, int LPW>
void launch_ns_p3(void *w6, long nlines, int KZC, const void *tw, float *part, hipStream_t s) {
    hipLaunchKernelGGL((k_ns_p3<T, L2, E2, LPW>), dim3(cdiv(nlines, LPW)), dim3(LPW * (L2 / E2)), 0, s,
                       (V2<T> *)w6, nlines, KZC, (const V2<T> *)tw, part);
}
template <typename T, int N, int E, int W>
void launch_ns_p5(const P5Args &a, int K, int KZC, const void *tw, hipStream_t s) {
    const long ncols = (long)(2 * K + 1) * ns_kzp<N>();
    hipLaunchKernelGGL((k_ns_p5<T, N, E, W>), dim3(cdiv(ncols, W)), dim3(W * (N / E)), 0, s, (const V2<T> *)a.c3,
                       (const V2<T> *)a.add3, (V2<T> *)a.u, (V2<T> *)a.aux, (V2<T> *)a.ust, (V2<T> *)a.out, a.st,
                       a.nu, a.mode, K, KZC, (const V2<T> *)tw);
}
template <typename T, int N, int E, int W>
void launch_ns_p51(const P5Args &a, int K, int KZC, const void *tw, hipStream_t s) {
    const long ncols = (long)(2 * K + 1) * ns_kzp<N>();
    hipLaunchKernelGGL((k_ns_p51<T, N, E, W>), dim3(cdiv(ncols, W)), dim3(W * (N / E)), 0, s, (V2<T> *)a.c3,
                       (const V2<T> *)a.add3, (V2<T> *)a.u, (V2<T> *)a.aux, a.st, a.nu, a.mode, K, KZC,
                       (const V2<T> *)tw);
}

// Column-pass variant (E, W) of P1 / P5 / P5+P1 (FP32, N >= 128): kept when it differs
// from the default, W is whole, the workgroup has 64 threads up to the cap of ns_x_cap
// and the LDS tile fits; the 512- and 1024-thread tiles of E = default_E(N) are offered.
// (Persistent P1 workgroups loading the next tile ahead measured 1.5x slower at 512^3.)
template <typename T, int N, int E, int W> constexpr bool ns_x_var_ok() {
    return sizeof(T) == 4 && N >= 128 && E <= N && N % E == 0 && rplan_ok(N, E) && W >= 1 &&
           W * (N / E) >= 64 && W * (N / E) <= ns_x_cap<T>(N) && (long)(N * (W + 1) + N) * 2 * (long)sizeof(T) <= 163840 &&
           !(E == ns_x_E<T>(N) && W == ns_x_W<T>(N));
}
template <typename T, int N, int E, int W> void add_ns_p1_var(NsKernels &k) {
    if constexpr (ns_x_var_ok<T, N, E, W>()) k.p1v[k.np1++] = {W, E, 0, &launch_ns_p1<T, N, E, W>};
}
template <typename T, int N, int E, int W> void add_ns_p5_var(NsKernels &k) {
    // (a variant loading the stage combine's operands with the input, before the
    // transforms, measured 10% slower at 512^3: the registers it takes cost occupancy)
    if constexpr (ns_x_var_ok<T, N, E, W>()) {
        k.p5v[k.np5++] = {W, E, 0, &launch_ns_p5<T, N, E, W>};
        k.p51v[k.np51++] = {W, E, 0, &launch_ns_p51<T, N, E, W>};
    }
}
// Line-pass variant E2 of P3 (FP32, N >= 128; L2 = N / 2 points per complex line, 256
// threads): kept when it differs from the default and a line stays inside one wavefront.
template <typename T, int N, int E2> constexpr bool ns_z_var_ok() {
    constexpr int L2 = N / 2;
    return sizeof(T) == 4 && N >= 128 && E2 >= 2 && E2 <= L2 && L2 % E2 == 0 && rplan_ok(L2, E2) &&
           L2 / E2 <= 64 && E2 != default_E(L2);
}
template <typename T, int N, int E2> void add_ns_z_var(NsKernels &k) {
    if constexpr (ns_z_var_ok<T, N, E2>()) {
        constexpr int L2 = N / 2;
        constexpr int LPW = 256 / (L2 / E2);
        k.p3v[k.np3++] = {LPW, E2, 0, &launch_ns_p3<T, L2, E2, LPW>};
    }
}

template <typename T, int N> NsKernels make_ns_kernels() {
    constexpr int E = ns_x_E<T>(N);
    constexpr int W = ns_x_W<T>(N);
    constexpr int L2 = N / 2;
    constexpr int E2 = default_E(L2);
    constexpr int LPW = ns_z_LPW(N);
    constexpr int Ed = default_E(N);
    NsKernels k;
    k.N = N;
    k.dt = sizeof(T) == 4 ? TK_F32 : TK_F64;
    k.p1v[k.np1++] = {W, E, 0, &launch_ns_p1<T, N, E, W>};
    k.p5v[k.np5++] = {W, E, 0, &launch_ns_p5<T, N, E, W>};
    k.p51v[k.np51++] = {W, E, 0, &launch_ns_p51<T, N, E, W>};
    k.p3v[k.np3++] = {LPW, E2, 0, &launch_ns_p3<T, L2, E2, LPW>};
    add_ns_p1_var<T, N, Ed, 512 * Ed / N>(k);
    add_ns_p1_var<T, N, Ed, 1024 * Ed / N>(k);
    add_ns_p5_var<T, N, Ed, 512 * Ed / N>(k);
    add_ns_p5_var<T, N, Ed, 1024 * Ed / N>(k);
    add_ns_z_var<T, N, default_E(L2) / 2>(k);
    constexpr int Wr = ns_rbc_W<T>(N);
    k.p1r = [](const void *u, void *w7, int K, int KZC, const void *tw, double ka, hipStream_t s) {
        // the convection solver keeps its stage buffers in the state layout
        const long ncols = (long)(2 * K + 1) * ns_kzp<N>();
        hipLaunchKernelGGL((k_ns_p1<T, N, E, Wr, true>), dim3(cdiv(ncols, Wr)), dim3(Wr * (N / E)), 0, s,
                           (const V2<T> *)u, (V2<T> *)w7, K, 0, (const V2<T> *)tw, (T)ka);
    };
    k.p3r = [](void *w7, long nlines, int KZC, const void *tw, float *part, hipStream_t s) {
        hipLaunchKernelGGL((k_ns_p3<T, L2, E2, LPW, true>), dim3(cdiv(nlines, LPW)), dim3(LPW * (L2 / E2)), 0, s,
                           (V2<T> *)w7, nlines, KZC, (const V2<T> *)tw, part);
    };
    k.p5r = [](const void *c6, const void *uin, void *u, void *aux, void *ust, void *out, const NsState *st,
               double nu_a, double kap_a, double ka, int mode, int K, int KZC, const void *tw, hipStream_t s) {
        const long ncols = (long)(2 * K + 1) * KZC;
        hipLaunchKernelGGL((k_rbc_p5<T, N, E, Wr>), dim3(cdiv(ncols, Wr)), dim3(Wr * (N / E)), 0, s,
                           (const V2<T> *)c6, (const V2<T> *)uin, (V2<T> *)u, (V2<T> *)aux, (V2<T> *)ust,
                           (V2<T> *)out, st, nu_a, kap_a, (T)ka, mode, K, KZC, (const V2<T> *)tw);
    };
    return k;
}

}  // namespace tk
