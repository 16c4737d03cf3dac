// Device building blocks of the 1D transforms: radix-2/3/4/8 butterflies and Stockham
// autosort stages with the line held in registers between LDS exchanges.
//
// A line of L complex points is transformed by TPL = L / E threads; thread jt owns the
// E points x[jt + i TPL], i < E.  Stage s has radix R and span NS (product of the
// radices before it): butterfly j takes x[j + m L/R], m < R, multiplies leg m by
// W_{NS R}^{(j mod NS) m}, applies the R-point DFT and sends leg m to position
// (j - j mod NS) R + j mod NS + m NS.  With the thread's butterflies j = jt + b TPL,
// b < E/R, every stage reads exactly the thread's own points x[jt + i TPL], and the
// last stage (NS = L/R) writes exactly them: so loads from and stores to global memory
// go straight to registers and only the exchanges between stages pass through LDS.
// After the last stage the line is in natural order (Stockham autosort).
#pragma once

#include "common.hpp"

namespace tk {

// ---- radix plan -----------------------------------------------------------------------------
struct RPlan {
    int n;
    int r[16];
};

// Factor L into radices that all divide E: a single 3 first (L = 3 * 2^a), then 8s
// while at least 8 remains (never leaving a lone 2 after 16), then 4, then 2.
constexpr RPlan make_rplan(int L, int E) {
    RPlan p{};
    p.n = 0;
    int rem = L;
    if (rem % 3 == 0) {
        p.r[p.n++] = 3;
        rem /= 3;
    }
    while (rem > 1) {
        int r = 2;
        if (rem % 8 == 0 && E % 8 == 0 && rem != 16) r = 8;
        else if (rem % 4 == 0 && E % 4 == 0) r = 4;
        p.r[p.n++] = r;
        rem /= r;
    }
    return p;
}

constexpr int rplan_span(RPlan p, int s) {
    int ns = 1;
    for (int i = 0; i < s; ++i) ns *= p.r[i];
    return ns;
}

// Elements per thread: 8 for powers of two >= 8, 12 for 3 * 2^a >= 12, else the line.
constexpr int default_E(int L) {
    if (L % 3 == 0) return L >= 12 ? 12 : L;
    return L >= 8 ? 8 : L;
}

constexpr bool rplan_ok(int L, int E) {
    if (E <= 0 || L % E != 0) return false;
    RPlan p = make_rplan(L, E);
    int prod = 1;
    for (int i = 0; i < p.n; ++i) {
        if (E % p.r[i] != 0) return false;
        prod *= p.r[i];
    }
    return prod == L;
}

// ---- butterflies (forward sign, exp(-2 pi i / R)) --------------------------------------------
template <int R, typename C> struct Dft;

template <typename C> struct Dft<2, C> {
    static __device__ __forceinline__ void run(C &a, C &b) {
        C t = a;
        a = cadd(t, b);
        b = csub(t, b);
    }
};

template <typename C> struct Dft<3, C> {
    static __device__ __forceinline__ void run(C &x0, C &x1, C &x2) {
        using T = decltype(x0.x);
        const T s3 = (T)0.86602540378443864676372317075294;  // sin(2 pi / 3)
        C p = cadd(x1, x2);
        C m = csub(x1, x2);
        C t = x0;
        t.x -= (T)0.5 * p.x;
        t.y -= (T)0.5 * p.y;
        x0 = cadd(x0, p);
        C q;  // -i s3 m
        q.x = s3 * m.y;
        q.y = -s3 * m.x;
        x1 = cadd(t, q);
        x2 = csub(t, q);
    }
};

template <typename C> struct Dft<4, C> {
    static __device__ __forceinline__ void run(C &x0, C &x1, C &x2, C &x3) {
        C t0 = cadd(x0, x2);
        C t1 = csub(x0, x2);
        C t2 = cadd(x1, x3);
        C t3 = cmul_mi(csub(x1, x3));
        x0 = cadd(t0, t2);
        x2 = csub(t0, t2);
        x1 = cadd(t1, t3);
        x3 = csub(t1, t3);
    }
};

template <typename C> struct Dft<8, C> {
    static __device__ __forceinline__ void run(C &x0, C &x1, C &x2, C &x3, C &x4, C &x5, C &x6, C &x7) {
        using T = decltype(x0.x);
        const T r2 = (T)0.70710678118654752440084436210485;
        Dft<4, C>::run(x0, x2, x4, x6);  // even legs -> E0..E3 in x0, x2, x4, x6
        Dft<4, C>::run(x1, x3, x5, x7);  // odd legs  -> O0..O3 in x1, x3, x5, x7
        C o1, o3;
        o1.x = r2 * (x3.x + x3.y);  // O1 W8
        o1.y = r2 * (x3.y - x3.x);
        C o2 = cmul_mi(x5);         // O2 W8^2
        o3.x = r2 * (x7.y - x7.x);  // O3 W8^3
        o3.y = -r2 * (x7.x + x7.y);
        C e0 = x0, e1 = x2, e2 = x4, e3 = x6, o0 = x1;
        x0 = cadd(e0, o0);
        x4 = csub(e0, o0);
        x1 = cadd(e1, o1);
        x5 = csub(e1, o1);
        x2 = cadd(e2, o2);
        x6 = csub(e2, o2);
        x3 = cadd(e3, o3);
        x7 = csub(e3, o3);
    }
};

// Butterfly b of a stage: legs v[b + m NB], m < R.
template <int R, int NB, typename C> __device__ __forceinline__ void dft_legs(C *v, int b) {
    if constexpr (R == 2) Dft<2, C>::run(v[b], v[b + NB]);
    else if constexpr (R == 3) Dft<3, C>::run(v[b], v[b + NB], v[b + 2 * NB]);
    else if constexpr (R == 4) Dft<4, C>::run(v[b], v[b + NB], v[b + 2 * NB], v[b + 3 * NB]);
    else Dft<8, C>::run(v[b], v[b + NB], v[b + 2 * NB], v[b + 3 * NB], v[b + 4 * NB], v[b + 5 * NB],
                        v[b + 6 * NB], v[b + 7 * NB]);
}

// ---- LDS addressing ---------------------------------------------------------------------------
// Contiguous lines (ES == 1): one padding slot every 32 complex values, so that the
// stride-R scatter of a stage spreads over the banks.
template <int ES> __device__ __forceinline__ int lds_at(int e) {
    if constexpr (ES == 1) return e + (e >> 5);
    else return e * ES;
}
template <int L> constexpr int lds_line_len() { return L + (L >> 5) + 1; }

// ---- synchronisation of the exchanges ------------------------------------------------------------
// A contiguous line (ES == 1) is handled by TPL consecutive lanes of one wavefront (TPL
// divides 64) and owns its LDS row, so its exchanges only have to be ordered within the
// wavefront: the LDS executes a wavefront's instructions in order, and waiting for the
// wavefront's own LDS operations (lgkmcnt 0) behind a compiler memory barrier is enough.
// Waves of a workgroup then run their lines independently instead of meeting at a
// workgroup barrier twice per stage.  Column tiles spread a line over several waves and
// use the workgroup barrier.
template <int ES> __device__ __forceinline__ void exchange_sync() {
    if constexpr (ES == 1) asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    else __syncthreads();
}

// Exchange between stage S and S + 1: leg m of butterfly j goes to position
// (j - j mod NS) R + j mod NS + m NS, and the thread reads back its own points.
template <typename T, int L, int E, int ES, int S, bool SPLIT>
__device__ __forceinline__ void stage_exchange(V2<T> (&v)[E], V2<T> *d, int jt) {
    constexpr RPlan P = make_rplan(L, E);
    constexpr int R = P.r[S];
    constexpr int NS = rplan_span(P, S);
    constexpr int NB = E / R;
    constexpr int TPL = L / E;
    if constexpr (SPLIT) {
        T *ds = reinterpret_cast<T *>(d);
#pragma unroll
        for (int part = 0; part < 2; ++part) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int j = jt + b * TPL;
                const int k = j % NS;
                const int base = (j - k) * R + k;
#pragma unroll
                for (int m = 0; m < R; ++m) ds[lds_at<ES>(base + m * NS)] = part ? v[b + m * NB].y : v[b + m * NB].x;
            }
            exchange_sync<ES>();
#pragma unroll
            for (int i = 0; i < E; ++i) {
                if (part) v[i].y = ds[lds_at<ES>(jt + i * TPL)];
                else v[i].x = ds[lds_at<ES>(jt + i * TPL)];
            }
            exchange_sync<ES>();
        }
    } else {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = jt + b * TPL;
            const int k = j % NS;
            const int base = (j - k) * R + k;
#pragma unroll
            for (int m = 0; m < R; ++m) d[lds_at<ES>(base + m * NS)] = v[b + m * NB];
        }
        exchange_sync<ES>();
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = d[lds_at<ES>(jt + i * TPL)];
        exchange_sync<ES>();
    }
}

// ---- the transform -------------------------------------------------------------------------------
// v[i] = x[jt + i TPL] on entry, X[jt + i TPL] on exit (forward DFT, unscaled).
// d: this line's LDS (element e at d[lds_at<ES>(e)]), tw: LDS table with W_L^j at
// tw[j * TS].
// Column tiles (ES > 1): every thread of the workgroup must call it (it contains
// barriers); on exit the LDS may be reused only after a barrier.  Contiguous lines
// (ES == 1): the lanes of a line call it together and may reuse their LDS row at once.
// TWP: twiddle powers by multiplication (for LDS-bound callers; HBM-bound passes keep the
// table reads, which cost fewer registers).
// SPLIT: exchange the real parts, then the imaginary parts, through an LDS line of scalars
// (d is then a T pointer in disguise, element e at ((T *)d)[lds_at<ES>(e)]): half the LDS
// of a column tile, so more workgroups fit on a CU, for two more barriers per exchange.
// RS: the stage whose twiddles the caller holds in registers (wr[m - 1] for leg m; -1: none).
// Allowed only for a stage with one butterfly per thread (E == R there), whose twiddles
// depend on the lane alone: see stage_twiddles.
template <typename T, int L, int E, int ES, int TS = 1, int S = 0, bool TWP = false, bool SPLIT = false, int RS = -1>
__device__ __forceinline__ void line_fft(V2<T> (&v)[E], V2<T> *d, int jt, const V2<T> *tw,
                                         const V2<T> *wr = nullptr) {
    using C = V2<T>;
    constexpr RPlan P = make_rplan(L, E);
    constexpr int R = P.r[S];
    constexpr int NS = rplan_span(P, S);
    constexpr int NB = E / R;
    constexpr int TPL = L / E;
    static_assert(ES != 1 || (TPL <= 64 && 64 % TPL == 0), "a contiguous line must sit inside one wavefront");
    static_assert(S != RS || NB == 1, "register twiddles need one butterfly per thread at that stage");
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = jt + b * TPL;
        const int k = j % NS;
        if constexpr (NS > 1 && S == RS) {
#pragma unroll
            for (int m = 1; m < R; ++m) v[b + m * NB] = cmul(v[b + m * NB], wr[m - 1]);
        } else if constexpr (NS > 1) {
            if constexpr (TWP) {
                // leg m takes W^m, W = W_{NS R}^k: one table read, the powers by
                // multiplication (R - 2 complex products instead of R - 2 more LDS reads;
                // the error grows by about one rounding per power)
                const C w = tw[k * (L / (NS * R)) * TS];
                C wm = w;
#pragma unroll
                for (int m = 1; m < R; ++m) {
                    v[b + m * NB] = cmul(v[b + m * NB], wm);
                    if (m + 1 < R) wm = cmul(wm, w);
                }
            } else {
#pragma unroll
                for (int m = 1; m < R; ++m) v[b + m * NB] = cmul(v[b + m * NB], tw[k * m * (L / (NS * R)) * TS]);
            }
        }
        dft_legs<R, NB>(v, b);
    }
    if constexpr (S + 1 < P.n) {
        stage_exchange<T, L, E, ES, S, SPLIT>(v, d, jt);
        line_fft<T, L, E, ES, TS, S + 1, TWP, SPLIT, RS>(v, d, jt, tw, wr);
    }
}

// The first stage after stage 0 whose butterflies are one per thread (E == R), or -1: its
// twiddles W_{NS R}^{(jt mod NS) m} depend on the lane alone, so a caller that runs many
// transforms can hold them in registers.
template <int L, int E> constexpr int lane_twiddle_stage() {
    constexpr RPlan P = make_rplan(L, E);
    for (int s = 1; s < P.n; ++s)
        if (P.r[s] == E) return s;
    return -1;
}

// wr[m - 1] = W_{NS R}^{k m}, k = jt mod NS, for stage S (one table read, the powers by
// multiplication); tw is the W_{L TS}^j table the transforms use.
template <typename T, int L, int E, int TS, int S>
__device__ __forceinline__ void stage_twiddles(int jt, const V2<T> *tw, V2<T> (&wr)[E - 1]) {
    constexpr RPlan P = make_rplan(L, E);
    constexpr int R = P.r[S];
    constexpr int NS = rplan_span(P, S);
    static_assert(R == E, "one butterfly per thread");
    const V2<T> w = tw[(jt % NS) * (L / (NS * R)) * TS];
    wr[0] = w;
#pragma unroll
    for (int m = 1; m < R - 1; ++m) wr[m] = cmul(wr[m - 1], w);
}

// ---- mirror exchange ---------------------------------------------------------------------------------
// The real-FFT split and merge need x[(L - k) mod L] next to x[k].  With thread jt of a
// line holding x[jt + i TPL], that value sits in thread (TPL - jt) mod TPL, register
// E - 1 - i (jt > 0), or in the thread itself, register (E - i) mod E (jt = 0).  A line's
// TPL threads are consecutive lanes of one wavefront (TPL divides 64), so a cross-lane
// shuffle fetches it without LDS or barriers.
template <typename T, int L, int E>
__device__ __forceinline__ void mirror(const V2<T> (&v)[E], V2<T> (&m)[E], int jt) {
    constexpr int TPL = L / E;
    static_assert(TPL <= 64 && (64 % TPL) == 0, "a line must sit inside one wavefront");
    const int lane = threadIdx.x & 63;
    const int src = lane - jt + ((TPL - jt) & (TPL - 1));
#pragma unroll
    for (int i = 0; i < E; ++i) {
        V2<T> p;
        if constexpr (TPL > 1) {
            p.x = __shfl(v[E - 1 - i].x, src, 64);
            p.y = __shfl(v[E - 1 - i].y, src, 64);
        } else {
            p = v[E - 1 - i];
        }
        m[i] = (jt != 0) ? p : v[(E - i) % E];
    }
}

// Cooperative copy of a twiddle table of n entries into LDS; the caller places a
// barrier before its first use.
template <typename T>
__device__ __forceinline__ void load_twiddles(V2<T> *dst, const V2<T> *__restrict__ src, int n, int tid, int nt) {
    for (int j = tid; j < n; j += nt) dst[j] = src[j];
}

}  // namespace tk
