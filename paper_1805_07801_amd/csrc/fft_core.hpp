// Device building blocks of the 1D transforms: radix-2/3/4/8 butterflies and Stockham
// autosort stages over a line that lives in LDS.
//
// A line of L complex points is transformed by TPL = L / E threads; each thread owns E
// points per stage (E / R butterflies of radix R).  Stage s has radix R and span NS (the
// product of the radices before it): butterfly j takes x[j + m L/R], m < R, multiplies
// leg m by W_{NS R}^{(j mod NS) m}, applies the R-point DFT and writes leg m to
// (j - j mod NS) R + j mod NS + m NS.  After the last stage the line is in natural
// order (Stockham autosort), so no bit reversal pass exists.
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
    static __device__ __forceinline__ void run(C *v) {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <typename C> struct Dft<3, C> {
    static __device__ __forceinline__ void run(C *v) {
        using T = decltype(v[0].x);
        const T s3 = (T)0.86602540378443864676372317075294;  // sin(2 pi / 3)
        C a = v[0];
        C p = cadd(v[1], v[2]);
        C m = csub(v[1], v[2]);
        C t = a;
        t.x -= (T)0.5 * p.x;
        t.y -= (T)0.5 * p.y;
        v[0] = cadd(a, p);
        // y1 = t - i s3 m ; y2 = t + i s3 m
        C q;
        q.x = s3 * m.y;
        q.y = -s3 * m.x;  // -i s3 m
        v[1] = cadd(t, q);
        v[2] = csub(t, q);
    }
};

template <typename C> struct Dft<4, C> {
    static __device__ __forceinline__ void run(C *v) {
        C t0 = cadd(v[0], v[2]);
        C t1 = csub(v[0], v[2]);
        C t2 = cadd(v[1], v[3]);
        C t3 = cmul_mi(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

template <typename C> struct Dft<8, C> {
    static __device__ __forceinline__ void run(C *v) {
        using T = decltype(v[0].x);
        const T r2 = (T)0.70710678118654752440084436210485;
        C e[4] = {v[0], v[2], v[4], v[6]};
        C o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4, C>::run(e);
        Dft<4, C>::run(o);
        // o[k] *= W8^k, W8 = (1 - i)/sqrt2
        C o1, o3;
        o1.x = r2 * (o[1].x + o[1].y);
        o1.y = r2 * (o[1].y - o[1].x);
        C o2 = cmul_mi(o[2]);
        o3.x = r2 * (o[3].y - o[3].x);
        o3.y = -r2 * (o[3].x + o[3].y);
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    }
};

// ---- one Stockham stage on an LDS line -----------------------------------------------------------
// d: the line's element 0; element e at d[e * ES].  tw: table of W_TB^j with TB = L * TS.
template <typename T, int L, int R, int NS, int TPL, int ES, int TS>
__device__ __forceinline__ void stockham_stage(V2<T> *d, int jt, const V2<T> *__restrict__ tw) {
    using C = V2<T>;
    constexpr int NB = L / (R * TPL);
    static_assert(NB * R * TPL == L, "stage does not tile the line");
    C v[NB][R];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = jt + b * TPL;
#pragma unroll
        for (int m = 0; m < R; ++m) v[b][m] = d[(j + m * (L / R)) * ES];
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = jt + b * TPL;
        const int k = j % NS;
        if constexpr (NS > 1) {
#pragma unroll
            for (int m = 1; m < R; ++m) v[b][m] = cmul(v[b][m], tw[k * m * (L / (NS * R)) * TS]);
        }
        Dft<R, C>::run(v[b]);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int m = 0; m < R; ++m) d[(base + m * NS) * ES] = v[b][m];
    }
    __syncthreads();
}

template <typename T, int L, int E, int ES, int TS, int S = 0>
__device__ __forceinline__ void line_fft(V2<T> *d, int jt, const V2<T> *__restrict__ tw) {
    constexpr RPlan P = make_rplan(L, E);
    if constexpr (S < P.n) {
        constexpr int R = P.r[S];
        constexpr int NS = rplan_span(P, S);
        stockham_stage<T, L, R, NS, L / E, ES, TS>(d, jt, tw);
        line_fft<T, L, E, ES, TS, S + 1>(d, jt, tw);
    }
}

}  // namespace tk
