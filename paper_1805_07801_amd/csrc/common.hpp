// Shared host/device helpers of libtk: status handling, complex vector types,
// twiddle tables and launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/tk.h"

namespace tk {

// ---- status / error text -----------------------------------------------------------
void set_error(const char *fmt, ...);
tk_status fail(tk_status st, const char *fmt, ...);

#define TK_HIP_CHECK(expr)                                                              \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::tk::fail(TK_EHIP, "%s failed: %s (%s:%d)", #expr,                  \
                              hipGetErrorString(e_), __FILE__, __LINE__);               \
    } while (0)

#define TK_TRY(expr)                     \
    do {                                 \
        tk_status s_ = (expr);           \
        if (s_ != TK_OK) return s_;      \
    } while (0)

// Checks the launch status of the last kernel.
tk_status launch_check(const char *what);

// ---- supported line lengths: 2^a or 3*2^a, 8..1024 -------------------------------------
inline bool supported_len(int n) {
    if (n < 8 || n > 1024) return false;
    int m = n;
    if (m % 3 == 0) m /= 3;
    return (m & (m - 1)) == 0;
}

// ---- complex vector types ----------------------------------------------------------------
template <typename T> struct V2T;
template <> struct V2T<float> { using type = float2; };
template <> struct V2T<double> { using type = double2; };
template <typename T> using V2 = typename V2T<T>::type;

template <typename T> __host__ __device__ inline V2<T> mk(T x, T y) {
    V2<T> r;
    r.x = x;
    r.y = y;
    return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename C> __device__ __forceinline__ C cconj(C a) { a.y = -a.y; return a; }
// -i * a
template <typename C> __device__ __forceinline__ C cmul_mi(C a) { C r; r.x = a.y; r.y = -a.x; return r; }
// +i * a
template <typename C> __device__ __forceinline__ C cmul_pi(C a) { C r; r.x = -a.y; r.y = a.x; return r; }
template <typename C, typename S> __device__ __forceinline__ C cscale(C a, S s) { a.x *= s; a.y *= s; return a; }

// ---- twiddle tables ------------------------------------------------------------------------
// w[j] = exp(-2 pi i j / n), j < n, evaluated in FP64 with the exact integer argument,
// then rounded to T.  Device copy owned by the caller of make_twiddles.
template <typename T> std::vector<V2<T>> twiddles_host(int n);

// Per-device cache of twiddle tables keyed by (n, dtype); lives until process exit.
const void *twiddle_table(int n, tk_dtype dt, tk_status *st);

// ---- launch helpers -------------------------------------------------------------------------
// Workgroup index remapped so that consecutive logical tiles land on the same XCD:
// the hardware hands out workgroups round-robin over the 8 XCDs, so block b runs on XCD
// b % 8.  Logical tile = (b % 8) * (nb / 8) + b / 8 for the first 8 * (nb / 8) blocks.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb) {
    unsigned full = nb & ~7u;
    if (b >= full) return b;
    unsigned per = full >> 3;
    return (b & 7u) * per + (b >> 3);
}

// Tile of block b of nb for a pass that sweeps its data once from one end to the other
// (from the far end when rev): blocks are dealt to the 8 XCDs in turn, and inside each
// window of 64 blocks an XCD takes 8 consecutive tiles (neighbours share the cache lines
// at their boundaries); windows follow each other in order.  A pass that starts where
// the previous pass ended finds that pass's last writes still in the memory-side cache.
// The partial last window keeps the identity.
__device__ __forceinline__ unsigned sweep_tile(unsigned b, unsigned nb, int rev) {
    const unsigned full = nb & ~63u;
    const unsigned t = b >= full ? b : (b & ~63u) | ((b & 7u) << 3) | ((b >> 3) & 7u);
    return rev ? nb - 1 - t : t;
}

inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace tk
