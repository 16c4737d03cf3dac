// Registry builders: instantiate every pass kernel for the supported line lengths.
#pragma once

#include "fft_kernels.hpp"

namespace tk {

template <typename T> constexpr tk_dtype dtype_of();
template <> constexpr tk_dtype dtype_of<float>() { return TK_F32; }
template <> constexpr tk_dtype dtype_of<double>() { return TK_F64; }

template <typename T, int L, int C> void add_strided(std::vector<StridedKernel> &v) {
    constexpr int E = default_E(L);
    constexpr int W = strided_Wb(L, E) << C;
    static_assert(rplan_ok(L, E), "bad radix plan");
    if constexpr (strided_ok<T>(L, E, W))
        v.push_back({L, dtype_of<T>(), W, E, W * (L / E), (int)(L * W * sizeof(V2<T>)), &launch_strided<T, L, E, W>});
}

template <typename T, int N> void add_z(std::vector<ZKernel> &v) {
    constexpr int L = N / 2;
    constexpr int E = default_E(L);
    constexpr int LPW = z_LPW(L, E);
    static_assert(rplan_ok(L, E), "bad radix plan");
    v.push_back({N, dtype_of<T>(), LPW, E, LPW * (L / E), (int)(LPW * (L + 1) * sizeof(V2<T>)),
                 &launch_z_r2c<T, L, E, LPW>, &launch_z_c2r<T, L, E, LPW>});
}

// The supported lengths: 2^a and 3 * 2^a in [8, 1024].
#define TK_FOR_EACH_LEN(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

}  // namespace tk
