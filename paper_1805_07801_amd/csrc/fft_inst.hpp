// Registry builders: instantiate the pass kernels for the supported line lengths and
// every tile-shape candidate that fits.
#pragma once

#include "fft_kernels.hpp"

namespace tk {

template <typename T> constexpr tk_dtype dtype_of();
template <> constexpr tk_dtype dtype_of<float>() { return TK_F32; }
template <> constexpr tk_dtype dtype_of<double>() { return TK_F64; }

template <typename T, int L, int CE, int CN> void add_strided(std::vector<StridedKernel> &v) {
    if constexpr (strided_cand_ok<T>(L, CE, CN)) {
        constexpr int E = default_E(L) << CE;
        constexpr int NT = 256 << CN;
        constexpr int W = NT * E / L;
        v.push_back({L, dtype_of<T>(), W, E, NT, strided_lds<T>(L, W), &launch_strided<T, L, E, W>, 0});
        v.push_back({L, dtype_of<T>(), W, E, NT, strided_lds<T>(L, W), &launch_strided<T, L, E, W, 1>, 4});
        // split exchanges where the full LDS tile leaves room for one or two workgroups per CU
        if constexpr (sizeof(T) == 4 && L >= 512 && strided_lds<T>(L, W) > 65536) {
            constexpr int lds_split = (L * (W + 1) + 2 * L) * (int)sizeof(T);
            v.push_back({L, dtype_of<T>(), W, E, NT, lds_split, &launch_strided<T, L, E, W, 0, true>, 5});
            v.push_back({L, dtype_of<T>(), W, E, NT, lds_split, &launch_strided<T, L, E, W, 1, true>, 6});
        }
        // the persistent variant holds two tiles' points per thread: kept where they take
        // under half of the registers a thread has at this workgroup size (512 / (NT / 256))
        if constexpr (E <= 32 && 2 * E * 2 * (int)sizeof(T) / 4 <= 512 / (NT / 256) / 2 - 8)
        {
            v.push_back({L, dtype_of<T>(), W, E, NT, strided_lds<T>(L, W), &launch_strided_pp<T, L, E, W, 1>, 1});
            v.push_back({L, dtype_of<T>(), W, E, NT, strided_lds<T>(L, W), &launch_strided_pp<T, L, E, W, 2>, 2});
            v.push_back({L, dtype_of<T>(), W, E, NT, strided_lds<T>(L, W), &launch_strided_pp<T, L, E, W, 3>, 3});
        }
        // the same with two workgroups per CU: the LDS must hold two tiles and the two
        // tiles' points must fit in the registers a thread keeps at 2 NT / 256 waves per SIMD
        if constexpr (sizeof(T) == 4 && NT >= 512 && 2 * strided_lds<T>(L, W) <= 160 * 1024 &&
                      4 * E <= 512 / (2 * NT / 256) - 40) {
            constexpr int WPE = 2 * NT / 256;
            v.push_back({L, dtype_of<T>(), W, E, NT, strided_lds<T>(L, W), &launch_strided_pp<T, L, E, W, 1, WPE>, 7});
            v.push_back({L, dtype_of<T>(), W, E, NT, strided_lds<T>(L, W), &launch_strided_pp<T, L, E, W, 2, WPE>, 8});
            v.push_back({L, dtype_of<T>(), W, E, NT, strided_lds<T>(L, W), &launch_strided_pp<T, L, E, W, 3, WPE>, 9});
        }
    }
}

template <typename T, int N, int CE, int CN> void add_z(std::vector<ZKernel> &v) {
    if constexpr (z_cand_ok<T>(N, CE, CN)) {
        constexpr int L = N / 2;
        constexpr int E = default_E(L) << CE;
        constexpr int NT = 256 << CN;
        constexpr int LPW = NT / (L / E);
        v.push_back({N, dtype_of<T>(), LPW, E, NT, (int)((LPW * lds_line_len<L>() + 2 * L) * sizeof(V2<T>)),
                     &launch_z_r2c<T, L, E, LPW>, &launch_z_c2r<T, L, E, LPW>});
    }
}

// FP32: E in {Ed, 2 Ed, 4 Ed} x NT in {256, 512, 1024} for strided passes,
//       E in {Ed, 2 Ed} x NT in {256, 512} for Z passes.
template <int L> void add_all_f32(std::vector<StridedKernel> &s, std::vector<ZKernel> &z) {
    add_strided<float, L, 0, 0>(s); add_strided<float, L, 0, 1>(s); add_strided<float, L, 0, 2>(s);
    add_strided<float, L, 1, 0>(s); add_strided<float, L, 1, 1>(s); add_strided<float, L, 1, 2>(s);
    add_strided<float, L, 2, 0>(s); add_strided<float, L, 2, 1>(s);
    add_z<float, L, 0, 0>(z); add_z<float, L, 0, 1>(z); add_z<float, L, 1, 0>(z); add_z<float, L, 1, 1>(z);
}

// FP64: E = Ed, NT in {256, 512} (strided) and NT = 256 (Z).
template <int L> void add_all_f64(std::vector<StridedKernel> &s, std::vector<ZKernel> &z) {
    add_strided<double, L, 0, 0>(s); add_strided<double, L, 0, 1>(s);
    add_z<double, L, 0, 0>(z);
}

}  // namespace tk
