// Internal interface of the 3D transform passes, shared by the FFT plans and the solver.
#pragma once

#include "fft_kernels.hpp"

namespace tk {

// Kernels and twiddle tables for one (nx, ny, nz, dtype) grid.
struct FftAxes {
    int nx, ny, nz;
    tk_dtype dt;
    const void *twx, *twy, *twz;
    const StridedKernel *kx, *ky;
    const ZKernel *kz;
    // bases along x and y: 0 Fourier, 1 sine, 2 cosine (z is always Fourier)
    int bx = 0, by = 0;
    const R2RKernel *rx = nullptr, *ry = nullptr;
    const void *twqx = nullptr, *twqy = nullptr;
};

tk_status axes_init(FftAxes *ax, int nx, int ny, int nz, tk_dtype dt, bool use_tune);
// Sine / cosine bases along x and/or y (after axes_init).
tk_status axes_set_basis(FftAxes *ax, int bx, int by);
// want_W / want_nt = 0 selects the default candidate.
const StridedKernel *pick_strided(int L, tk_dtype dt, int want_W, int want_E, int want_v);
const ZKernel *pick_z(int N, tk_dtype dt, int want_nt, int want_E);
tk_status strided_pass(const StridedKernel *k, const void *src, void *dst, long ncols, long CB, long SO,
                       long SI, const void *tw, int inv, double scale, hipStream_t s, int rev = 0);

// Passes over `nfields` consecutive spectral fields [nfields][nx][ny][nz/2+1].  rev: sweep
// the data from the far end, to start where the previous pass ended (see sweep_tile).
tk_status fft_y_pass(const FftAxes &ax, const void *src, void *dst, long nfields, int inv, hipStream_t s,
                     int rev = 0);
tk_status fft_x_pass(const FftAxes &ax, const void *src, void *dst, long nfields, int inv, double scale,
                     hipStream_t s, int rev = 0);
tk_status fft_z_r2c(const FftAxes &ax, const void *src, void *dst, long nfields, double scale, hipStream_t s,
                    int rev = 0);
tk_status fft_z_c2r(const FftAxes &ax, const void *src, void *dst, long nfields, hipStream_t s, int rev = 0);

}  // namespace tk
