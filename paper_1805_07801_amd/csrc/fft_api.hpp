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
    // bases along x, y and z: 0 Fourier, 1 sine, 2 cosine (a sine / cosine z basis only
    // with sine / cosine x and y bases: the SSS family, whose spectral data stay real)
    int bx = 0, by = 0, bz = 0;
    const R2RKernel *rx = nullptr, *ry = nullptr;
    const ZR2RKernel *rz = nullptr;
    const void *twqx = nullptr, *twqy = nullptr, *twqz = nullptr;
};

tk_status axes_init(FftAxes *ax, int nx, int ny, int nz, tk_dtype dt, bool use_tune);
// Sine / cosine bases along x and/or y, and along z for the SSS family (after axes_init).
tk_status axes_set_basis(FftAxes *ax, int bx, int by, int bz = 0);
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

// The three passes of the SSS family over `nfields` real fields [nfields][nx][ny][nz]: the z
// sine / cosine pass (src -> dst, not in place) and the x and y passes on the data viewed as
// complex pairs along z (in place allowed).
tk_status sss_z_pass(const FftAxes &ax, const void *src, void *dst, long nfields, int inv, hipStream_t s);
tk_status sss_y_pass(const FftAxes &ax, const void *src, void *dst, long nfields, int inv, hipStream_t s);
tk_status sss_x_pass(const FftAxes &ax, const void *src, void *dst, long nfields, int inv, double scale,
                     hipStream_t s);

}  // namespace tk
