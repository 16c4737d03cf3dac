/*
 * FP64 CPU oracle for the 3D real-to-complex / complex-to-real Fourier transform.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
 * that the GPU library is checked against.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * tables or headers with the GPU library.
 *
 * Conventions (paper, Section "Fast Fourier Transform", Eq. for f(x,y,z) with the
 * Fourier basis exp(iks)):
 *   inverse:  f(x) = sum_k F(k) exp(+i k.x)           (plain sum, no 1/N)
 *   forward:  F(k) = N^-3 sum_x f(x) exp(-i k.x)       (so inverse(forward) = id)
 * Array layout: real [nx][ny][nz], complex [nx][ny][nz/2+1], C order, z fastest
 * (the n0 x n1 x (n2/2+1) layout of the paper's Appendix A).
 *
 * The 3D transform is done axis by axis: Z first on the forward transform, then Y,
 * then X (paper, Section "Parallelization Strategy", steps 1, 3, 5); the inverse is
 * the reverse order.  Each 1D transform is a textbook recursive decimation-in-time
 * mixed-radix Cooley-Tukey FFT: n = p*m with p the smallest prime factor of n,
 *   X[k + q m] = sum_{r<p} w_n^{r(k+qm)} Y_r[k],   Y_r = DFT_m(x[r + p j]).
 * Roots of unity are cos/sin of 2*pi*(j mod n)/n evaluated in double precision,
 * with the integer reduction done exactly.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;

/* Smallest prime factor of n (n >= 2). */
static int smallest_factor(int n) {
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* w[j] = exp(sign * 2*pi*i * j / n), j = 0..n-1. */
static void roots(cplx *w, int n, int sign) {
    const double two_pi = 6.283185307179586476925286766559;
    for (int j = 0; j < n; ++j) {
        double a = two_pi * (double)j / (double)n;
        w[j] = cos(a) + sign * I * sin(a);
    }
}

/*
 * out[0..n-1] = DFT_n of in[0], in[istr], in[2 istr], ...
 * w is the root table of the top-level length ntop; the n-th root used here is
 * w[wstep] with wstep = ntop / n.
 */
static void fft_rec(const cplx *in, long istr, cplx *out, int n, const cplx *w, int wstep, int ntop) {
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    int p = smallest_factor(n);
    int m = n / p;
    for (int r = 0; r < p; ++r)
        fft_rec(in + r * istr, istr * p, out + (long)r * m, m, w, wstep * p, ntop);
    cplx t[64];
    cplx *tp = (p <= 64) ? t : (cplx *)malloc(sizeof(cplx) * p);
    for (int k = 0; k < m; ++k) {
        for (int r = 0; r < p; ++r) {
            long e = ((long)r * k) % n; /* w_n^{r k} */
            tp[r] = out[(long)r * m + k] * w[e * wstep];
        }
        for (int q = 0; q < p; ++q) {
            cplx s = 0;
            for (int r = 0; r < p; ++r) {
                long e = ((long)r * q * m) % n; /* w_n^{r q m} = w_p^{r q} */
                s += tp[r] * w[e * wstep];
            }
            out[k + (long)q * m] = s;
        }
    }
    if (tp != t) free(tp);
}

/* In-place 1D DFT of a strided line: x[j*stride], j < n; sign -1 forward, +1 inverse, unscaled. */
static void fft_line(cplx *x, long stride, int n, const cplx *w, cplx *buf_in, cplx *buf_out) {
    for (int j = 0; j < n; ++j) buf_in[j] = x[j * stride];
    fft_rec(buf_in, 1, buf_out, n, w, 1, n);
    for (int j = 0; j < n; ++j) x[j * stride] = buf_out[j];
}

/* Exported: 1D complex DFT, in place, unscaled. sign = -1 or +1. Returns 0 on success. */
int orc_fft1d(double *data, int n, int sign) {
    if (n < 1 || (sign != 1 && sign != -1)) return -1;
    cplx *x = (cplx *)data;
    cplx *w = (cplx *)malloc(sizeof(cplx) * n);
    cplx *a = (cplx *)malloc(sizeof(cplx) * n);
    cplx *b = (cplx *)malloc(sizeof(cplx) * n);
    roots(w, n, sign);
    fft_line(x, 1, n, w, a, b);
    free(w); free(a); free(b);
    return 0;
}

/*
 * Batched complex transform along one axis of a C-order complex array of shape
 * [n0][n1][n2]: axis 0, 1 or 2.  Unscaled; sign -1 forward, +1 inverse.
 */
static void c2c_axis(cplx *a, int n0, int n1, int n2, int axis, int sign) {
    int n = axis == 0 ? n0 : axis == 1 ? n1 : n2;
    long stride = axis == 0 ? (long)n1 * n2 : axis == 1 ? n2 : 1;
    long nlines = ((long)n0 * n1 * n2) / n;
    cplx *w = (cplx *)malloc(sizeof(cplx) * n);
    roots(w, n, sign);
#pragma omp parallel
    {
        cplx *bi = (cplx *)malloc(sizeof(cplx) * n);
        cplx *bo = (cplx *)malloc(sizeof(cplx) * n);
#pragma omp for schedule(static)
        for (long l = 0; l < nlines; ++l) {
            long base;
            if (axis == 2) base = l * n2;
            else if (axis == 1) base = (l / n2) * (long)n1 * n2 + (l % n2);
            else base = l;
            fft_line(a + base, stride, n, w, bi, bo);
        }
        free(bi); free(bo);
    }
    free(w);
}

/*
 * Exported: forward 3D r2c.  in: real [nx][ny][nz]; out: complex [nx][ny][nz/2+1]
 * (interleaved re, im doubles).  out = N^-3 sum_x f(x) exp(-i k.x), N^3 = nx*ny*nz.
 * Z is transformed first as a full complex line, of which kz = 0..nz/2 is kept.
 */
int orc_rfft3(const double *in, double *out_d, int nx, int ny, int nz) {
    if (nx < 1 || ny < 1 || nz < 2 || (nz & 1)) return -1;
    int nzh = nz / 2 + 1;
    cplx *out = (cplx *)out_d;
    cplx *w = (cplx *)malloc(sizeof(cplx) * nz);
    roots(w, nz, -1);
    long nlines = (long)nx * ny;
#pragma omp parallel
    {
        cplx *bi = (cplx *)malloc(sizeof(cplx) * nz);
        cplx *bo = (cplx *)malloc(sizeof(cplx) * nz);
#pragma omp for schedule(static)
        for (long l = 0; l < nlines; ++l) {
            for (int j = 0; j < nz; ++j) bi[j] = in[l * nz + j];
            fft_rec(bi, 1, bo, nz, w, 1, nz);
            for (int k = 0; k < nzh; ++k) out[l * nzh + k] = bo[k];
        }
        free(bi); free(bo);
    }
    free(w);
    c2c_axis(out, nx, ny, nzh, 1, -1);
    c2c_axis(out, nx, ny, nzh, 0, -1);
    double s = 1.0 / ((double)nx * (double)ny * (double)nz);
    long tot = nlines * nzh;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < tot; ++i) out[i] *= s;
    return 0;
}

/*
 * Exported: inverse 3D c2r, unscaled.  in: complex [nx][ny][nz/2+1] (not modified);
 * out: real [nx][ny][nz].
 *   f(x) = sum_{kz=0}^{nz/2} w(kz) Re[ sum_{kx,ky} F(k) exp(i k.x) ],
 * w = 1 at kz = 0 and nz/2, 2 otherwise: the plain sum over the Hermitian extension.
 * X then Y are full complex inverses; the Z line is extended by F(-kz) = conj F(kz),
 * with the kz = 0 and nz/2 entries replaced by their real parts, and the real part of
 * its complex inverse is kept.
 */
int orc_irfft3(const double *in_d, double *out, int nx, int ny, int nz) {
    if (nx < 1 || ny < 1 || nz < 2 || (nz & 1)) return -1;
    int nzh = nz / 2 + 1;
    long nlines = (long)nx * ny;
    long tot = nlines * nzh;
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * tot);
    if (!tmp) return -2;
    memcpy(tmp, in_d, sizeof(cplx) * tot);
    c2c_axis(tmp, nx, ny, nzh, 0, +1);
    c2c_axis(tmp, nx, ny, nzh, 1, +1);
    cplx *w = (cplx *)malloc(sizeof(cplx) * nz);
    roots(w, nz, +1);
#pragma omp parallel
    {
        cplx *bi = (cplx *)malloc(sizeof(cplx) * nz);
        cplx *bo = (cplx *)malloc(sizeof(cplx) * nz);
#pragma omp for schedule(static)
        for (long l = 0; l < nlines; ++l) {
            const cplx *g = tmp + l * nzh;
            bi[0] = creal(g[0]);
            bi[nz / 2] = creal(g[nz / 2]);
            for (int k = 1; k < nz / 2; ++k) {
                bi[k] = g[k];
                bi[nz - k] = conj(g[k]);
            }
            fft_rec(bi, 1, bo, nz, w, 1, nz);
            for (int j = 0; j < nz; ++j) out[l * nz + j] = creal(bo[j]);
        }
        free(bi); free(bo);
    }
    free(w);
    free(tmp);
    return 0;
}

/* Exported: number of OpenMP threads the oracle uses. */
int orc_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
