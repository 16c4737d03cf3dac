/*
 * tk.h -- C ABI of libtk, an MI355X (gfx950) implementation of the FFTK/Tarang hot path:
 * the 3D real-to-complex / complex-to-real FFT and the pseudo-spectral Navier-Stokes
 * step built on it (Chatterjee et al., "Scaling of a Fast Fourier Transform and a
 * Pseudo-spectral Fluid Solver up to 196608 cores").
 *
 * General conventions
 *  - Every data pointer is a DEVICE pointer owned by the caller, unless stated.  Handles
 *    own their internal tables and scratch memory.  Nothing is freed behind the caller.
 *  - Streams are hipStream_t values passed as void*; NULL is the default stream.  Calls
 *    are asynchronous on the stream unless documented as synchronising.
 *  - Every call returns a tk_status; no exception crosses the ABI.  On a non-OK status,
 *    tk_last_error() returns a thread-local message, and no partial work was queued
 *    unless the status is TK_EHIP (a launch failure).
 *  - Calls on one handle must not overlap in time from several host threads.
 *  - Real fields are C-order [nx][ny][nz] (z fastest); spectral fields are C-order
 *    [nx][ny][nz/2+1] complex, interleaved (re, im): the n0 x n1 x (n2/2+1) layout of the
 *    paper's Appendix A.  Wavenumbers along x and y are 0..n/2-1, -n/2..-1; kz = 0..nz/2.
 *  - Supported line lengths: n = 2^a or 3 * 2^a with 8 <= n <= 1024 (the paper's XC40
 *    grids are 3 * 2^n; Section "Scaling on Cray XC40").  Others give TK_EUNSUPPORTED.
 */
#ifndef TK_H
#define TK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TK_OK = 0,
    TK_EINVAL = -1,        /* bad argument (null pointer, negative count, ...) */
    TK_EUNSUPPORTED = -2,  /* valid request this library does not implement (size, dtype) */
    TK_ENOMEM = -3,        /* device or host allocation failed */
    TK_EHIP = -4,          /* a HIP call or kernel launch failed */
    TK_ESTATE = -5         /* handle in the wrong state, or non-finite diagnostics */
} tk_status;

typedef enum { TK_F32 = 0, TK_F64 = 1 } tk_dtype;

typedef struct tk_fft3d_s *tk_fft3d_t;
typedef struct tk_ns_s *tk_ns_t;
typedef struct tk_nsb_s *tk_nsb_t;
typedef struct tk_rbc_s *tk_rbc_t;

/* Thread-local text describing the last non-OK status of this thread ("" if none). */
const char *tk_last_error(void);

/* ABI version (major * 10000 + minor * 100 + patch). */
int tk_version(void);

/* *out = sum of x_i^2 over n real values (device, dtype dt), accumulated in FP64 with a
 * fixed reduction order.  Synchronises stream. */
tk_status tk_sum_squares(const void *x, long n, tk_dtype dt, double *out, void *stream);

/* ------------------------------------------------------------------------------------
 * 3D FFT in the Fourier (FFF) basis.
 * Paper, Section "Fast Fourier Transform": the inverse transform is the plain sum
 *   f(x) = sum_k F(k) exp(+i k.x),
 * so the forward transform carries the 1/(nx ny nz) factor:
 *   F(k) = (nx ny nz)^-1 sum_x f(x) exp(-i k.x).
 * Section "Parallelization Strategy": forward = Z r2c, then Y c2c, then X c2c; the
 * inverse is the reverse.  On one GPU the two all-to-all exchanges of the pencil
 * algorithm disappear and, as in the transpose-free scheme of Appendix A, the axes
 * are never permuted: the Y and X passes read strided columns through LDS tiles.
 * ------------------------------------------------------------------------------------ */

/* Flags for fft3d_plan_create. */
#define TK_FFT_TIMING 0x1u    /* record per-pass HIP events (fft3d_pass_times) */
#define TK_FFT_NO_TUNE 0x2u   /* ignore the autotuner cache, use default tiles */
#define TK_FFT_C2R_Y_FIRST 0x4u /* c2r: inverse Y (out of place) before X (in place); same result */
#define TK_FFT_C2R_OVERWRITE 0x8u /* c2r may overwrite cplx_in: X and Y inverses in place on it, no
                                     workspace (FFTW's default for c2r); same result */

/* Create a plan for `batch` fields of nx*ny*nz points in dtype dt.  Allocates twiddle
 * tables (a few KB) on the current device.  Sizes must be supported (see above);
 * batch >= 1.  Returns TK_EUNSUPPORTED for unsupported sizes, TK_EINVAL for null. */
tk_status fft3d_plan_create(tk_fft3d_t *plan, int nx, int ny, int nz, int batch, tk_dtype dt,
                            unsigned flags);

/* Bases of an axis (paper, Section "Fast Fourier Transform": exp(iks), 2 sin(ks), 2 cos(ks);
 * the SFF / SSF combinations for free-slip walls). */
#define TK_FOURIER 0
#define TK_SINE 1
#define TK_COSINE 2

/* As fft3d_plan_create, with the sine or cosine basis along x and/or y (z stays Fourier).
 * On a sine/cosine axis of N points the grid is x_j = pi (j + 1/2) / N; the forward
 * transform is F_k = (1/N) sum_j f_j cos(k x_j) (k = 0..N-1) or (1/N) sum_j f_j sin(k x_j)
 * (k = 1..N, stored at index k - 1), and the inverse f = F_0 + sum_{k>0} 2 F_k cos(k x) or
 * f = sum_{k<N} 2 F_k sin(k x) + F_N sin(N x).  Layouts as for the Fourier basis. */
tk_status fft3d_plan_create_basis(tk_fft3d_t *plan, int nx, int ny, int nz, int batch, tk_dtype dt, int basis_x,
                                  int basis_y, unsigned flags);

/* As fft3d_plan_create_basis with a basis along z too.  basis_z = TK_FOURIER is
 * fft3d_plan_create_basis.  A sine or cosine z basis (the SSS family of the paper's
 * Section "Fast Fourier Transform", e.g. cos x cos y sin z for u_z of free-slip walls)
 * needs sine or cosine x and y bases (else TK_EUNSUPPORTED): every axis then takes its
 * sine / cosine transform as above (z on the grid z_j = pi (j + 1/2) / nz too, 1/N per axis
 * forward), and the spectral data are REAL, [batch][nx][ny][nz] of dtype dt, coefficient
 * (kx, ky, kz) at [kx][ky][kz] (sine k at index k - 1), wherever the calls below say
 * "cplx".  fft3d_parseval does not apply to such plans (TK_EUNSUPPORTED). */
tk_status fft3d_plan_create_basis3(tk_fft3d_t *plan, int nx, int ny, int nz, int batch, tk_dtype dt, int basis_x,
                                   int basis_y, int basis_z, unsigned flags);

/* Bytes of device workspace fft3d_c2r needs (one spectral field per batch member; none
 * with TK_FFT_C2R_OVERWRITE). */
tk_status fft3d_workspace_size(tk_fft3d_t plan, size_t *bytes);

/* Supply caller-owned device workspace of at least fft3d_workspace_size bytes (NULL
 * returns to plan-owned workspace, allocated lazily on the first c2r).  The caller must
 * keep it alive while the plan uses it. */
tk_status fft3d_set_workspace(tk_fft3d_t plan, void *dev_ptr);

/* Forward r2c: real_in [batch][nx][ny][nz] -> cplx_out [batch][nx][ny][nz/2+1],
 * scaled by 1/(nx ny nz).  real_in is not modified.  The buffers must not overlap. */
tk_status fft3d_r2c(tk_fft3d_t plan, const void *real_in, void *cplx_out, void *stream);

/* Inverse c2r, unscaled: cplx_in -> real_out.  cplx_in is preserved (the solver needs
 * its spectral state intact) unless the plan has TK_FFT_C2R_OVERWRITE, which leaves it
 * holding the partial (X- and Y-inverted) transform.  On the kz = 0 and kz = nz/2 planes only the Hermitian
 * part matters: the result is sum_{kz} w(kz) Re[sum_{kx,ky} F(k) exp(i k.x)] with
 * w = 1 on those planes and 2 elsewhere. */
tk_status fft3d_c2r(tk_fft3d_t plan, const void *cplx_in, void *real_out, void *stream);

/* Bytes of the static device scratch fft3d_c2r_noalloc uses as its workspace (80 MiB: a
 * 256^3 FP32 or 192^3 FP64 half spectrum fits). */
#define TK_SCRATCH_BYTES (80u << 20)

/* As fft3d_c2r (same passes, same result, input preserved), but allocation-free: for
 * callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The workspace is a static device
 * array of TK_SCRATCH_BYTES that every device running this library holds until the
 * process ends; its address is looked up once per device on the first call there.  The
 * call allocates nothing and needs no clearing (the first pass overwrites the whole
 * workspace).  Plans whose spectral field (times batch) exceeds TK_SCRATCH_BYTES get
 * TK_EINVAL with nothing queued.  All calls on one device share the one array: calls
 * that may overlap in time on one device (several streams, several host threads) race
 * and must be serialised by the caller.  Plans with TK_FFT_C2R_OVERWRITE need no
 * workspace and behave exactly as fft3d_c2r. */
tk_status fft3d_c2r_noalloc(tk_fft3d_t plan, const void *cplx_in, void *real_out, void *stream);

/* Parseval sums in FP64: out[0] = sum f^2 / (nx ny nz) over the real field (batch
 * member 0), out[1] = sum w(kz) |F|^2 over its half spectrum.  Synchronises stream. */
tk_status fft3d_parseval(tk_fft3d_t plan, const void *real, const void *cplx, double out[2],
                         void *stream);

/* Average per-pass durations in ms (t[0..2] = Z, Y, X of r2c; t[3..5] = X, Y, Z of c2r)
 * over the calls made since the previous query (at most the last 256), for a plan created
 * with TK_FFT_TIMING, which records HIP events around every pass on the call's stream
 * without synchronising.  This call synchronises those events and resets the average. */
tk_status fft3d_pass_times(tk_fft3d_t plan, float t[6]);

/* Describe the tile configuration the plan uses for pass p (0 = Z, 1 = Y, 2 = X) as
 * text in buf (NUL-terminated, at most len bytes). */
tk_status fft3d_describe(tk_fft3d_t plan, int pass, char *buf, int len);

tk_status fft3d_plan_destroy(tk_fft3d_t plan);

/* ---- autotuner (tile shapes of the three passes) ----------------------------------------
 * Runs every compiled tile candidate of each pass of an (nx, ny, nz, batch, dt) grid on
 * a pseudo-random field on the current device, timed with HIP events (median of iters
 * launches).  A candidate is admitted only if its output matches the default tile's
 * to relative L2 1e-5 (FP32) / 1e-12 (FP64).  The fastest admitted tile per (length,
 * dtype, pass) goes into a process-wide table that plans created afterwards use (unless
 * created with TK_FFT_NO_TUNE).  Allocates and frees three spectral-field buffers.
 * report (may be NULL) receives one text line per candidate.  Synchronises. */
tk_status fft3d_autotune(int nx, int ny, int nz, int batch, tk_dtype dt, int iters, char *report,
                         int report_len);

/* Force the tile of (L, dt, pass): pass 0 = Z (a = threads per workgroup), 1 = Y and
 * 2 = X (a = columns per tile); E = points per thread; variant (strided passes; 0 for Z):
 * 0 = one tile per workgroup sweeping the tiles once; 1..3 = persistent workgroups that
 * issue the next tile's loads before transforming the current one (1: tiles dealt
 * round-robin, 2: round-robin with a contiguous run per XCD, 3: consecutive tiles per
 * workgroup); 4 = one tile per workgroup, each XCD sweeping its own eighth of the tiles;
 * 5, 6 = 0 and 4 with split exchanges (real, then imaginary parts through half the LDS);
 * 7..9 = 1..3 with the registers held to what two resident workgroups per CU allow.
 * Passes 3, 4, 5 are the solver passes P1 (a = columns), P3 (a = lines per workgroup) and
 * P5 (a = columns) of an L^3 grid (variant 0), pass 6 the solver's Y passes P2 / P4 (a
 * strided tile as for pass 1), pass 7 the time stepper's P5 fused with the next P1 (a =
 * columns); solver handles created afterwards use them.  Pass 8 is the tile of the ensemble
 * kernels of grid size L (FP32 only): a = threads per workgroup, E = default_E(L) (8, or 12
 * for 3 * 2^a), variant v = persistent grid of 256 << v workgroups (v = 0..6); ensembles
 * created afterwards use it.  a <= 0 removes the entry.
 * TK_EUNSUPPORTED if no such tile is compiled. */
tk_status fft3d_tune_set(int L, tk_dtype dt, int pass, int a, int E, int variant);

/* Autotune the solver passes P1, P2 / P4, P3, P5 and the fused P5 + P1 of an n^3 grid in
 * dtype dt: every compiled tile variant runs on pseudo-random fields of the grid's size,
 * is admitted only if its output matches the first variant's (the fused pass: P1's) to
 * relative L2 1e-5 (FP32) / 1e-12 (FP64), and is timed (median of iters launches); the
 * fastest admitted variant of each pass goes into the tile table (passes 3..7).
 * Allocates 18 spectral fields for the duration of the call.
 * report (may be NULL) receives one text line per variant.  Synchronises. */
tk_status ns_autotune(int n, tk_dtype dt, int iters, char *report, int report_len);

/* Autotune the ensemble kernels of grid size n (16..128, FP32): an ensemble of `members`
 * random solenoidal states of that size runs with every compiled thread count (128, 256,
 * 512 per workgroup) and persistent grid (256 ... 16384 workgroups); a candidate is admitted
 * only if its states after two fixed steps match the default shape's (256 threads, 1024
 * workgroups) to relative L2 1e-5, and is timed over `iters` graph-replayed steps; the
 * fastest admitted one goes into the tile table (pass 8).  Allocates three state copies per
 * member for the call.  report (may be NULL) receives one line per candidate.  Synchronises. */
tk_status ns_batch_autotune(int n, int members, int iters, char *report, int report_len);

/* Forget every tuned tile. */
tk_status fft3d_tune_clear(void);

/* Number of compiled tile candidates of (L, dt, pass); the first `cap` are written to
 * a[], E[] and variant[] (any may be NULL). */
int fft3d_tile_candidates(int L, tk_dtype dt, int pass, int *a, int *E, int *variant, int cap);

/* ------------------------------------------------------------------------------------
 * Pseudo-spectral incompressible Navier-Stokes in the periodic (2 pi)^3 box.
 * Paper, Section "Spectral Solver": the Fourier-space momentum equation (eq:NSk) with
 * the constraint k . u^ = 0 (eq:continuity2); nonlinear term pseudo-spectral (to real
 * space, multiply, back), dealiased by the 2/3 rule.  Nine 3D transforms per
 * right-hand side: six inverse (u, omega), three forward (u x omega).
 * State: u^ [3][n][n][n/2+1] complex in dtype, zero outside the 2/3 set and solenoidal.
 * ------------------------------------------------------------------------------------ */

typedef struct {
    int n;            /* grid points per axis (supported length, see above) */
    tk_dtype dtype;   /* TK_F32 or TK_F64 */
    double nu;        /* kinematic viscosity */
    double cfl;       /* > 0: ns_step ignores dt and uses h = cfl (2 pi / n) / max(|ux|+|uy|+|uz|) */
    int scheme;       /* 0: integrating-factor RK2 (Heun); 1: integrating-factor RK4 */
    unsigned flags;   /* reserved, 0 */
} ns_config;

/* Create a solver; allocates its workspace (about 12 spectral fields). */
tk_status ns_create(tk_ns_t *ns, const ns_config *cfg);

/* N(u^) = P M F[u x omega] for state uhat (viscous term excluded): rhs_out has the
 * state's layout.  uhat is not modified. */
tk_status ns_rhs(tk_ns_t ns, const void *uhat, void *rhs_out, void *stream);

/* Advance uhat in place by nsteps steps.  With cfg.cfl > 0 the step size is computed on
 * the device each step (dt is ignored); else h = dt.  *t_inout (host) is advanced by the
 * elapsed time; this synchronises the stream at the end of the call. */
tk_status ns_step(tk_ns_t ns, void *uhat_inout, double dt, int nsteps, double *t_inout,
                  void *stream);

/* FP64 diagnostics of state uhat: energy E = sum w 1/2|u^|^2, dissipation 2 nu sum w
 * 1/2 |k|^2 |u^|^2, shell spectrum E(s) for s < nshell (shell s: (2s-1)^2 <= 4|k|^2 <
 * (2s+1)^2; any pointer may be NULL), and the divergence max_k |k.u^|/|k| relative to
 * max_k |u^|.  Synchronises stream.  Returns TK_ESTATE if the energy is not finite. */
tk_status ns_diagnostics(tk_ns_t ns, const void *uhat, double *energy, double *dissipation,
                         double *spectrum, int nshell, double *max_div, void *stream);

/* Initial state from real Gaussian noise [3][n][n][n] (dtype of the solver): r2c,
 * projection, 2/3 mask, k = 0 removed, each shell s >= 1 rescaled to s^4 exp(-2(s/4)^2),
 * total energy set to `energy`.  Synchronises stream. */
tk_status ns_init_random(tk_ns_t ns, const void *noise, void *uhat_out, double energy,
                         void *stream);

/* Last step size used by ns_step (host value; synchronises nothing). */
tk_status ns_last_dt(tk_ns_t ns, double *dt);

/* Mean duration in ms of each pass of the right-hand side of state uhat, over iters runs
 * timed with HIP events on `stream` (passes of Section "Spectral Solver": curl and
 * X-inverse P1, Y-inverse P2, the fused Z pass with u x omega P3, Y-forward P4, X-forward
 * with projection P5), then of the time stepper's P5 fused with the next P1 (timed in
 * its first-stage form, which writes only the solver's workspace).  ms[0..5] = P1, P2,
 * P3, P4, P5, P5+P1.  uhat is read, never written; the workspace and the step state's
 * CFL maximum are overwritten (ns_step starts afresh).  Synchronises. */
tk_status ns_pass_times(tk_ns_t ns, const void *uhat, int iters, float ms[6], void *stream);

tk_status ns_destroy(tk_ns_t ns);

/* Energy transfer (the paper lists energy flux and shell-to-shell transfer among the
 * solver's diagnostics).  T[s] = sum_{k in shell s} w Re[u^*(k) . N(k)] for the first
 * nshell integer shells (N the nonlinear term of ns_rhs), FP64; the energy flux out of
 * the sphere s0 is -sum_{s <= s0} T[s].  Uses the solver's workspace.  Synchronises. */
tk_status ns_energy_transfer(tk_ns_t ns, const void *uhat, double *T, int nshell, void *stream);

/* Giver/receiver shell-to-shell transfer between bands of integer shells
 * (band_of_shell[s] in [0, nbands) or -1, host array of nshell ints):
 *   Tnm[n * nbands + m] = - sum_{k in band n} w Re[u^*(k) . F((u . grad) u^(m))(k)],
 * u^(m) = u restricted to band m (energy given by band m to band n).  Allocates about
 * 25 real / spectral fields of workspace for the call.  Synchronises. */
tk_status ns_shell_to_shell(tk_ns_t ns, const void *uhat, const int *band_of_shell, int nshell, int nbands,
                            double *Tnm, void *stream);

/* ------------------------------------------------------------------------------------
 * Rayleigh-Benard (Boussinesq) convection, periodic FFF basis: paper, Section "Spectral
 * Solver", eq:u_Usmall_Plarge and eq:T_Usmall_Plarge (viscosity sqrt(Pr/Ra), thermal
 * diffusivity 1/sqrt(Ra Pr), buoyancy theta z, source u_z in the temperature equation), in
 * a periodic box of side `box` (the paper's unit cube: box = 1; wavenumbers 2 pi k / box).
 * State [4][n][n][n/2+1]: u_x, u_y, u_z, theta; 2/3-masked, u solenoidal.  One right-hand
 * side = 7 inverse + 6 forward transforms (13, as the paper counts); IF-RK2 steps.
 * ------------------------------------------------------------------------------------ */
typedef struct {
    int n;
    tk_dtype dtype;
    double Ra, Pr; /* Rayleigh and Prandtl numbers */
    double box;    /* box side (> 0) */
    double cfl;    /* > 0: h = cfl (box / n) / max(|ux|+|uy|+|uz|); else the dt given to rbc_step */
    unsigned flags;
} rbc_config;

tk_status rbc_create(tk_rbc_t *rbc, const rbc_config *cfg);
/* (N_u, N_theta) = (P M [F(u x omega) + theta z], M [-i a k . F(u theta) + u_z]), diffusion
 * excluded, a = 2 pi / box; rhs_out has the state's layout. */
tk_status rbc_rhs(tk_rbc_t rbc, const void *state, void *rhs_out, void *stream);
/* Advance in place by nsteps IF-RK2 steps (one HIP-graph launch each); synchronises. */
tk_status rbc_step(tk_rbc_t rbc, void *state, double dt, int nsteps, double *t_inout, void *stream);
/* FP64: kinetic energy, thermal variance 1/2 <theta^2>, <u_z theta> and the Nusselt number
 * 1 + sqrt(Ra Pr) <u_z theta> (any pointer may be NULL).  Synchronises. */
tk_status rbc_diagnostics(tk_rbc_t rbc, const void *state, double *kinetic, double *thermal, double *uz_theta,
                          double *nusselt, void *stream);
tk_status rbc_last_dt(tk_rbc_t rbc, double *dt);
/* Mean duration in ms of each pass of one right-hand side of state s4 over iters runs timed
 * with HIP events on `stream`: ms[0..4] = P1 (curl and x-inverse of u, theta: 4 -> 7 fields),
 * P2 (y-inverse, 7 fields), P3 (z pass: 7 c2r, u x omega and u theta, 6 r2c), P4 (y-forward,
 * 6 fields), P5 (x-forward, buoyancy, projection).  s4 is only read; the solver's workspace
 * is overwritten.  Synchronises. */
tk_status rbc_pass_times(tk_rbc_t rbc, const void *s4, int iters, float ms[5], void *stream);
tk_status rbc_destroy(tk_rbc_t rbc);

/* ------------------------------------------------------------------------------------
 * Ensembles: `count` independent FP32 solves of mixed grid sizes n[i] in {16, 24, 32,
 * 48, 64, 96, 128} with viscosities nu[i], advanced together by IF-RK2.  Every pass of
 * the right-hand side is one persistent kernel over a work list of all members' tiles
 * (largest grids first), and one step of all members is a single HIP-graph launch (after
 * one transform of the states per call: each step's last pass prepares the next step).
 * Each member's state has the single solver's layout.  flags >> 16, if nonzero, sets
 * the persistent grid size (workgroups; default 1024).
 * ------------------------------------------------------------------------------------ */
tk_status ns_batch_create(tk_nsb_t *b, int count, const int *n, const double *nu, tk_dtype dt, double cfl,
                          unsigned flags);

/* Advance every member by nsteps steps.  uhat: host array of `count` device pointers
 * (member states, in place).  With cfl > 0 each member's step is from its own CFL
 * condition, else h = dt.  t (host, count values, may be NULL) is advanced.
 * Synchronises the stream at the end. */
tk_status ns_batch_step(tk_nsb_t b, void *const *uhat, double dt, int nsteps, double *t, void *stream);

/* Member i's random initial state (as ns_init_random).  Synchronises. */
tk_status ns_batch_init_random(tk_nsb_t b, int i, const void *noise, void *uhat_out, double energy,
                               void *stream);

/* Member i's energy, dissipation and relative divergence (as ns_diagnostics). */
tk_status ns_batch_diagnostics(tk_nsb_t b, int i, const void *uhat, double *energy, double *dissipation,
                               double *max_div, void *stream);

/* Step sizes of the last step of every member (host array of count values). */
tk_status ns_batch_last_dt(tk_nsb_t b, double *dt);

tk_status ns_batch_destroy(tk_nsb_t b);

/* ------------------------------------------------------------------------------------
 * Learned sub-grid closure for coarse LES (not part of the paper's solver: a pointwise
 * network stands in for the sub-grid stress of a filtered field).
 * Network: 9 inputs (the filtered velocity gradients d_j ubar_i, component 3 i + j,
 * divided by in_scale) -> 64 GELU -> 64 GELU -> 6 outputs (tau_xx, yy, zz, xy, xz, yz,
 * in units of out_scale); GELU(x) = x/2 (1 + erf(x/sqrt 2)).  Parameters: TK_MLP_NPARAM
 * BF16 values in the order W1[64][9], b1[64], W2[64][64], b2[64], W3[6][64], b3[6];
 * every product and sum is FP32.  Point arrays are structure-of-arrays: x9 [9][M],
 * y6 / t6 / dy6 [6][M], FP32, device memory.
 * ------------------------------------------------------------------------------------ */
#define TK_MLP_NPARAM 5190

typedef struct {
    const uint16_t *w; /* device: TK_MLP_NPARAM BF16 parameters */
    float in_scale;    /* inputs are divided by it (> 0) */
    float out_scale;   /* outputs are multiplied by it (> 0) */
} tk_mlp;

typedef struct {
    float *w, *m, *v;  /* device: FP32 master parameters and Adam moments (TK_MLP_NPARAM each) */
    float lr, beta1, beta2, eps;
    int step;          /* updates done so far; incremented by sgs_adam_step */
} tk_adam;

/* y6 = out_scale * f(x9 / in_scale) at M points. */
tk_status sgs_mlp_forward(const tk_mlp *w, const float *x9, float *y6, long M, void *stream);

/* grad (device, TK_MLP_NPARAM FP32) = sum over the M points of (d f(x9/in_scale) / d theta)^T
 * dy6, with dy6 the gradient with respect to the normalised network outputs.  Each
 * workgroup sums its points in FP32 (a fixed order), and the workgroups' partial sums are
 * added in a fixed order in FP64, so a result is reproducible on one device.  The partial
 * sums live in a per-device library buffer: backward calls that overlap on one device
 * (concurrent streams, or host threads) must be serialised by the caller. */
tk_status sgs_mlp_backward(const tk_mlp *w, const float *x9, const float *dy6, long M, float *grad,
                           void *stream);

/* Mean-square loss in normalised units, L = mean over the 6 M values of (f(x9/in_scale) -
 * t6/out_scale)^2 (host, FP64; may be NULL: then no synchronisation), and its gradient
 * into grad (as sgs_mlp_backward with dy6 = dL/dy). */
tk_status sgs_mlp_loss_grad(const tk_mlp *w, const float *x9, const float *t6, long M, float *grad,
                            double *loss, void *stream);

/* One Adam update (Kingma & Ba) of opt->w from grad; increments opt->step and writes the
 * BF16-rounded (nearest, ties to even) parameters to w_bf16. */
tk_status sgs_adam_step(tk_adam *opt, const float *grad, uint16_t *w_bf16, void *stream);

/* BF16 (nearest, ties to even) copy of n FP32 values. */
tk_status sgs_weights_to_bf16(const float *w, uint16_t *w_bf16, int n, void *stream);

/* LES steps (FP32, IF-RK2, the solver's CFL or fixed dt): the right-hand side is
 * P M [F(u x omega) - i k_j F(tau_ij)] with tau = out_scale f(grad(u)/in_scale) evaluated
 * from the stage state on the grid.  w_or_null = NULL: plain DNS right-hand side.  If
 * the weights hold a non-finite value the steps run without the model (*fallback = 1);
 * if the state is not finite after the steps, it is restored and the steps are redone
 * without the model (*fallback = 2); else *fallback = 0 (fallback may be NULL).
 * Synchronises. */
tk_status les_step(tk_ns_t ns, const tk_mlp *w_or_null, void *uhat_inout, double dt, int nsteps,
                   double *t_inout, int *fallback, void *stream);

/* Training data from a DNS state uhat_dns [3][n_dns][n_dns][n_dns/2+1] (FP32, not
 * modified): box filter |k_i| <= kc (3 kc < n_les), truncated onto the n_les grid:
 * grad9 [9][n_les^3] = d_j ubar_i, tau6 [6][n_les^3] = G(u_i u_j) - G(ubar_i ubar_j) (the
 * stress the dealiased LES lacks: its own nonlinear term is G(ubar_i ubar_j)), the first
 * product formed on the DNS grid and the second on the LES grid, and optionally
 * ubar_hat [3][n_les][n_les][n_les/2+1].
 * Allocates and frees its own workspace (about 6 DNS fields).  Synchronises. */
tk_status les_filter_dns(const void *uhat_dns, int n_dns, int n_les, int kc, float *grad9, float *tau6,
                         void *ubar_hat, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TK_H */
