// Internal interface of the Navier-Stokes solver (shared by the single solver, the
// ensemble and the LES).
#pragma once

#include "fft_api.hpp"
#include "ns_kernels.hpp"

namespace tk {

constexpr int NS_DIAG_BLOCKS = 1024;
constexpr int NS_DIAG_HEAD = 4;
inline int ns_num_shells(int N) { return (int)(0.8660254037844386 * N) + 2; }

// Diagnostics into hout[0..NS_DIAG_HEAD+nshell): energy, enstrophy, max |k.u^|^2/|k|^2,
// max |u^|^2, E(s).
tk_status ns_diag_run(const void *u, int N, tk_dtype dt, int nshell, double *dscratch, double *hout, hipStream_t s);
tk_status ns_init_project(void *u, int N, tk_dtype dt, hipStream_t s);
tk_status ns_scale_shells(void *u, int N, tk_dtype dt, const double *fac_dev, int nshell, hipStream_t s);

// Everything one grid size needs to evaluate right-hand sides.
struct NsGrid {
    int n, K, KZC;
    int KZP;  // transit row length of the workspace fields (see ns_kzp)
    tk_dtype dt;
    FftAxes ax;
    const NsKernels *nk;
    int v1, v3, v5, v51;  // chosen variants of P1, P3, P5, fused P5+P1 (autotuner table, else 0)
    const StridedKernel *ky;  // Y passes P2 / P4 (autotuner table pass 6, else the transform's)
};
tk_status ns_grid_init(NsGrid *g, int n, tk_dtype dt);

// One right-hand side of input uin (3 fields) through P1..P5 with workspace w6 (6 fields);
// P5 combines according to `mode` (see NsMode); the stage buffers aux and ust are in the
// transit layout (uin_transit = 1 when uin is ust).  part != null (n^2 floats): P3 records
// max |u|_1 per workgroup and, when st_set != null, the step-size kernel reduces them
// after P3.  flags: NS_SKIP_P1 (w6 already holds P1's output for uin, uin unused),
// NS_FUSE_P1 (P5 runs fused with the next right-hand side's P1: w6 receives P1's output
// for the stage input instead of ust; not with NS_RHS).
enum : int { NS_SKIP_P1 = 1, NS_FUSE_P1 = 2 };
// ev (optional, 6 events): recorded before P1 and after each of P1..P5.
tk_status ns_rhs_eval(const NsGrid &g, const void *uin, void *w6, const P5Args &p5, float *part,
                      NsState *st_set, hipStream_t s, int uin_transit = 0, int flags = 0,
                      hipEvent_t *ev = nullptr);
// P1 alone (the first right-hand side of a run of fused ones).
tk_status ns_p1_only(const NsGrid &g, const void *uin, void *w6, hipStream_t s, int uin_transit = 0);

// Random solenoidal initial state from real noise [3][n][n][n] (see ns_init_random).
tk_status ns_init_random_grid(const NsGrid &g, const void *noise, void *u, double energy, double *dscratch,
                              hipStream_t s);

// Workspace of the learned-closure LES (allocated on first use by les_step).
struct LesWork {
    void *gsp = nullptr;   // 9 spectral gradient fields
    float *greal = nullptr;  // [9][n^3] gradients
    float *tau = nullptr;    // [6][n^3] stress
    void *tauh = nullptr;  // 6 spectral stress fields
    void *add3 = nullptr;  // 3 spectral fields: -i k_j tau^_ij
    void *backup = nullptr;  // 3 spectral fields: state at entry (fallback)
};

void les_work_free(LesWork &w);

}  // namespace tk

struct tk_ns_s {
    ns_config cfg;
    tk::NsGrid g;
    size_t fbytes;  // one spectral field
    void *w6 = nullptr, *aux = nullptr, *ust = nullptr;
    tk::NsState *st = nullptr;
    float *umax_part = nullptr;  // per-workgroup CFL maxima of P3 (n^2 floats)
    double *dscratch = nullptr;
    int nshell = 0;
    double last_dt = 0;
    tk::NsState hstage{};  // host staging copy of the step state (outlives async copies)
    tk::LesWork les;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    void *graph_u = nullptr;
};


