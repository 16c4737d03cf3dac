// Rayleigh-Benard (Boussinesq) convection in the periodic FFF basis (paper, Section
// "Spectral Solver", eq:u_Usmall_Plarge and eq:T_Usmall_Plarge; Section "Scaling of RBC
// spectral solver": 13 transforms per right-hand side).  State [4][n][n][n/2+1]:
// u_x, u_y, u_z, theta.  The passes are the solver's with a temperature field carried
// along: P1 4 -> 7 fields (u, omega, theta), P2 Y-inverse of 7, P3 7 c2r -> u x omega
// and u theta -> 6 r2c, P4 Y-forward of 6, P5 X-forward with buoyancy, projection,
// -i a k . (u theta)^ + u_z and the IF-RK2 combine (viscosity sqrt(Pr/Ra) for u,
// diffusivity 1/sqrt(Ra Pr) for theta).
#include <cmath>
#include <new>

#include "ns_api.hpp"
#include "reduce.hpp"

namespace tk {

static constexpr int RB = 256;

// part[blk][0..3] = kinetic energy, thermal variance (1/2 <theta^2>), <u_z theta>, unused.
template <typename T>
__global__ __launch_bounds__(RB) void k_rbc_diag(const V2<T> *__restrict__ s4, int N, double *__restrict__ part) {
    __shared__ double sh[RB / 64];
    const int NZH = N / 2 + 1;
    const long FS = (long)N * N * NZH;
    double ke = 0, te = 0, fl = 0;
    for (long m = (long)blockIdx.x * RB + threadIdx.x; m < FS; m += (long)gridDim.x * RB) {
        const int kz = (int)(m % NZH);
        const double w = (kz == 0 || 2 * kz == N) ? 1.0 : 2.0;
        const V2<T> a = s4[m], b = s4[FS + m], c = s4[2 * FS + m], t = s4[3 * FS + m];
        ke += 0.5 * w * ((double)a.x * a.x + (double)a.y * a.y + (double)b.x * b.x + (double)b.y * b.y +
                         (double)c.x * c.x + (double)c.y * c.y);
        te += 0.5 * w * ((double)t.x * t.x + (double)t.y * t.y);
        fl += w * ((double)c.x * t.x + (double)c.y * t.y);
    }
    ke = block_sum(ke, sh);
    te = block_sum(te, sh);
    fl = block_sum(fl, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4] = ke;
        part[blockIdx.x * 4 + 1] = te;
        part[blockIdx.x * 4 + 2] = fl;
        part[blockIdx.x * 4 + 3] = 0;
    }
}

__global__ __launch_bounds__(RB) void k_rbc_diag_final(const double *__restrict__ part, int nb, double *__restrict__ out) {
    __shared__ double sh[RB / 64];
    const int i = blockIdx.x;
    double acc = 0;
    for (int b = threadIdx.x; b < nb; b += RB) acc += part[b * 4 + i];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) out[i] = acc;
}

}  // namespace tk

using namespace tk;

struct tk_rbc_s {
    rbc_config cfg;
    NsGrid g;
    size_t fbytes = 0;
    void *w7 = nullptr, *aux = nullptr, *ust = nullptr;
    NsState *st = nullptr;
    float *umax_part = nullptr;  // per-workgroup CFL maxima of P3 (n^2 floats)
    double *dscratch = nullptr;
    NsState hstage{};
    double nu_a = 0, kap_a = 0, ka = 1;
    double last_dt = 0;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    void *graph_u = nullptr;
};

static void rbc_free(tk_rbc_s *p) {
    if (p->gexec) hipGraphExecDestroy(p->gexec);
    if (p->graph) hipGraphDestroy(p->graph);
    void *ps[] = {p->w7, p->aux, p->ust, p->st, p->umax_part, p->dscratch};
    for (void *q : ps)
        if (q) hipFree(q);
    delete p;
}

// One right-hand side of uin (4 fields): P1..P5 with the stage combine `mode`.
// ev (optional, 6 events): recorded before P1 and after each pass.
static tk_status rbc_rhs_eval(tk_rbc_s *p, const void *uin, void *u, void *out, int mode, bool first_stage,
                              hipStream_t s, hipEvent_t *ev = nullptr) {
    const NsGrid &g = p->g;
    const int n = g.n;
    auto mark = [&](int i) -> tk_status {
        if (ev) TK_HIP_CHECK(hipEventRecord(ev[i], s));
        return TK_OK;
    };
    TK_TRY(mark(0));
    g.nk->p1r(uin, p->w7, g.K, g.KZC, g.ax.twx, p->ka, s);
    TK_TRY(launch_check("rbc P1"));
    TK_TRY(mark(1));
    StridedArgs y2{p->w7, p->w7, 7L * n * g.KZP, g.KZP, (long)n * g.KZP, g.KZP, g.ax.twy, 1, 1.0, g.K, -1};
    g.ky->fn(y2, s);
    TK_TRY(launch_check("rbc P2"));
    TK_TRY(mark(2));
    g.nk->p3r(p->w7, (long)n * n, g.KZC, g.ax.twz, first_stage ? p->umax_part : nullptr, s);
    TK_TRY(launch_check("rbc P3"));
    if (first_stage) {
        const int nparts = (int)cdiv((long)n * n, ns_z_LPW(n));
        hipLaunchKernelGGL(k_ns_set_h, dim3(1), dim3(1024), 0, s, p->st, p->umax_part, nparts);
        TK_TRY(launch_check("rbc step size"));
    }
    TK_TRY(mark(3));
    StridedArgs y4{p->w7, p->w7, 6L * n * g.KZP, g.KZP, (long)n * g.KZP, g.KZP, g.ax.twy, 0, 1.0, -1, g.K};
    g.ky->fn(y4, s);
    TK_TRY(launch_check("rbc P4"));
    TK_TRY(mark(4));
    g.nk->p5r(p->w7, uin, u, p->aux, p->ust, out, p->st, p->nu_a, p->kap_a, p->ka, mode, g.K, g.KZC, g.ax.twx, s);
    TK_TRY(launch_check("rbc P5"));
    return mark(5);
}

static tk_status rbc_one_step(tk_rbc_s *p, void *u, hipStream_t s) {
    TK_TRY(rbc_rhs_eval(p, u, u, nullptr, RK2_S1, true, s));
    return rbc_rhs_eval(p, p->ust, u, nullptr, RK2_S2, false, s);
}

extern "C" tk_status rbc_create(tk_rbc_t *out, const rbc_config *cfg) {
    if (!out || !cfg) return fail(TK_EINVAL, "NULL argument");
    *out = nullptr;
    if (!(cfg->Ra > 0) || !(cfg->Pr > 0) || !std::isfinite(cfg->Ra) || !std::isfinite(cfg->Pr))
        return fail(TK_EINVAL, "Ra and Pr must be finite and > 0");
    if (!(cfg->box > 0) || !std::isfinite(cfg->box)) return fail(TK_EINVAL, "box side must be > 0");
    if (cfg->cfl < 0 || !std::isfinite(cfg->cfl)) return fail(TK_EINVAL, "cfl must be finite and >= 0");
    if (!supported_len(cfg->n)) return fail(TK_EUNSUPPORTED, "unsupported n=%d", cfg->n);
    tk_rbc_s *p = new (std::nothrow) tk_rbc_s();
    if (!p) return fail(TK_ENOMEM, "host allocation failed");
    p->cfg = *cfg;
    tk_status st = ns_grid_init(&p->g, cfg->n, cfg->dtype);
    if (st != TK_OK) {
        delete p;
        return st;
    }
    const int n = cfg->n;
    p->ka = 2.0 * M_PI / cfg->box;
    p->nu_a = std::sqrt(cfg->Pr / cfg->Ra) * p->ka * p->ka;
    p->kap_a = 1.0 / std::sqrt(cfg->Ra * cfg->Pr) * p->ka * p->ka;
    p->fbytes = (size_t)n * n * (n / 2 + 1) * (cfg->dtype == TK_F32 ? 8 : 16);
    NsState h0{};
    if (hipMalloc(&p->w7, 7 * p->fbytes) != hipSuccess || hipMalloc(&p->aux, 4 * p->fbytes) != hipSuccess ||
        hipMalloc(&p->ust, 4 * p->fbytes) != hipSuccess || hipMalloc((void **)&p->st, sizeof(NsState)) != hipSuccess ||
        hipMalloc((void **)&p->umax_part, sizeof(float) * n * n) != hipSuccess ||
        hipMalloc((void **)&p->dscratch, sizeof(double) * 4 * (NS_DIAG_BLOCKS + 1)) != hipSuccess ||
        hipMemset(p->aux, 0, 4 * p->fbytes) != hipSuccess || hipMemset(p->ust, 0, 4 * p->fbytes) != hipSuccess ||
        hipMemset(p->w7, 0, 7 * p->fbytes) != hipSuccess ||
        hipMemcpy(p->st, &h0, sizeof(h0), hipMemcpyHostToDevice) != hipSuccess) {
        rbc_free(p);
        return fail(TK_ENOMEM, "convection solver workspace allocation failed");
    }
    *out = p;
    return TK_OK;
}

extern "C" tk_status rbc_rhs(tk_rbc_t p, const void *s4, void *rhs_out, void *stream) {
    if (!p || !s4 || !rhs_out) return fail(TK_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const long nvals = 4L * p->g.n * p->g.n * (p->g.n / 2 + 1);
    if (p->cfg.dtype == TK_F32) hipLaunchKernelGGL(k_zero<float2>, dim3(4096), dim3(256), 0, s, (float2 *)rhs_out, nvals);
    else hipLaunchKernelGGL(k_zero<double2>, dim3(4096), dim3(256), 0, s, (double2 *)rhs_out, nvals);
    TK_TRY(launch_check("zero rhs"));
    return rbc_rhs_eval(p, s4, const_cast<void *>(s4), rhs_out, NS_RHS, false, s);
}

extern "C" tk_status rbc_pass_times(tk_rbc_t p, const void *s4, int iters, float ms[5], void *stream) {
    if (!p || !s4 || !ms) return fail(TK_EINVAL, "NULL argument");
    if (iters < 1) return fail(TK_EINVAL, "iters must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev[6] = {};
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &f : ev)
                if (f) hipEventDestroy(f);
            return fail(TK_EHIP, "event creation failed");
        }
    double acc[5] = {0, 0, 0, 0, 0};
    tk_status st = TK_OK;
    for (int it = 0; it < iters && st == TK_OK; ++it) {
        // one right-hand side into the stage-input buffer; the state is only read
        st = rbc_rhs_eval(p, s4, const_cast<void *>(s4), p->ust, NS_RHS, false, s, ev);
        if (st == TK_OK && hipEventSynchronize(ev[5]) != hipSuccess) st = fail(TK_EHIP, "event synchronisation failed");
        for (int i = 0; i < 5 && st == TK_OK; ++i) {
            float t = 0;
            if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) st = fail(TK_EHIP, "event timing failed");
            acc[i] += t;
        }
    }
    for (auto &e : ev) hipEventDestroy(e);
    for (int i = 0; i < 5; ++i) ms[i] = (float)(acc[i] / iters);
    return st;
}

extern "C" tk_status rbc_step(tk_rbc_t p, void *u, double dt, int nsteps, double *t_inout, void *stream) {
    if (!p || !u) return fail(TK_EINVAL, "NULL argument");
    if (nsteps < 0) return fail(TK_EINVAL, "nsteps must be >= 0");
    if (p->cfg.cfl <= 0 && !(dt > 0 && std::isfinite(dt))) return fail(TK_EINVAL, "dt must be > 0 without CFL");
    hipStream_t s = (hipStream_t)stream;
    NsState &h0 = p->hstage;
    h0 = NsState{};
    h0.t = t_inout ? *t_inout : 0.0;
    h0.hfix = dt > 0 ? dt : 0.0;
    h0.cfl_dx = p->cfg.cfl > 0 ? p->cfg.cfl * p->cfg.box / p->cfg.n : 0.0;
    h0.h = h0.hfix;
    TK_HIP_CHECK(hipMemcpyAsync(p->st, &h0, sizeof(h0), hipMemcpyHostToDevice, s));
    if (nsteps > 0) {
        if (p->graph_u != u || !p->gexec) {
            if (p->gexec) hipGraphExecDestroy(p->gexec);
            if (p->graph) hipGraphDestroy(p->graph);
            p->gexec = nullptr;
            p->graph = nullptr;
            p->graph_u = nullptr;
            hipStream_t cs;
            TK_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            TK_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            tk_status st = rbc_one_step(p, u, cs);
            hipGraph_t gr = nullptr;
            hipError_t e = hipStreamEndCapture(cs, &gr);
            hipStreamDestroy(cs);
            if (st != TK_OK) {
                if (gr) hipGraphDestroy(gr);
                return st;
            }
            if (e != hipSuccess) return fail(TK_EHIP, "graph capture failed: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&p->gexec, gr, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                hipGraphDestroy(gr);
                return fail(TK_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
            }
            p->graph = gr;
            p->graph_u = u;
        }
        for (int i = 0; i < nsteps; ++i) TK_HIP_CHECK(hipGraphLaunch(p->gexec, s));
    }
    NsState hf{};
    TK_HIP_CHECK(hipMemcpyAsync(&hf, p->st, sizeof(hf), hipMemcpyDeviceToHost, s));
    TK_HIP_CHECK(hipStreamSynchronize(s));
    if (t_inout) *t_inout = hf.t;
    p->last_dt = hf.h;
    return TK_OK;
}

extern "C" tk_status rbc_diagnostics(tk_rbc_t p, const void *s4, double *kinetic, double *thermal, double *uz_theta,
                                     double *nusselt, void *stream) {
    if (!p || !s4) return fail(TK_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const int nb = NS_DIAG_BLOCKS;
    if (p->cfg.dtype == TK_F32)
        hipLaunchKernelGGL(k_rbc_diag<float>, dim3(nb), dim3(RB), 0, s, (const float2 *)s4, p->g.n, p->dscratch);
    else
        hipLaunchKernelGGL(k_rbc_diag<double>, dim3(nb), dim3(RB), 0, s, (const double2 *)s4, p->g.n, p->dscratch);
    TK_TRY(launch_check("rbc diagnostics"));
    double *o = p->dscratch + 4 * nb;
    hipLaunchKernelGGL(k_rbc_diag_final, dim3(3), dim3(RB), 0, s, p->dscratch, nb, o);
    TK_TRY(launch_check("rbc diagnostics final"));
    double h[3];
    TK_HIP_CHECK(hipMemcpyAsync(h, o, sizeof(h), hipMemcpyDeviceToHost, s));
    TK_HIP_CHECK(hipStreamSynchronize(s));
    if (kinetic) *kinetic = h[0];
    if (thermal) *thermal = h[1];
    if (uz_theta) *uz_theta = h[2];
    if (nusselt) *nusselt = 1.0 + std::sqrt(p->cfg.Ra * p->cfg.Pr) * h[2];
    if (!std::isfinite(h[0]) || !std::isfinite(h[1])) return fail(TK_ESTATE, "energy is not finite");
    return TK_OK;
}

extern "C" tk_status rbc_last_dt(tk_rbc_t p, double *dt) {
    if (!p || !dt) return fail(TK_EINVAL, "NULL argument");
    *dt = p->last_dt;
    return TK_OK;
}

extern "C" tk_status rbc_destroy(tk_rbc_t p) {
    if (p) rbc_free(p);
    return TK_OK;
}
