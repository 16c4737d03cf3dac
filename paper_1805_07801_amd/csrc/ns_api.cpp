// Navier-Stokes solver handle: workspace, right-hand sides, IF-RK2 / IF-RK4 steps (one
// step captured once as a HIP graph and replayed), diagnostics and the random initial
// field.  Paper, Section "Spectral Solver" (eq:NSk, eq:continuity2) and Section "Scaling
// of Fluid spectral solver" (fourth-order Runge-Kutta, 2/3 rule, nine transforms per
// right-hand side).
#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>

#include "ns_api.hpp"
#include "tune.hpp"

namespace tk {

void register_ns_a(std::vector<NsKernels> &v);
void register_ns_b(std::vector<NsKernels> &v);
void register_ns_c(std::vector<NsKernels> &v);

const std::vector<NsKernels> &ns_kernels() {
    static std::vector<NsKernels> K;
    static std::once_flag once;
    std::call_once(once, [] {
        register_ns_a(K);
        register_ns_b(K);
        register_ns_c(K);
    });
    return K;
}

tk_status ns_grid_init(NsGrid *g, int n, tk_dtype dt) {
    TK_TRY(axes_init(&g->ax, n, n, n, dt, true));
    g->n = n;
    g->dt = dt;
    g->K = (n - 1) / 3;
    g->KZC = g->K + 1;
    g->KZP = std::min((g->KZC + 15) / 16 * 16, n / 2 + 1);  // = ns_kzp<n>()
    g->nk = nullptr;
    for (const auto &k : ns_kernels())
        if (k.N == n && k.dt == dt) g->nk = &k;
    if (!g->nk) return fail(TK_EUNSUPPORTED, "no solver kernels for n=%d", n);
    auto pick = [&](int pass, auto *v, int nv) {
        const TileChoice c = tuned_tile(n, dt, pass);
        for (int i = 0; i < nv; ++i)
            if (v[i].a == c.a && v[i].E == c.E && v[i].v == c.v) return i;
        return 0;
    };
    g->v1 = pick(3, g->nk->p1v, g->nk->np1);
    g->v3 = pick(4, g->nk->p3v, g->nk->np3);
    g->v5 = pick(5, g->nk->p5v, g->nk->np5);
    g->v51 = pick(7, g->nk->p51v, g->nk->np51);
    const TileChoice cy = tuned_tile(n, dt, 6);
    g->ky = cy.a > 0 ? pick_strided(n, dt, cy.a, cy.E, cy.v) : nullptr;
    if (!g->ky) g->ky = g->ax.ky;
    return TK_OK;
}

tk_status ns_p1_only(const NsGrid &g, const void *uin, void *w6, hipStream_t s, int uin_transit) {
    g.nk->p1v[g.v1].fn(uin, w6, g.K, uin_transit, g.ax.twx, s);
    return launch_check("ns P1");
}

tk_status ns_rhs_eval(const NsGrid &g, const void *uin, void *w6, const P5Args &p5, float *part,
                      NsState *st_set, hipStream_t s, int uin_transit, int flags, hipEvent_t *ev) {
    const int n = g.n;
    auto mark = [&](int i) -> tk_status {
        if (ev) TK_HIP_CHECK(hipEventRecord(ev[i], s));
        return TK_OK;
    };
    TK_TRY(mark(0));
    // P1: x-inverse of u^ and omega^ = i k x u^
    if (!(flags & NS_SKIP_P1)) TK_TRY(ns_p1_only(g, uin, w6, s, uin_transit));
    TK_TRY(mark(1));
    // P2: y-inverse of the 6 fields, kept kz columns, kept ky rows read
    StridedArgs y2{w6, w6, 6L * n * g.KZP, g.KZP, (long)n * g.KZP, g.KZP, g.ax.twy, 1, 1.0, g.K, -1};
    g.ky->fn(y2, s);
    TK_TRY(launch_check("ns P2"));
    TK_TRY(mark(2));
    // P3: z fused c2r -> u x omega -> r2c
    g.nk->p3v[g.v3].fn(w6, (long)n * n, g.KZC, g.ax.twz, part, s);
    TK_TRY(launch_check("ns P3"));
    if (st_set) {
        const int nparts = (int)cdiv((long)n * n, g.nk->p3v[g.v3].a);
        hipLaunchKernelGGL(k_ns_set_h, dim3(1), dim3(1024), 0, s, st_set, part, nparts);
        TK_TRY(launch_check("ns step size"));
    }
    TK_TRY(mark(3));
    // P4: y-forward of the 3 products, kept ky rows written
    StridedArgs y4{w6, w6, 3L * n * g.KZP, g.KZP, (long)n * g.KZP, g.KZP, g.ax.twy, 0, 1.0, -1, g.K};
    g.ky->fn(y4, s);
    TK_TRY(launch_check("ns P4"));
    TK_TRY(mark(4));
    // P5: x-forward, projection, stage combine (and the next P1)
    P5Args a = p5;
    a.c3 = w6;
    if (flags & NS_FUSE_P1) {
        if (p5.mode == NS_RHS || g.nk->np51 == 0) return fail(TK_EINVAL, "no fused P5 for this right-hand side");
        g.nk->p51v[g.v51].fn(a, g.K, g.KZC, g.ax.twx, s);
        TK_TRY(launch_check("ns P5+P1"));
    } else {
        g.nk->p5v[g.v5].fn(a, g.K, g.KZC, g.ax.twx, s);
        TK_TRY(launch_check("ns P5"));
    }
    return mark(5);
}

// Random solenoidal initial state: r2c of the noise, projection, 2/3 mask and k = 0
// removed, each shell s >= 1 rescaled to s^4 exp(-2 (s/4)^2), total energy `energy`.
tk_status ns_init_random_grid(const NsGrid &g, const void *noise, void *u, double energy, double *dscratch,
                              hipStream_t s) {
    const int n = g.n;
    const int nshell = ns_num_shells(n);
    TK_TRY(fft_z_r2c(g.ax, noise, u, 3, 1.0, s));
    TK_TRY(fft_y_pass(g.ax, u, u, 3, 0, s));
    TK_TRY(fft_x_pass(g.ax, u, u, 3, 0, 1.0 / ((double)n * n * n), s));
    TK_TRY(ns_init_project(u, n, g.dt, s));
    std::vector<double> h(NS_DIAG_HEAD + nshell);
    TK_TRY(ns_diag_run(u, n, g.dt, nshell, dscratch, h.data(), s));
    std::vector<double> fac(nshell, 0.0);
    double total = 0;
    for (int sh = 1; sh < nshell; ++sh) {
        const double es = h[NS_DIAG_HEAD + sh];
        if (es > 0) {
            const double et = std::pow((double)sh, 4) * std::exp(-2.0 * (sh / 4.0) * (sh / 4.0));
            fac[sh] = std::sqrt(et / es);
            total += et;
        }
    }
    if (!(total > 0)) return fail(TK_ESTATE, "noise field has no energy in the kept shells");
    const double g2 = std::sqrt(energy / total);
    for (auto &f : fac) f *= g2;
    TK_HIP_CHECK(hipMemcpyAsync(dscratch, fac.data(), sizeof(double) * nshell, hipMemcpyHostToDevice, s));
    TK_TRY(ns_scale_shells(u, n, g.dt, dscratch, nshell, s));
    TK_HIP_CHECK(hipStreamSynchronize(s));
    return TK_OK;
}

}  // namespace tk

using namespace tk;

static void ns_free(tk_ns_s *p) {
    les_work_free(p->les);
    if (p->gexec) hipGraphExecDestroy(p->gexec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->w6) hipFree(p->w6);
    if (p->aux) hipFree(p->aux);
    if (p->ust) hipFree(p->ust);
    if (p->st) hipFree(p->st);
    if (p->umax_part) hipFree(p->umax_part);
    if (p->dscratch) hipFree(p->dscratch);
    delete p;
}

extern "C" tk_status ns_create(tk_ns_t *out, const ns_config *cfg) {
    if (!out || !cfg) return fail(TK_EINVAL, "NULL argument");
    *out = nullptr;
    if (cfg->nu < 0 || !std::isfinite(cfg->nu)) return fail(TK_EINVAL, "nu must be finite and >= 0");
    if (cfg->cfl < 0 || !std::isfinite(cfg->cfl)) return fail(TK_EINVAL, "cfl must be finite and >= 0");
    if (cfg->scheme != 0 && cfg->scheme != 1) return fail(TK_EUNSUPPORTED, "scheme must be 0 (RK2) or 1 (RK4)");
    if (!supported_len(cfg->n)) return fail(TK_EUNSUPPORTED, "unsupported n=%d", cfg->n);
    tk_ns_s *p = new (std::nothrow) tk_ns_s();
    if (!p) return fail(TK_ENOMEM, "host allocation failed");
    p->cfg = *cfg;
    tk_status st = ns_grid_init(&p->g, cfg->n, cfg->dtype);
    if (st != TK_OK) {
        delete p;
        return st;
    }
    const int n = cfg->n;
    p->fbytes = (size_t)n * n * (n / 2 + 1) * (cfg->dtype == TK_F32 ? 8 : 16);
    p->nshell = ns_num_shells(n);
    const size_t dbytes = sizeof(double) * ((size_t)(NS_DIAG_BLOCKS + 2) * (NS_DIAG_HEAD + p->nshell));
    if (hipMalloc(&p->w6, 6 * p->fbytes) != hipSuccess || hipMalloc(&p->aux, 3 * p->fbytes) != hipSuccess ||
        hipMalloc(&p->ust, 3 * p->fbytes) != hipSuccess || hipMalloc((void **)&p->st, sizeof(NsState)) != hipSuccess ||
        hipMalloc((void **)&p->umax_part, sizeof(float) * cfg->n * cfg->n) != hipSuccess ||
        hipMalloc((void **)&p->dscratch, dbytes) != hipSuccess) {
        ns_free(p);
        return fail(TK_ENOMEM, "solver workspace allocation (%zu bytes) failed", 12 * p->fbytes);
    }
    NsState h0{};
    // stage buffers start at zero: passes write only the 2/3-rule modes
    if (hipMemset(p->aux, 0, 3 * p->fbytes) != hipSuccess || hipMemset(p->ust, 0, 3 * p->fbytes) != hipSuccess ||
        hipMemset(p->w6, 0, 6 * p->fbytes) != hipSuccess ||
        hipMemcpy(p->st, &h0, sizeof(h0), hipMemcpyHostToDevice) != hipSuccess) {
        ns_free(p);
        return fail(TK_EHIP, "state upload failed");
    }
    *out = p;
    return TK_OK;
}

// One step with every P5 fused with the P1 after it: on entry w6 holds P1's output for the
// state u (ns_p1_only before the first step), on exit P1's output for the new state.
static tk_status ns_one_step(tk_ns_s *p, void *u, hipStream_t s) {
    const NsGrid &g = p->g;
    P5Args a{};
    a.u = u;
    a.aux = p->aux;
    a.ust = p->ust;
    a.st = p->st;
    a.nu = p->cfg.nu;
    const int fl = NS_SKIP_P1 | NS_FUSE_P1;
    a.mode = p->cfg.scheme == 0 ? RK2_S1 : RK4_S1;
    TK_TRY(ns_rhs_eval(g, u, p->w6, a, p->umax_part, p->st, s, 0, fl));
    const int last = p->cfg.scheme == 0 ? RK2_S2 : RK4_S4;
    for (int m = a.mode + 1; m <= last; ++m) {
        a.mode = m;
        TK_TRY(ns_rhs_eval(g, nullptr, p->w6, a, nullptr, nullptr, s, 1, fl));
    }
    return TK_OK;
}

extern "C" tk_status ns_rhs(tk_ns_t p, const void *uhat, void *rhs_out, void *stream) {
    if (!p || !uhat || !rhs_out) return fail(TK_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const long nvals = 3L * p->g.n * p->g.n * (p->g.n / 2 + 1);
    if (p->cfg.dtype == TK_F32) hipLaunchKernelGGL(k_zero<float2>, dim3(4096), dim3(256), 0, s, (float2 *)rhs_out, nvals);
    else hipLaunchKernelGGL(k_zero<double2>, dim3(4096), dim3(256), 0, s, (double2 *)rhs_out, nvals);
    TK_TRY(launch_check("zero rhs"));
    P5Args a{};
    a.u = const_cast<void *>(uhat);
    a.out = rhs_out;
    a.st = p->st;
    a.nu = p->cfg.nu;
    a.mode = NS_RHS;
    return ns_rhs_eval(p->g, uhat, p->w6, a, nullptr, nullptr, s);
}

extern "C" tk_status ns_step(tk_ns_t p, void *u, double dt, int nsteps, double *t_inout, void *stream) {
    if (!p || !u) return fail(TK_EINVAL, "NULL argument");
    if (nsteps < 0) return fail(TK_EINVAL, "nsteps must be >= 0");
    if (p->cfg.cfl <= 0 && !(dt > 0 && std::isfinite(dt))) return fail(TK_EINVAL, "dt must be > 0 without CFL");
    hipStream_t s = (hipStream_t)stream;
    NsState &h0 = p->hstage;
    h0 = NsState{};
    h0.t = t_inout ? *t_inout : 0.0;
    h0.hfix = dt > 0 ? dt : 0.0;
    h0.cfl_dx = p->cfg.cfl > 0 ? p->cfg.cfl * 2.0 * M_PI / p->cfg.n : 0.0;
    h0.h = h0.hfix;
    TK_HIP_CHECK(hipMemcpyAsync(p->st, &h0, sizeof(h0), hipMemcpyHostToDevice, s));
    if (nsteps > 0) {
        // one step as a graph, captured once per state buffer and replayed
        if (p->graph_u != u || !p->gexec) {
            if (p->gexec) hipGraphExecDestroy(p->gexec);
            if (p->graph) hipGraphDestroy(p->graph);
            p->gexec = nullptr;
            p->graph = nullptr;
            p->graph_u = nullptr;
            hipStream_t cs;
            TK_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            TK_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            tk_status st = ns_one_step(p, u, cs);
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
        TK_TRY(ns_p1_only(p->g, u, p->w6, s));
        for (int i = 0; i < nsteps; ++i) TK_HIP_CHECK(hipGraphLaunch(p->gexec, s));
    }
    NsState hf{};
    TK_HIP_CHECK(hipMemcpyAsync(&hf, p->st, sizeof(hf), hipMemcpyDeviceToHost, s));
    TK_HIP_CHECK(hipStreamSynchronize(s));
    if (t_inout) *t_inout = hf.t;
    p->last_dt = hf.h;
    return TK_OK;
}

extern "C" tk_status ns_pass_times(tk_ns_t p, const void *uhat, int iters, float ms[6], void *stream) {
    if (!p || !uhat || !ms) return fail(TK_EINVAL, "NULL argument");
    if (iters < 1) return fail(TK_EINVAL, "iters must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    const NsGrid &g = p->g;
    hipEvent_t ev[8] = {};
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &f : ev)
                if (f) hipEventDestroy(f);
            return fail(TK_EHIP, "event creation failed");
        }
    double acc[6] = {0, 0, 0, 0, 0, 0};
    tk_status st = TK_OK;
    for (int it = 0; it < iters && st == TK_OK; ++it) {
        // one right-hand side (P5 writes its result into the stage-input buffer)
        P5Args a{};
        a.u = const_cast<void *>(uhat);
        a.out = p->ust;
        a.st = p->st;
        a.nu = p->cfg.nu;
        a.mode = NS_RHS;
        st = ns_rhs_eval(g, uhat, p->w6, a, nullptr, nullptr, s, 0, 0, ev);
        // the fused pass in its first-stage form: reads the workspace and u, writes aux
        // and the workspace
        if (st == TK_OK && g.nk->np51 > 0) {
            P5Args b = a;
            b.c3 = p->w6;
            b.aux = p->aux;
            b.mode = RK2_S1;
            if (hipEventRecord(ev[6], s) != hipSuccess) st = fail(TK_EHIP, "event record failed");
            g.nk->p51v[g.v51].fn(b, g.K, g.KZC, g.ax.twx, s);
            if (st == TK_OK) st = launch_check("ns P5+P1");
            if (st == TK_OK && hipEventRecord(ev[7], s) != hipSuccess) st = fail(TK_EHIP, "event record failed");
        }
        if (st == TK_OK && hipEventSynchronize(ev[g.nk->np51 > 0 ? 7 : 5]) != hipSuccess)
            st = fail(TK_EHIP, "event synchronisation failed");
        for (int i = 0; i < 5 && st == TK_OK; ++i) {
            float t = 0;
            if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) st = fail(TK_EHIP, "event timing failed");
            acc[i] += t;
        }
        if (st == TK_OK && g.nk->np51 > 0) {
            float t = 0;
            if (hipEventElapsedTime(&t, ev[6], ev[7]) != hipSuccess) st = fail(TK_EHIP, "event timing failed");
            acc[5] += t;
        }
    }
    for (auto &e : ev) hipEventDestroy(e);
    TK_TRY(st);
    for (int i = 0; i < 6; ++i) ms[i] = (float)(acc[i] / iters);
    return TK_OK;
}

extern "C" tk_status ns_last_dt(tk_ns_t p, double *dt) {
    if (!p || !dt) return fail(TK_EINVAL, "NULL argument");
    *dt = p->last_dt;
    return TK_OK;
}

extern "C" tk_status ns_diagnostics(tk_ns_t p, const void *u, double *energy, double *dissipation, double *spectrum,
                                    int nshell, double *max_div, void *stream) {
    if (!p || !u) return fail(TK_EINVAL, "NULL argument");
    if (nshell < 0 || (nshell > 0 && !spectrum)) return fail(TK_EINVAL, "bad spectrum arguments");
    std::vector<double> h(NS_DIAG_HEAD + p->nshell);
    TK_TRY(ns_diag_run(u, p->g.n, p->cfg.dtype, p->nshell, p->dscratch, h.data(), (hipStream_t)stream));
    if (energy) *energy = h[0];
    if (dissipation) *dissipation = 2.0 * p->cfg.nu * h[1];
    if (max_div) *max_div = h[3] > 0 ? std::sqrt(h[2] / h[3]) : 0.0;
    for (int i = 0; i < nshell; ++i) spectrum[i] = i < p->nshell ? h[NS_DIAG_HEAD + i] : 0.0;
    if (!std::isfinite(h[0])) return fail(TK_ESTATE, "energy is not finite");
    return TK_OK;
}

extern "C" tk_status ns_init_random(tk_ns_t p, const void *noise, void *u, double energy, void *stream) {
    if (!p || !noise || !u) return fail(TK_EINVAL, "NULL argument");
    if (!(energy > 0) || !std::isfinite(energy)) return fail(TK_EINVAL, "energy must be > 0");
    return ns_init_random_grid(p->g, noise, u, energy, p->dscratch, (hipStream_t)stream);
}

extern "C" tk_status ns_destroy(tk_ns_t p) {
    if (p) ns_free(p);
    return TK_OK;
}
