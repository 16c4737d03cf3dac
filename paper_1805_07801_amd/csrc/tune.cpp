// Autotuner cache (process-wide table; filled by fft3d_autotune or fft3d_tune_set).
#include <cmath>
#include <functional>
#include <map>
#include <mutex>
#include <tuple>

#include "tune.hpp"

namespace tk {

static std::mutex g_mu;
static std::map<std::tuple<int, int, int>, TileChoice> g_tiles;

TileChoice tuned_tile(int L, tk_dtype dt, int pass) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tiles.find(std::make_tuple(L, (int)dt, pass));
    return it == g_tiles.end() ? TileChoice{0, 0} : it->second;
}

void set_tuned_tile(int L, tk_dtype dt, int pass, TileChoice c) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tiles[std::make_tuple(L, (int)dt, pass)] = c;
}

void clear_tuned_tiles() {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tiles.clear();
}

}  // namespace tk

// ---- the autotuner ---------------------------------------------------------------------------
// For each pass of an (nx, ny, nz, dtype) grid, every compiled tile candidate is run on
// a pseudo-random field, timed with HIP events (median of `iters` launches), and
// admitted only if its output agrees with the default candidate's to within the
// dtype's transform tolerance (relative L2 1e-5 for FP32, 1e-12 for FP64).  The fastest
// admitted candidate is recorded in the in-process cache, which later plans consult.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fft_api.hpp"
#include "reduce.hpp"

namespace tk {

struct TuneBufs {
    void *a = nullptr, *b = nullptr, *ref = nullptr;
    ~TuneBufs() {
        if (a) hipFree(a);
        if (b) hipFree(b);
        if (ref) hipFree(ref);
    }
};

static tk_status time_it(const std::function<void()> &f, int iters, hipStream_t s, float *ms_out) {
    hipEvent_t e0, e1;
    TK_HIP_CHECK(hipEventCreate(&e0));
    TK_HIP_CHECK(hipEventCreate(&e1));
    std::vector<float> t;
    f();  // warm-up
    for (int i = 0; i < iters; ++i) {
        hipEventRecord(e0, s);
        f();
        hipEventRecord(e1, s);
        hipEventSynchronize(e1);
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        t.push_back(ms);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    std::sort(t.begin(), t.end());
    *ms_out = t[t.size() / 2];
    return launch_check("autotune candidate");
}

}  // namespace tk

using namespace tk;

extern "C" tk_status fft3d_autotune(int nx, int ny, int nz, int batch, tk_dtype dt, int iters, char *report,
                                    int report_len) {
    if (batch < 1 || iters < 1) return fail(TK_EINVAL, "batch and iters must be >= 1");
    FftAxes ax;
    TK_TRY(axes_init(&ax, nx, ny, nz, dt, false));
    const size_t esz = dt == TK_F32 ? 4 : 8;
    const long nzh = nz / 2 + 1;
    const long ncplx_reals = 2L * batch * nx * ny * nzh;
    const long nreal = (long)batch * nx * ny * nz;
    TuneBufs B;
    TK_HIP_CHECK(hipMalloc(&B.a, ncplx_reals * esz));
    TK_HIP_CHECK(hipMalloc(&B.b, ncplx_reals * esz));
    TK_HIP_CHECK(hipMalloc(&B.ref, ncplx_reals * esz));
    hipStream_t s = nullptr;
    const double tol = dt == TK_F32 ? 1e-5 : 1e-12;
    std::string rep;
    char line[256];
    for (int pass = 0; pass < 3; ++pass) {
        const int L = pass == 0 ? nz : pass == 1 ? ny : nx;
        // the input: a real field (Z pass) or a complex field (strided passes)
        TK_TRY(fill_pattern(B.a, pass == 0 ? nreal : ncplx_reals, dt, 1234u + pass, s));
        auto run_z = [&](const ZKernel *k, void *out) {
            ZArgs za{B.a, out, (long)batch * nx * ny, ax.twz, 1.0};
            k->r2c(za, s);
        };
        auto run_s = [&](const StridedKernel *k, void *out) {
            FftAxes a2 = ax;
            if (pass == 1) {
                a2.ky = k;
                fft_y_pass(a2, B.a, out, batch, 0, s);
            } else {
                a2.kx = k;
                fft_x_pass(a2, B.a, out, batch, 0, 1.0, s);
            }
        };
        const long nout = pass == 0 ? ncplx_reals : ncplx_reals;
        // reference output: the default candidate
        if (pass == 0) run_z(ax.kz, B.ref);
        else run_s(pass == 1 ? ax.ky : ax.kx, B.ref);
        TK_TRY(launch_check("autotune reference"));
        float best_ms = 1e30f;
        TileChoice best{0, 0};
        if (pass == 0) {
            for (const auto &k : z_kernels()) {
                if (k.N != L || k.dt != dt) continue;
                float ms;
                TK_TRY(time_it([&] { run_z(&k, B.b); }, iters, s, &ms));
                double num, den;
                TK_TRY(reduce_diff(B.b, B.ref, nout, dt, &num, &den, s));
                const bool ok = std::sqrt(num / den) <= tol;
                snprintf(line, sizeof(line), "pass z L=%d nt=%d E=%d lds=%d: %.4f ms %s\n", L, k.nt, k.E, k.lds, ms,
                         ok ? "ok" : "REJECTED");
                rep += line;
                if (ok && ms < best_ms) {
                    best_ms = ms;
                    best = {k.nt, k.E};
                }
            }
        } else {
            for (const auto &k : strided_kernels()) {
                if (k.L != L || k.dt != dt) continue;
                float ms;
                TK_TRY(time_it([&] { run_s(&k, B.b); }, iters, s, &ms));
                double num, den;
                TK_TRY(reduce_diff(B.b, B.ref, nout, dt, &num, &den, s));
                const bool ok = std::sqrt(num / den) <= tol;
                snprintf(line, sizeof(line), "pass %c L=%d W=%d E=%d nt=%d lds=%d: %.4f ms %s\n", pass == 1 ? 'y' : 'x',
                         L, k.W, k.E, k.nt, k.lds, ms, ok ? "ok" : "REJECTED");
                rep += line;
                if (ok && ms < best_ms) {
                    best_ms = ms;
                    best = {k.W, k.E};
                }
            }
        }
        if (best.a > 0) set_tuned_tile(L, dt, pass, best);
        snprintf(line, sizeof(line), "chosen pass %d L=%d: a=%d E=%d (%.4f ms)\n", pass, L, best.a, best.E, best_ms);
        rep += line;
    }
    if (report && report_len > 0) {
        strncpy(report, rep.c_str(), report_len - 1);
        report[report_len - 1] = 0;
    }
    return TK_OK;
}

extern "C" tk_status fft3d_tune_set(int L, tk_dtype dt, int pass, int a, int E) {
    if (pass < 0 || pass > 2) return fail(TK_EINVAL, "pass must be 0, 1 or 2");
    if (a <= 0) {
        set_tuned_tile(L, dt, pass, {0, 0});
        return TK_OK;
    }
    bool found = false;
    if (pass == 0) {
        for (const auto &k : z_kernels()) found |= (k.N == L && k.dt == dt && k.nt == a && k.E == E);
    } else {
        for (const auto &k : strided_kernels()) found |= (k.L == L && k.dt == dt && k.W == a && k.E == E);
    }
    if (!found) return fail(TK_EUNSUPPORTED, "no compiled tile L=%d pass=%d a=%d E=%d", L, pass, a, E);
    set_tuned_tile(L, dt, pass, {a, E});
    return TK_OK;
}

extern "C" tk_status fft3d_tune_clear(void) {
    clear_tuned_tiles();
    return TK_OK;
}

extern "C" int fft3d_tile_candidates(int L, tk_dtype dt, int pass, int *a, int *E, int cap) {
    int n = 0;
    if (pass == 0) {
        for (const auto &k : z_kernels())
            if (k.N == L && k.dt == dt) {
                if (n < cap && a && E) {
                    a[n] = k.nt;
                    E[n] = k.E;
                }
                ++n;
            }
    } else {
        for (const auto &k : strided_kernels())
            if (k.L == L && k.dt == dt) {
                if (n < cap && a && E) {
                    a[n] = k.W;
                    E[n] = k.E;
                }
                ++n;
            }
    }
    return n;
}
