// Autotuner cache (filled by fft3d_autotune; see tk.h).
#include <map>
#include <mutex>
#include <tuple>

#include "tune.hpp"

namespace tk {

static std::mutex g_mu;
static std::map<std::tuple<int, int, int>, int> g_width;

int tuned_width(int L, tk_dtype dt, int pass) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_width.find(std::make_tuple(L, (int)dt, pass));
    return it == g_width.end() ? 0 : it->second;
}

void set_tuned_width(int L, tk_dtype dt, int pass, int W) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_width[std::make_tuple(L, (int)dt, pass)] = W;
}

}  // namespace tk
