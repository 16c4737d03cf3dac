// Status text, twiddle tables and kernel registries.
#include <cmath>
#include <cstdarg>
#include <map>
#include <mutex>
#include <tuple>

#include "fft_kernels.hpp"

namespace tk {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}

tk_status fail(tk_status st, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

tk_status launch_check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TK_EHIP, "%s: launch failed: %s", what, hipGetErrorString(e));
    return TK_OK;
}

template <typename T> std::vector<V2<T>> twiddles_host(int n) {
    std::vector<V2<T>> w(n);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int j = 0; j < n; ++j) {
        // exact integer argument j/n; evaluate in long double, round once to T
        long double a = two_pi * (long double)j / (long double)n;
        w[j] = mk<T>((T)cosl(a), (T)(-sinl(a)));
    }
    return w;
}
template std::vector<V2<float>> twiddles_host<float>(int);
template std::vector<V2<double>> twiddles_host<double>(int);

const void *twiddle_table(int n, tk_dtype dt, tk_status *st) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int>, void *> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *st = fail(TK_EHIP, "hipGetDevice failed");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    auto key = std::make_tuple(dev, n, (int)dt);
    auto it = cache.find(key);
    if (it != cache.end()) {
        *st = TK_OK;
        return it->second;
    }
    void *p = nullptr;
    size_t bytes = (size_t)n * (dt == TK_F32 ? sizeof(float2) : sizeof(double2));
    if (hipMalloc(&p, bytes) != hipSuccess) {
        *st = fail(TK_ENOMEM, "twiddle table allocation failed");
        return nullptr;
    }
    hipError_t e;
    if (dt == TK_F32) {
        auto h = twiddles_host<float>(n);
        e = hipMemcpy(p, h.data(), bytes, hipMemcpyHostToDevice);
    } else {
        auto h = twiddles_host<double>(n);
        e = hipMemcpy(p, h.data(), bytes, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        hipFree(p);
        *st = fail(TK_EHIP, "twiddle upload failed: %s", hipGetErrorString(e));
        return nullptr;
    }
    cache[key] = p;
    *st = TK_OK;
    return p;
}

int resident_groups(const void *kernel, int nt) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void *, int>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    std::lock_guard<std::mutex> lk(mu);
    auto key = std::make_tuple(dev, kernel, nt);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    // a failed query (it has been seen to fail for kernels that use accumulation registers)
    // must not leave its error for the caller's next launch check: clear it and assume one
    // workgroup per CU, which any launchable kernel reaches
    int cus = 0, occ = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
        (void)hipGetLastError();
        cus = 256;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, nt, 0) != hipSuccess || occ < 1) {
        (void)hipGetLastError();
        occ = 1;
    }
    return cache[key] = occ * cus;
}

#define TK_REG(name) void name(std::vector<StridedKernel> &s, std::vector<ZKernel> &z);
TK_REG(register_f32_a) TK_REG(register_f32_b) TK_REG(register_f32_c) TK_REG(register_f32_d)
TK_REG(register_f32_e) TK_REG(register_f32_f) TK_REG(register_f64_a) TK_REG(register_f64_b)
#undef TK_REG

static void build_registry(std::vector<StridedKernel> *&s, std::vector<ZKernel> *&z) {
    static std::vector<StridedKernel> S;
    static std::vector<ZKernel> Z;
    static std::once_flag once;
    std::call_once(once, [] {
        register_f32_a(S, Z);
        register_f32_b(S, Z);
        register_f32_c(S, Z);
        register_f32_d(S, Z);
        register_f32_e(S, Z);
        register_f32_f(S, Z);
        register_f64_a(S, Z);
        register_f64_b(S, Z);
    });
    s = &S;
    z = &Z;
}

const std::vector<StridedKernel> &strided_kernels() {
    std::vector<StridedKernel> *s;
    std::vector<ZKernel> *z;
    build_registry(s, z);
    return *s;
}

const std::vector<ZKernel> &z_kernels() {
    std::vector<StridedKernel> *s;
    std::vector<ZKernel> *z;
    build_registry(s, z);
    return *z;
}

}  // namespace tk

extern "C" const char *tk_last_error(void) { return tk::g_err.c_str(); }
extern "C" int tk_version(void) { return 10000; }
