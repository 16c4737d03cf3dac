// Solver pass kernels (FP32 and FP64) for grid sizes 256,384,512,768,1024.
#include "ns_kernels.hpp"

namespace tk {

void register_ns_c(std::vector<NsKernels> &v) {
    v.push_back(make_ns_kernels<float, 256>());
    v.push_back(make_ns_kernels<double, 256>());
    v.push_back(make_ns_kernels<float, 384>());
    v.push_back(make_ns_kernels<double, 384>());
    v.push_back(make_ns_kernels<float, 512>());
    v.push_back(make_ns_kernels<double, 512>());
    v.push_back(make_ns_kernels<float, 768>());
    v.push_back(make_ns_kernels<double, 768>());
    v.push_back(make_ns_kernels<float, 1024>());
    v.push_back(make_ns_kernels<double, 1024>());
}

}  // namespace tk
