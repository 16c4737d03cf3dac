// Solver pass kernels (FP32 and FP64) for grid sizes 48,64,96,128,192.
#include "ns_kernels.hpp"

namespace tk {

void register_ns_b(std::vector<NsKernels> &v) {
    v.push_back(make_ns_kernels<float, 48>());
    v.push_back(make_ns_kernels<double, 48>());
    v.push_back(make_ns_kernels<float, 64>());
    v.push_back(make_ns_kernels<double, 64>());
    v.push_back(make_ns_kernels<float, 96>());
    v.push_back(make_ns_kernels<double, 96>());
    v.push_back(make_ns_kernels<float, 128>());
    v.push_back(make_ns_kernels<double, 128>());
    v.push_back(make_ns_kernels<float, 192>());
    v.push_back(make_ns_kernels<double, 192>());
}

}  // namespace tk
