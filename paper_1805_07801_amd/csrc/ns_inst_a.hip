// Solver pass kernels (FP32 and FP64) for grid sizes 8,12,16,24,32.
#include "ns_kernels.hpp"

namespace tk {

void register_ns_a(std::vector<NsKernels> &v) {
    v.push_back(make_ns_kernels<float, 8>());
    v.push_back(make_ns_kernels<double, 8>());
    v.push_back(make_ns_kernels<float, 12>());
    v.push_back(make_ns_kernels<double, 12>());
    v.push_back(make_ns_kernels<float, 16>());
    v.push_back(make_ns_kernels<double, 16>());
    v.push_back(make_ns_kernels<float, 24>());
    v.push_back(make_ns_kernels<double, 24>());
    v.push_back(make_ns_kernels<float, 32>());
    v.push_back(make_ns_kernels<double, 32>());
}

}  // namespace tk
