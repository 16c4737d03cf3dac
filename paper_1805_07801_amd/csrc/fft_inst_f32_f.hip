// FP32 pass kernels for lengths 1024.
#include "fft_inst.hpp"

namespace tk {

void register_f32_f(std::vector<StridedKernel> &s, std::vector<ZKernel> &z) {
    add_all_f32<1024>(s, z);
}

}  // namespace tk
