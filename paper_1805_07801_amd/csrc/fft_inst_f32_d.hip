// FP32 pass kernels for lengths 512.
#include "fft_inst.hpp"

namespace tk {

void register_f32_d(std::vector<StridedKernel> &s, std::vector<ZKernel> &z) {
    add_all_f32<512>(s, z);
}

}  // namespace tk
