// FP32 pass kernels for lengths 768.
#include "fft_inst.hpp"

namespace tk {

void register_f32_e(std::vector<StridedKernel> &s, std::vector<ZKernel> &z) {
    add_all_f32<768>(s, z);
}

}  // namespace tk
