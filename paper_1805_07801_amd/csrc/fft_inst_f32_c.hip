// FP32 pass kernels for lengths 256,384.
#include "fft_inst.hpp"

namespace tk {

void register_f32_c(std::vector<StridedKernel> &s, std::vector<ZKernel> &z) {
    add_all_f32<256>(s, z);
    add_all_f32<384>(s, z);
}

}  // namespace tk
