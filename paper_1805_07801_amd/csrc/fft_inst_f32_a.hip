// FP32 pass kernels for lengths 8,12,16,24,32.
#include "fft_inst.hpp"

namespace tk {

void register_f32_a(std::vector<StridedKernel> &s, std::vector<ZKernel> &z) {
    add_all_f32<8>(s, z);
    add_all_f32<12>(s, z);
    add_all_f32<16>(s, z);
    add_all_f32<24>(s, z);
    add_all_f32<32>(s, z);
}

}  // namespace tk
