// FP32 pass kernels for lengths 48,64,96,128,192.
#include "fft_inst.hpp"

namespace tk {

void register_f32_b(std::vector<StridedKernel> &s, std::vector<ZKernel> &z) {
    add_all_f32<48>(s, z);
    add_all_f32<64>(s, z);
    add_all_f32<96>(s, z);
    add_all_f32<128>(s, z);
    add_all_f32<192>(s, z);
}

}  // namespace tk
