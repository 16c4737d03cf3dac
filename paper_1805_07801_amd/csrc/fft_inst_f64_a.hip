// FP64 pass kernels for lengths 8,12,16,24,32,48,64,96.
#include "fft_inst.hpp"

namespace tk {

void register_f64_a(std::vector<StridedKernel> &s, std::vector<ZKernel> &z) {
    add_all_f64<8>(s, z);
    add_all_f64<12>(s, z);
    add_all_f64<16>(s, z);
    add_all_f64<24>(s, z);
    add_all_f64<32>(s, z);
    add_all_f64<48>(s, z);
    add_all_f64<64>(s, z);
    add_all_f64<96>(s, z);
}

}  // namespace tk
