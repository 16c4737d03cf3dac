// FP64 pass kernels for lengths 128,192,256,384,512,768,1024.
#include "fft_inst.hpp"

namespace tk {

void register_f64_b(std::vector<StridedKernel> &s, std::vector<ZKernel> &z) {
    add_all_f64<128>(s, z);
    add_all_f64<192>(s, z);
    add_all_f64<256>(s, z);
    add_all_f64<384>(s, z);
    add_all_f64<512>(s, z);
    add_all_f64<768>(s, z);
    add_all_f64<1024>(s, z);
}

}  // namespace tk
