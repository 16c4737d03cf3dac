// FP32 instantiations of the pass kernels.
#include "fft_inst.hpp"

namespace tk {

void register_f32(std::vector<StridedKernel> &s, std::vector<ZKernel> &z) {
#define TK_S(L) add_strided<float, L, 0>(s); add_strided<float, L, 1>(s); add_strided<float, L, 2>(s);
#define TK_Z(L) add_z<float, L>(z);
    TK_FOR_EACH_LEN(TK_S)
    TK_FOR_EACH_LEN(TK_Z)
#undef TK_S
#undef TK_Z
}

}  // namespace tk
