// Instantiations of the fused DReLU (Alg. 7) kernel for 32-bit share storage,
// one kernel per window count N = l_x + 1 in [2, 17].
#include "drelu_kernel.h"

namespace bc {

hipError_t launch_drelu_u32(const DreluLaunch& L, hipStream_t st) {
    return launch_range<uint32_t, false, 2, 17>(L, st);
}

}  // namespace bc
