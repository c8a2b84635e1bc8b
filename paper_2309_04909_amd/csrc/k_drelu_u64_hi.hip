// Instantiations of the fused DReLU (Alg. 7) kernel for 64-bit share storage,
// one kernel per window count N = l_x + 1 in [25, 33].
#include "drelu_kernel.h"

namespace bc {

hipError_t launch_drelu_u64_hi(const DreluLaunch& L, hipStream_t st) {
    return launch_range<uint64_t, false, 25, 33>(L, st);
}

}  // namespace bc
