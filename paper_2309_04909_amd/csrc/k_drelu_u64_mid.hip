// Instantiations of the fused DReLU (Alg. 7) kernel for 64-bit share storage,
// one kernel per window count N = l_x + 1 in [13, 24].
#include "drelu_kernel.h"

namespace bc {

hipError_t launch_drelu_u64_mid(const DreluLaunch& L, hipStream_t st) {
    return launch_range<uint64_t, false, 13, 24>(L, st);
}

}  // namespace bc
