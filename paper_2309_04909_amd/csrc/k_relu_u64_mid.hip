// Instantiations of the fused ReLU (Alg. 8) kernel for 64-bit share storage,
// one kernel per window count N = l_x + 1 in [13, 24].
#include "drelu_kernel.h"

namespace bc {

hipError_t launch_relu_u64_mid(const DreluLaunch& L, hipStream_t st) {
    return launch_range<uint64_t, true, 13, 24>(L, st);
}

}  // namespace bc
