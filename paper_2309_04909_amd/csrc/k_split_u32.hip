// Instantiations of the parties-apart DReLU kernels (P0 / P1 send, P2 reply)
// for 32-bit share storage, one set per window count N = l_x + 1 in [2, 17].
#include "split_kernel.h"

namespace bc {

hipError_t launch_split_u32(const SplitLaunch& L, hipStream_t st) {
    return launch_split_range<uint32_t, 2, 17>(L, st);
}

}  // namespace bc
