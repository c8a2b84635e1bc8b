// Instantiations of the replicated-sharing DReLU / ReLU kernel (Alg. drelu2)
// for 32-bit share storage, one kernel per window count N = l_x + 1 in
// [2, 17].
#include "rss_kernel.h"

namespace bc {

hipError_t launch_rss_u32(const RssLaunch& L, hipStream_t st) {
    return launch_rss_range<uint32_t, 2, 17>(L, st);
}

}  // namespace bc
