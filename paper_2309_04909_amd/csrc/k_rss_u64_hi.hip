// Instantiations of the replicated-sharing DReLU / ReLU kernel (Alg. drelu2)
// for 64-bit share storage, one kernel per window count N = l_x + 1 in
// [25, 33].
#include "rss_kernel.h"

namespace bc {

hipError_t launch_rss_u64_hi(const RssLaunch& L, hipStream_t st) {
    return launch_rss_range<uint64_t, 25, 33>(L, st);
}

}  // namespace bc
