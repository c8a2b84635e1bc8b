// P0's / P1's unflip of the parties-apart DReLU, for both storage widths.
#include "split_kernel.h"

namespace bc {

template <typename T>
static hipError_t launch_finish_t(const SplitLaunch& L, hipStream_t st) {
    const SplitKArgs A = make_split_kargs(L);
    if (L.party == 0)
        hipLaunchKernelGGL((k_finish<T, 0>), dim3(L.grid), dim3(256), 0, st, A);
    else
        hipLaunchKernelGGL((k_finish<T, 1>), dim3(L.grid), dim3(256), 0, st, A);
    return hipGetLastError();
}

hipError_t launch_split_finish(const SplitLaunch& L, hipStream_t st) {
    return L.ell > 32 ? launch_finish_t<uint64_t>(L, st) : launch_finish_t<uint32_t>(L, st);
}

}  // namespace bc
