// Precomputed-randomness kernels (offline expansion and online DReLU/ReLU)
// for 64-bit share storage, one set per window count N in [25, 33].
#include "pre_kernel.h"

namespace bc {

hipError_t launch_pre_u64_hi(const PreLaunch& L, hipStream_t st) { return launch_pre_range<uint64_t, 25, 33>(L, st); }

}  // namespace bc
