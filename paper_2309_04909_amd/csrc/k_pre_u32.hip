// Precomputed-randomness kernels (offline expansion and online DReLU/ReLU)
// for 32-bit share storage, one set per window count N in [2, 17].
#include "pre_kernel.h"

namespace bc {

hipError_t launch_pre_u32(const PreLaunch& L, hipStream_t st) { return launch_pre_range<uint32_t, 2, 17>(L, st); }

}  // namespace bc
