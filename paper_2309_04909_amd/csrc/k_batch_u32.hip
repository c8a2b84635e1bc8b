// Persistent ragged-batch kernels for 32-bit share storage, one per
// window count N = l_x + 1 in [2, 17].
#include "batch_kernel.h"

namespace bc {

hipError_t launch_batch_u32(const BatchLaunch& L, hipStream_t st) { return launch_batch_range<uint32_t, 2, 17>(L, st); }

}  // namespace bc
