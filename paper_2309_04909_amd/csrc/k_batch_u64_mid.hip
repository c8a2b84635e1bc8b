// Persistent ragged-batch kernels for 64-bit share storage, one per
// window count N = l_x + 1 in [13, 24].
#include "batch_kernel.h"

namespace bc {

hipError_t launch_batch_u64_mid(const BatchLaunch& L, hipStream_t st) { return launch_batch_range<uint64_t, 13, 24>(L, st); }

}  // namespace bc
