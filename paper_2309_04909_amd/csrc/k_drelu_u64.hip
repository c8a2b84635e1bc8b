// Instantiations of the fused DReLU (Alg. 7) kernel for 64-bit share storage
// (rings of 33..64 bits), one per window-count bucket.
#include "drelu_kernel.h"

namespace bc {

hipError_t launch_drelu_u64(const DreluLaunch& L, hipStream_t st) {
    constexpr bool RELU = false;
    using T = uint64_t;
    const uint32_t n = L.npos;
    if (n <= 8) return launch_bucket<T, 8, FieldSmall, RELU>(L, make_field_small(L.p), st);
    if (n <= 12) return launch_bucket<T, 12, FieldSmall, RELU>(L, make_field_small(L.p), st);
    if (n <= 16) return launch_bucket<T, 16, Field24, RELU>(L, make_field24(L.p), st);
    if (n <= 20) return launch_bucket<T, 20, Field24, RELU>(L, make_field24(L.p), st);
    if (n <= 24) return launch_bucket<T, 24, Field24, RELU>(L, make_field24(L.p), st);
    if (n <= 32) return launch_bucket<T, 32, Field32, RELU>(L, make_field32(L.p), st);
    if (n <= 33) return launch_bucket<T, 33, Field64, RELU>(L, make_field64(L.p), st);
    return hipErrorInvalidValue;
}

}  // namespace bc
