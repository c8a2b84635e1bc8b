// Instantiations of the fused ReLU (Alg. 8) kernel for 32-bit share storage
// (rings of 1..32 bits), one per window-count bucket.
#include "drelu_kernel.h"

namespace bc {

hipError_t launch_relu_u32(const DreluLaunch& L, hipStream_t st) {
    constexpr bool RELU = true;
    using T = uint32_t;
    const uint32_t n = L.npos;
    if (n <= 8) return launch_bucket<T, 8, FieldSmall, RELU>(L, make_field_small(L.p), st);
    if (n <= 12) return launch_bucket<T, 12, FieldSmall, RELU>(L, make_field_small(L.p), st);
    if (n <= 16) return launch_bucket<T, 16, Field24, RELU>(L, make_field24(L.p), st);
    if (n <= 20) return launch_bucket<T, 20, Field24, RELU>(L, make_field24(L.p), st);
    return hipErrorInvalidValue;
}

}  // namespace bc
