// Diagnostic: the Z_p multiply-add of the DReLU/ReLU kernels (the field that
// with_field picks for l_x and p, in the operand representation the kernels
// keep their masks in: shifted to the top of the word for the stream draws
// up to N = 24, see MaskDraws), applied elementwise to arrays, so the arithmetic
// can be checked against exact integers at its bounds.
#include "drelu_kernel.h"

namespace bc {

template <int N, typename F>
__global__ __launch_bounds__(256) void k_zp_mul_add(const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                                    const uint64_t* __restrict__ d, uint64_t* out, uint64_t n,
                                                    F f_arg) {
    using FT = typename F::T;
    constexpr int SH = MaskDraws<N, F>::SH;
    const F f = f_arg.vgpr();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (uint64_t)field_mul_add<SH>(f, (FT)a[i], (FT)((FT)b[i] << SH), (FT)((FT)d[i] << SH));
}

template <int N>
hipError_t launch_zp_exact(const ZpLaunch& L, hipStream_t st) {
    return with_field<N>(L.p, [&](auto f) {
        hipLaunchKernelGGL((k_zp_mul_add<N, decltype(f)>), dim3(L.grid), dim3(256), 0, st, L.a, L.b, L.d, L.out, L.n,
                           f);
        return hipGetLastError();
    });
}

template <int NLO, int NHI>
hipError_t launch_zp_range(const ZpLaunch& L, hipStream_t st) {
    if constexpr (NLO > NHI) {
        return hipErrorInvalidValue;
    } else {
        if (L.npos == (uint32_t)NLO) return launch_zp_exact<NLO>(L, st);
        return launch_zp_range<NLO + 1, NHI>(L, st);
    }
}

hipError_t launch_zp_mul_add(const ZpLaunch& L, hipStream_t st) { return launch_zp_range<2, 33>(L, st); }

}  // namespace bc
