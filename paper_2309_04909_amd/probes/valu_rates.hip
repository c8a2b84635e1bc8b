// VALU issue-rate probe for gfx950: one instruction kind per kernel, eight
// independent dependency chains per lane, 4096 blocks of 256 threads, so the
// SIMDs are issue-bound.  Prints lane-operations per second for each kind;
// the ALU roofline of the DReLU/ReLU kernels is discussed against these.
//
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         paper_2309_04909_amd/probes/valu_rates.hip -o /tmp/valu_rates && /tmp/valu_rates
//
// Every kernel writes only out[global thread id] (grid * 256 words, all allocated).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#define CHK(x)                                                                    \
    do {                                                                          \
        hipError_t e_ = (x);                                                      \
        if (e_ != hipSuccess) {                                                   \
            printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                             \
        }                                                                         \
    } while (0)

#define REP8(S) S(0) S(1) S(2) S(3) S(4) S(5) S(6) S(7)

// 32-bit chains a0..a7, 64-bit chains q0..q7, fp64 chains d0..d7.  b is a
// per-lane operand, bs a uniform (SGPR) operand, m a uniform lane mask.
#define K_XOR(k) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a##k) : "v"(b));
#define K_XOR_S(k) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a##k) : "s"(bs));
#define K_ADD(k) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a##k) : "v"(b));
#define K_ADD_C(k) asm volatile("v_add_u32 %0, 5, %0" : "+v"(a##k));
#define K_SUB(k) asm volatile("v_sub_u32 %0, %0, %1" : "+v"(a##k) : "v"(b));
#define K_AND(k) asm volatile("v_and_b32 %0, %0, %1" : "+v"(a##k) : "v"(b));
#define K_AND_L(k) asm volatile("v_and_b32 %0, 0x3ffff, %0" : "+v"(a##k));
#define K_OR(k) asm volatile("v_or_b32 %0, %0, %1" : "+v"(a##k) : "v"(b));
#define K_LSHR(k) asm volatile("v_lshrrev_b32 %0, %1, %0" : "+v"(a##k) : "v"(b));
#define K_ASHR(k) asm volatile("v_ashrrev_i32 %0, %1, %0" : "+v"(a##k) : "v"(b));
#define K_MIN(k) asm volatile("v_min_u32 %0, %0, %1" : "+v"(a##k) : "v"(b));
#define K_MAX(k) asm volatile("v_max_u32 %0, %0, %1" : "+v"(a##k) : "v"(b));
#define K_MIN3(k) asm volatile("v_min3_u32 %0, %0, %1, %1" : "+v"(a##k) : "v"(b));
#define K_ADD3(k) asm volatile("v_add3_u32 %0, %0, %1, %1" : "+v"(a##k) : "v"(b));
#define K_BITOP3(k) asm volatile("v_bitop3_b32 %0, %0, %1, %1 bitop3:0x96" : "+v"(a##k) : "v"(b));
#define K_BITOP3_S(k) asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a##k) : "v"(b), "s"(bs));
#define K_ALIGN(k) asm volatile("v_alignbit_b32 %0, %0, %1, %1" : "+v"(a##k) : "v"(b));
#define K_CND(k) asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(a##k) : "v"(b), "s"(m));
#define K_MULHI(k) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a##k) : "v"(b));
#define K_MULLO(k) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a##k) : "v"(b));
#define K_MUL24(k) asm volatile("v_mul_u32_u24 %0, %0, %1" : "+v"(a##k) : "v"(b));
#define K_MAD64(k) { uint64_t c_; asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(q##k), "=s"(c_) : "v"(a##k), "v"(b)); }
#define K_SHR64(k) asm volatile("v_lshrrev_b64 %0, %1, %0" : "+v"(q##k) : "v"(b));
#define K_MULF(k) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(a##k) : "v"(b));
#define K_ADDF(k) asm volatile("v_add_f32 %0, %0, %1" : "+v"(a##k) : "v"(b));
#define K_CVTF(k) asm volatile("v_cvt_f32_u32 %0, %0" : "+v"(a##k));
#define K_FMA64(k) asm volatile("v_fma_f64 %0, %0, %1, %1" : "+v"(d##k) : "v"(db));

#define KIND(ID, NAME, BODY)                                                                              \
    __global__ __launch_bounds__(256) void k_##NAME(uint32_t* out, int iters, uint32_t seed, uint32_t bs, \
                                                    uint64_t m) {                                         \
        const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;                                         \
        uint32_t a0 = t ^ seed, a1 = t + 1, a2 = t + 2, a3 = t + 3, a4 = t + 4, a5 = t + 5, a6 = t + 6,   \
                 a7 = t + 7;                                                                              \
        uint64_t q0 = a0, q1 = a1, q2 = a2, q3 = a3, q4 = a4, q5 = a5, q6 = a6, q7 = a7;                  \
        double d0 = a0, d1 = a1, d2 = a2, d3 = a3, d4 = a4, d5 = a5, d6 = a6, d7 = a7;                    \
        const uint32_t b = seed | 1;                                                                      \
        const double db = 1.0000001;                                                                      \
        for (int i = 0; i < iters; ++i) { REP8(BODY) }                                                    \
        (void)bs;                                                                                         \
        (void)m;                                                                                          \
        out[t] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7 ^ (uint32_t)(q0 ^ q1 ^ q2 ^ q3 ^ q4 ^ q5 ^ q6 ^ q7) ^ \
                 (uint32_t)(d0 + d1 + d2 + d3 + d4 + d5 + d6 + d7);                                       \
    }

KIND(0, xor, K_XOR)
KIND(1, xor_sgpr, K_XOR_S)
KIND(2, add, K_ADD)
KIND(3, add_inline_const, K_ADD_C)
KIND(4, sub, K_SUB)
KIND(5, and, K_AND)
KIND(6, and_literal, K_AND_L)
KIND(7, or, K_OR)
KIND(8, lshr, K_LSHR)
KIND(9, ashr, K_ASHR)
KIND(10, min_u32, K_MIN)
KIND(11, max_u32, K_MAX)
KIND(12, min3_u32, K_MIN3)
KIND(13, add3_u32, K_ADD3)
KIND(14, bitop3, K_BITOP3)
KIND(15, alignbit, K_ALIGN)
KIND(16, cndmask_e64, K_CND)
KIND(17, mul_hi_u32, K_MULHI)
KIND(18, mul_lo_u32, K_MULLO)
KIND(19, mul_u32_u24, K_MUL24)
KIND(20, mad_u64_u32, K_MAD64)
KIND(21, lshr_b64, K_SHR64)
KIND(22, mul_f32, K_MULF)
KIND(23, add_f32, K_ADDF)
KIND(24, cvt_f32_u32, K_CVTF)
KIND(25, fma_f64, K_FMA64)
KIND(26, bitop3_sgpr, K_BITOP3_S)

typedef void (*KernelFn)(uint32_t*, int, uint32_t, uint32_t, uint64_t);

static int run(const char* name, KernelFn k, uint32_t* dout, int grid, int iters, hipEvent_t e0, hipEvent_t e1) {
    hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, 0, dout, iters, 12345u, 0x9e3779b9u, 0x5555555555555555ull);
    CHK(hipGetLastError());
    CHK(hipDeviceSynchronize());
    CHK(hipEventRecord(e0));
    for (int r = 0; r < 5; ++r)
        hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, 0, dout, iters, 777u + r, 0x9e3779b9u, 0x5555555555555555ull);
    CHK(hipEventRecord(e1));
    CHK(hipEventSynchronize(e1));
    float ms;
    CHK(hipEventElapsedTime(&ms, e0, e1));
    const double ops = 5.0 * grid * 256.0 * iters * 8.0;
    printf("%-18s %8.3f ms  %7.2f T lane-ops/s\n", name, ms, ops / (ms * 1e-3) / 1e12);
    return 0;
}

int main() {
    const int grid = 4096, iters = 2000;
    uint32_t* dout;
    CHK(hipMalloc(&dout, (size_t)grid * 256 * sizeof(uint32_t)));
    hipEvent_t e0, e1;
    CHK(hipEventCreate(&e0));
    CHK(hipEventCreate(&e1));
    hipDeviceProp_t pr;
    CHK(hipGetDeviceProperties(&pr, 0));
    printf("device %s, %d CUs, clock %d kHz\n", pr.gcnArchName, pr.multiProcessorCount, pr.clockRate);
    struct { const char* name; KernelFn k; } kinds[] = {
        {"xor", k_xor}, {"xor_sgpr", k_xor_sgpr}, {"add", k_add}, {"add_inline_const", k_add_inline_const},
        {"sub", k_sub}, {"and", k_and}, {"and_literal", k_and_literal}, {"or", k_or}, {"lshr", k_lshr},
        {"ashr", k_ashr}, {"min_u32", k_min_u32}, {"max_u32", k_max_u32}, {"min3_u32", k_min3_u32},
        {"add3_u32", k_add3_u32}, {"bitop3", k_bitop3}, {"bitop3_sgpr", k_bitop3_sgpr}, {"alignbit", k_alignbit}, {"cndmask_e64", k_cndmask_e64},
        {"mul_hi_u32", k_mul_hi_u32}, {"mul_lo_u32", k_mul_lo_u32}, {"mul_u32_u24", k_mul_u32_u24},
        {"mad_u64_u32", k_mad_u64_u32}, {"lshr_b64", k_lshr_b64}, {"mul_f32", k_mul_f32}, {"add_f32", k_add_f32},
        {"cvt_f32_u32", k_cvt_f32_u32}, {"fma_f64", k_fma_f64},
    };
    for (auto& kd : kinds)
        if (run(kd.name, kd.k, dout, grid, iters, e0, e1)) return 1;
    CHK(hipFree(dout));
    return 0;
}
