// Fused Bicoptor 2.0 DReLU (Alg. 7) and UBL ReLU (Alg. 8) kernel.
//
// One thread owns one element and plays P0, P1 and P2 for it:
//   P0/P1  steps 1-2   flip both shares by the seed_01 bit t
//          step 3      l_x + 1 windows trc(x, k_lo + i, l - l_x - k_lo - i)
//          step 4      adjacent sums v_i = u_i + u_{i+1} - 1 (P0 adds the -1)
//          step 5      modulo switch to Z_p (Alg. 6)
//          step 6      shuffle: slot s takes the position with the s-th
//                      smallest seed_01 key (sorting network on 32-bit keys)
//          step 7-8    mask by r_s in Z_p^*, reshare by +-z_s
//   P2     step 9      reconstruct every slot, D' = [some slot is 0]
//          step 10     reshare D' with rho from seed_02 (DReLU)
//   P0/P1  step 11     unflip: t + (1 - 2t) [D']
// ReLU replaces steps 10-11 by the Beaver product of Alg. 8 with the
// triple generated from seed_02 / seed_12 and the unflipped input shares.
//
// The l_x + 1 window values never leave VGPRs.  The shuffle is applied by
// computing, for slot s, the window of the position the sorted key names:
// the message in slot s is v_{sigma(s)} r_s + z_s, exactly the shuffled and
// masked array of steps 6-8.  With a capture pointer the same code also
// stores both parties' round-1 messages.
#pragma once

#include <type_traits>

#include "bc_device.h"
#include "internal.h"

namespace bc {

struct DreluKArgs {
    const void* x0;
    const void* x1;
    void* y0;
    void* y1;
    void* cap;
    uint64_t n;
    uint64_t elem_base;
    uint64_t ring_mask;   // 2^l - 1
    uint32_t lx, k_lo, npos, pad;
    Stream s01, s02, s12;
};

template <typename T, int NMAX, typename F, bool RELU, bool CAP>
__global__ __launch_bounds__(256) void k_drelu(DreluKArgs A, F f) {
    using FT = typename F::T;
    constexpr bool WIDE = std::is_same<FT, uint64_t>::value;
    const T* __restrict__ X0 = static_cast<const T*>(A.x0);
    const T* __restrict__ X1 = static_cast<const T*>(A.x1);
    T* Y0 = static_cast<T*>(A.y0);
    T* Y1 = static_cast<T*>(A.y1);
    const T mask = (T)A.ring_mask;
    const uint32_t lx = A.lx;
    const uint32_t k_lo = A.k_lo;
    const uint32_t npos = A.npos;
    const FT two_lx = (FT)1 << lx;                       // 2^l_x mod p = 2^l_x
    const FT p_minus_two = f.p - two_lx;
    const FT win_mask = two_lx - 1;                      // Z_{2^l_x}
    const FT win1_mask = WIDE ? (FT)((1ull << 33) - 1) : (FT)((two_lx << 1) - 1);   // l_x + 1 bits

    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < A.n; e += stride) {
        const uint64_t g = A.elem_base + e;
        const T in0 = X0[e] & mask;
        const T in1 = X1[e] & mask;

        // Steps 1 and 6 (randomness): t and the shuffle keys from seed_01.
        uint32_t key[NMAX];
        uint32_t t = 0;
#pragma unroll
        for (int b = 0; b < (NMAX + 3) / 4; ++b) {
            if (4 * b < (int)npos) {
                const Words4 w = A.s01.block(g, TAG_SHUFFLE, b);
                if (b == 0) t = w.w0 & 1u;
                const uint32_t ws[4] = {w.w0, w.w1, w.w2, w.w3};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (4 * b + q < NMAX)
                        key[4 * b + q] = (4 * b + q < (int)npos) ? ((ws[q] & ~63u) | (uint32_t)(4 * b + q)) : 0xFFFFFFFFu;
                }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (4 * b + q < NMAX) key[4 * b + q] = 0xFFFFFFFFu;
            }
        }
        sort_keys<NMAX>(key);

        // Step 2: [x] := (-1)^t [x]  (both parties).
        const T a0 = t ? (T)((T)0 - in0) & mask : in0;
        const T a1 = t ? (T)((T)0 - in1) & mask : in1;
        const T nb1 = (T)((T)0 - a1) & mask;              // P1 cuts -[x]_1 mod 2^l

        bool zero = false;
        Words4 wm = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < NMAX; ++j) {
            if (j < (int)npos) {
                // Steps 7-8 randomness of slot j.
                FT r, z;
                if constexpr (WIDE) {
                    const Words4 w = A.s01.block(g, TAG_MASK, (uint32_t)j);
                    r = 1 + __umul64hi(join64(w.w0, w.w1), f.p - 1);
                    z = __umul64hi(join64(w.w2, w.w3), f.p);
                } else {
                    if ((j & 1) == 0) wm = A.s01.block(g, TAG_MASK, (uint32_t)(j >> 1));
                    r = Draw<F>::r((j & 1) ? wm.w2 : wm.w0, f);
                    z = Draw<F>::z((j & 1) ? wm.w3 : wm.w1, f);
                }
                // Steps 3-4 for the position sigma(j) placed in slot j.
                const uint32_t pos = key[j] & 63u;
                const uint32_t s = k_lo + pos;
                const bool last = pos == lx;                  // u_{l_x+1} := 0
                const FT W0 = (FT)(a0 >> s) & win1_mask;      // bits [s, s + l_x]
                const FT W1 = (FT)(nb1 >> s) & win1_mask;
                const FT u0n = last ? (FT)0 : (W0 >> 1);      // u_{i+1} of P0
                const FT u1n = last ? (FT)0 : (W1 >> 1);
                const FT v0 = (W0 + u0n - 1) & win_mask;              // u_i + u_{i+1} - 1
                const FT v1 = ((FT)0 - W1 - u1n) & win_mask;          // -(cut_i) - (cut_{i+1})
                // Step 5: Alg. 6.
                const FT s0 = v0 ? v0 : two_lx;
                const FT s1 = v1 + p_minus_two;
                // Steps 7-8: mask and reshare.
                const FT w0 = addmod(f.mul(s0, r), z, f);
                const FT w1 = addmod(f.mul(s1, r), (FT)(f.p - z), f);
                if constexpr (CAP) {
                    FT* C = static_cast<FT*>(A.cap);
                    C[e * npos + (uint64_t)j] = w0;
                    C[(A.n + e) * npos + (uint64_t)j] = w1;
                }
                // Step 9 (P2): reconstruct and test for zero.
                zero |= addmod(w0, w1, f) == 0;
            }
        }
        const T dp = zero ? 1 : 0;

        T y0, y1;
        if constexpr (!RELU) {
            // Step 10 (P2): fresh sharing (rho, D' - rho) with rho from seed_02.
            const Words4 w = A.s02.block(g, TAG_RESP, 0);
            const T rho = (T)join64(w.w0, w.w1) & mask;
            const T d1 = (T)(dp - rho) & mask;
            // Step 11: DReLU = t + (1 - 2t) D'.
            y0 = t ? (T)((T)1 - rho) & mask : rho;
            y1 = t ? (T)((T)0 - d1) & mask : d1;
        } else {
            // Alg. 8 preprocessing: [a]_0, [b]_0, [c]_0 from seed_02, [a]_1, [b]_1
            // from seed_12; P2 forms [c]_1 = (a0 + a1)(b0 + b1) - c0.
            const Words4 w0 = A.s02.block(g, TAG_BEAVER, 0);
            const Words4 w1 = A.s02.block(g, TAG_BEAVER, 1);
            const Words4 w2 = A.s12.block(g, TAG_BEAVER, 0);
            const T ba0 = (T)join64(w0.w0, w0.w1) & mask;
            const T bb0 = (T)join64(w0.w2, w0.w3) & mask;
            const T bc0 = (T)join64(w1.w0, w1.w1) & mask;
            const T ba1 = (T)join64(w2.w0, w2.w1) & mask;
            const T bb1 = (T)join64(w2.w2, w2.w3) & mask;
            const T bsum = (T)(bb0 + bb1);
            const T bc1 = (T)((T)(ba0 + ba1) * bsum - bc0) & mask;
            // Step 3 (P2): e = D' - b.  Step 4 (P0, P1): d = x - a, exchanged.
            const T ee = (T)(dp - bsum) & mask;
            const T dd = (T)((in0 - ba0) + (in1 - ba1)) & mask;
            // Step 5: [x D'] = de + d[b] + e[a] + [c]; ReLU = t[x] + (1 - 2t)[x D'].
            const T m0 = (T)(dd * ee + dd * bb0 + ee * ba0 + bc0) & mask;
            const T m1 = (T)(dd * bb1 + ee * ba1 + bc1) & mask;
            y0 = t ? (T)(in0 - m0) & mask : m0;
            y1 = t ? (T)(in1 - m1) & mask : m1;
        }
        Y0[e] = y0;
        Y1[e] = y1;
    }
}

// Host helpers: field parameters for each prime size.
inline FieldSmall make_field_small(uint64_t p) { return FieldSmall{(uint32_t)p, 1.0f / (float)p}; }
inline Field24 make_field24(uint64_t p) {
    uint32_t k = 0;
    if (((p + 1) & p) == 0) {   // p = 2^k - 1
        while ((1ull << k) - 1 != p) ++k;
    }
    return Field24{(uint32_t)p, k, (double)p, 1.0 / (double)p};
}
inline Field32 make_field32(uint64_t p) { return Field32{(uint32_t)p, UINT64_MAX / p}; }
inline Field64 make_field64(uint64_t p) { return Field64{p, (double)p, 1.0 / (double)p}; }

inline DreluKArgs make_kargs(const DreluLaunch& L) {
    DreluKArgs A;
    A.x0 = L.x0;
    A.x1 = L.x1;
    A.y0 = L.y0;
    A.y1 = L.y1;
    A.cap = L.cap;
    A.n = L.n;
    A.elem_base = L.elem_base;
    A.ring_mask = L.ell >= 64 ? ~0ull : ((1ull << L.ell) - 1);
    A.lx = L.lx;
    A.k_lo = L.k_lo;
    A.npos = L.npos;
    A.pad = 0;
    A.s01 = Stream{L.s01.k0, L.s01.k1, L.s01.n0, L.s01.n1};
    A.s02 = Stream{L.s02.k0, L.s02.k1, L.s02.n0, L.s02.n1};
    A.s12 = Stream{L.s12.k0, L.s12.k1, L.s12.n0, L.s12.n1};
    return A;
}

template <typename T, int NMAX, typename F, bool RELU>
hipError_t launch_bucket(const DreluLaunch& L, const F& f, hipStream_t st) {
    const DreluKArgs A = make_kargs(L);
    if (L.cap)
        hipLaunchKernelGGL((k_drelu<T, NMAX, F, RELU, true>), dim3(L.grid), dim3(L.block), 0, st, A, f);
    else
        hipLaunchKernelGGL((k_drelu<T, NMAX, F, RELU, false>), dim3(L.grid), dim3(L.block), 0, st, A, f);
    return hipGetLastError();
}

}  // namespace bc
