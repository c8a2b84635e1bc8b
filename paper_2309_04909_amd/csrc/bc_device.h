// Device building blocks of the DReLU/ReLU kernels (gfx950, wave64).
//
//  * Philox4x32-10 (Salmon et al., SC'11): the counter-based generator behind
//    every "generate ... using seed" of Alg. 7 and Alg. 8.
//  * Modular multiplication in Z_p for the four prime sizes the window width
//    l_x produces (p has l_x + 1 bits, notation table):
//      FieldSmall  p < 2^12   products < 2^24: one 24-bit multiply, fp32 quotient
//      FieldMersenne<K>  p = 2^K - 1 < 2^24: one fold
//      Field24     p < 2^24   products exact in fp64, fp64 quotient
//      Field32     p < 2^32   64-bit products, Barrett with a 64-bit reciprocal
//      Field64     p < 2^34   l_x = 32; 66-bit products, fp64 quotient
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Launch attributes of the DReLU/ReLU kernels (256-thread blocks).  A build
// may override them (e.g. with an amdgpu_waves_per_eu occupancy hint).
#ifndef BC_KERNEL_ATTRS
#define BC_KERNEL_ATTRS __launch_bounds__(256)
#endif

namespace bc {

// ------------------------------------------------------------------ Philox

constexpr uint32_t PHILOX_M0 = 0xD2511F53u;
constexpr uint32_t PHILOX_M1 = 0xCD9E8D57u;
constexpr uint32_t PHILOX_W0 = 0x9E3779B9u;
constexpr uint32_t PHILOX_W1 = 0xBB67AE85u;

// V consecutive elements of T, for one vector load or store per thread.
template <typename T, int V>
using vec_t = T __attribute__((ext_vector_type(V)));

// Loads and stores of data that a call reads or writes once (shares,
// records, messages), marked nontemporal: on gfx950 the truncation stream
// went from 5.6 to 6.2 TB/s with them.
template <typename P>
__device__ __forceinline__ P ld_nt(const P* p) {
    return __builtin_nontemporal_load(p);
}
template <typename P>
__device__ __forceinline__ void st_nt(P* p, P v) {
    __builtin_nontemporal_store(v, p);
}

constexpr uint32_t TAG_SHUFFLE = 1;
constexpr uint32_t TAG_MASK = 2;
constexpr uint32_t TAG_RESP = 3;
constexpr uint32_t TAG_BEAVER = 4;
constexpr uint32_t TAG_RSS = 5;      // replicated-sharing preprocessing (Alg. drelu2)
constexpr uint32_t TAG_MUL = 6;      // Beaver triple of the elementwise product (Alg. linear)

struct Words4 {
    uint32_t w0, w1, w2, w3;
};

// Three-input XOR in one gfx950 v_bitop3_b32 (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Rounds R0..9 of Philox4x32-10.  Round r uses key (k0 + r W0, k1 + r W1) and
// maps (c0, c1, c2, c3) to
//   (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)).
// In round 0, c2, c3 (the nonce) and the key are uniform, so the uniform
// pairs are left to plain XORs (scalar unit); later rounds use xor3.
template <int R0>
__device__ __forceinline__ Words4 philox_rounds(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                uint32_t k1) {
#pragma unroll
    for (int r = R0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        const uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        const uint32_t rk0 = k0 + (uint32_t)r * PHILOX_W0;
        const uint32_t rk1 = k1 + (uint32_t)r * PHILOX_W1;
        const uint32_t n0 = r == 0 ? ((uint32_t)(p1 >> 32) ^ rk0) ^ c1 : xor3((uint32_t)(p1 >> 32), c1, rk0);
        const uint32_t n2 = r == 0 ? (c3 ^ rk1) ^ (uint32_t)(p0 >> 32) : xor3((uint32_t)(p0 >> 32), c3, rk1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return {c0, c1, c2, c3};
}

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
    return philox_rounds<0>(c0, c1, c2, c3, k0, k1);
}

// The key is uniform.  Passing it through an empty asm stops the compiler
// from hoisting all round keys of every seed out of the element loop, and the
// scheduling barrier stops it from computing the round keys of later blocks
// ahead of time; either exhausts the SGPRs.  Each block recomputes its round
// keys with scalar adds.
__device__ __forceinline__ void launder_key(uint32_t& a, uint32_t& c) {
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" : "+s"(a), "+s"(c));
}

// Blocks of one stream at one element index g.  The counters of all its
// blocks, (lo g, hi16(g) | tag << 16 | b << 24, nonce), differ only in word 1,
// which round 0 folds into word 0 alone.  So hi/lo(M0 lo g) of round 0,
// M1 c2 of round 1 and M0 c0 of round 2 are the same for every block; they
// are computed once here, and each block runs 16 multiplies instead of 20.
// The shared words that meet a round key in rounds 1-3 are stored already
// XORed with it, so those XORs take two VGPR operands (a full-rate VOP2)
// instead of three.
struct StreamAt {
    uint32_t k0, k1;    // key
    uint32_t ghi;       // hi16(g)
    uint32_t u0;        // hi(M1 n0) ^ k0: round-0 word 0 without the block's word 1
    uint32_t c3k;       // round-0 output word 3 ^ round-1 key 1
    uint32_t c1k;       // round-1 output word 1 ^ round-2 key 0
    uint32_t h2k;       // hi(M0 c0) of round 2 ^ round-2 key 1
    uint32_t l2k;       // lo(M0 c0) of round 2 (round-3 word 3) ^ round-3 key 1

    __device__ __forceinline__ Words4 block(uint32_t tag, uint32_t b) const {
        uint32_t a = k0, c = k1;
        launder_key(a, c);
        const uint32_t x0 = u0 ^ (ghi | (tag << 16) | (b << 24));              // round 0, word 0
        const uint64_t p0 = (uint64_t)PHILOX_M0 * x0;                          // round 1
        const uint32_t y2 = (uint32_t)(p0 >> 32) ^ c3k;
        const uint32_t y3 = (uint32_t)p0;
        const uint64_t p1 = (uint64_t)PHILOX_M1 * y2;                          // round 2
        const uint32_t z0 = (uint32_t)(p1 >> 32) ^ c1k;
        const uint32_t z2 = y3 ^ h2k;
        const uint64_t q0 = (uint64_t)PHILOX_M0 * z0;                          // round 3
        const uint64_t q1 = (uint64_t)PHILOX_M1 * z2;
        const uint32_t n0 = xor3((uint32_t)(q1 >> 32), (uint32_t)p1, a + 3u * PHILOX_W0);
        const uint32_t n2 = (uint32_t)(q0 >> 32) ^ l2k;
        return philox_rounds<4>(n0, (uint32_t)q1, n2, (uint32_t)q0, a, c);
    }
};

// Counter of block b of stream `tag` for global element index g.
struct Stream {
    uint32_t k0, k1;   // key = seed
    uint32_t n0, n1;   // (c2, c3) = nonce
    __device__ __forceinline__ Words4 block(uint64_t g, uint32_t tag, uint32_t b) const {
        const uint32_t c1 = ((uint32_t)(g >> 32) & 0xFFFFu) | (tag << 16) | (b << 24);
        uint32_t a = k0, c = k1;
        launder_key(a, c);
        return philox4x32_10((uint32_t)g, c1, n0, n1, a, c);
    }
    // The shared rounds of every block at element g (same words as block()).
    __device__ __forceinline__ StreamAt at(uint64_t g) const {
        uint32_t a = k0, c = k1;
        launder_key(a, c);
        const uint64_t P0 = (uint64_t)PHILOX_M0 * (uint32_t)g;                // round 0
        const uint64_t P1 = (uint64_t)PHILOX_M1 * n0;
        const uint32_t e2 = (uint32_t)(P0 >> 32) ^ (n1 ^ c);
        const uint64_t Q1 = (uint64_t)PHILOX_M1 * e2;                         // round 1
        const uint32_t c0b = (uint32_t)(Q1 >> 32) ^ ((uint32_t)P1 ^ (a + PHILOX_W0));
        const uint64_t Q2 = (uint64_t)PHILOX_M0 * c0b;                        // round 2
        return StreamAt{k0,
                        k1,
                        (uint32_t)(g >> 32) & 0xFFFFu,
                        (uint32_t)(P1 >> 32) ^ a,
                        (uint32_t)P0 ^ (c + PHILOX_W1),
                        (uint32_t)Q1 ^ (a + 2u * PHILOX_W0),
                        (uint32_t)(Q2 >> 32) ^ (c + 2u * PHILOX_W1),
                        (uint32_t)Q2 ^ (c + 3u * PHILOX_W1)};
    }
};

__device__ __forceinline__ uint64_t join64(uint32_t lo, uint32_t hi) {
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// ------------------------------------------------------------ Z_p arithmetic

// A uniform value copied into a VGPR.  On gfx950 the VOP2 forms issue at about
// twice the rate with VGPR or literal operands as with an SGPR operand, so
// the runtime prime of the smaller fields is kept in VGPRs by the kernels.
__device__ __forceinline__ uint32_t in_vgpr(uint32_t x) {
    uint32_t v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
    return v;
}
__device__ __forceinline__ uint64_t in_vgpr(uint64_t x) {
    return (uint64_t)in_vgpr((uint32_t)x) | ((uint64_t)in_vgpr((uint32_t)(x >> 32)) << 32);
}
__device__ __forceinline__ float in_vgpr(float x) {
    float v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
    return v;
}

// a * b + c in one v_mad_u64_u32.  Written out because, with operands the
// compiler knows to be narrow, it otherwise splits the product into 24-bit
// multiplies and 64-bit shift-adds.
__device__ __forceinline__ uint64_t mad_u64_u32(uint32_t a, uint32_t b, uint64_t c) {
    uint64_t d, carry;
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(d), "=s"(carry) : "v"(a), "v"(b), "v"(c));
    return d;
}

// p < 2^12.  a, b < p, so a*b < 2^24 is exact in one v_mul_u32_u24 and in
// fp32.  The fp32 quotient is within one of floor(x / p); two corrections.
struct FieldSmall {
    using T = uint32_t;
    static constexpr bool kWrap = false;
    static constexpr bool kDefault = false;   // any prime below 2^12
    uint32_t p;
    float pinv;
    __device__ __forceinline__ uint32_t reduce24(uint32_t x) const {   // x < 2^24
        const uint32_t q = (uint32_t)((float)x * pinv);
        uint32_t r = x - __umul24(q, p);   // in (-p, 2p), mod 2^32
        r = min(r, r + p);                 // negative: the wrapped r + p is the small one
        return min(r, r - p);              // >= p: r - p; else r - p wraps and r stays
    }
    __device__ __forceinline__ FieldSmall vgpr() const { return FieldSmall{in_vgpr(p), in_vgpr(pinv)}; }
    __device__ __forceinline__ uint32_t mul(uint32_t a, uint32_t b) const { return reduce24(__umul24(a, b)); }
    // a, b, c < p: a*b + c <= p^2 - p < 2^24 as well.
    __device__ __forceinline__ uint32_t mul_add(uint32_t a, uint32_t b, uint32_t c) const {
        return reduce24(__umul24(a, b) + c);
    }
};

// p < 2^24, p = 2^K - 1 (Mersenne).  a*b < 2^48 from one 64-bit multiply;
// since a, b < p, (x mod 2^K) + (x >> K) < 2p, so one fold and one
// conditional subtraction reduce it.
template <int K>
struct FieldMersenne {
    using T = uint32_t;
    static constexpr bool kWrap = false;
    static constexpr bool kDefault = true;    // the largest prime below 2^K
    // A compile-time p becomes a literal operand: on gfx950 the VOP2 forms
    // issue at about twice the rate with literal or VGPR operands as with an
    // SGPR operand.
    static constexpr uint32_t p = (1u << K) - 1;
    static constexpr bool kLazy = true;       // the *_lazy forms: a value below 2p, 4p < 2^32
    __device__ __forceinline__ FieldMersenne vgpr() const { return *this; }
    __device__ __forceinline__ uint32_t mul(uint32_t a, uint32_t b) const {
        const uint64_t x = (uint64_t)a * b;
        const uint32_t s = ((uint32_t)x & p) + (uint32_t)(x >> K);
        return min(s, s - p);             // s < p: s - p wraps above s
    }
    // a, b, c < p: x = a*b + c <= p^2 - p, so x >> K <= p - 2 and the fold is
    // still below 2p; the addend rides in the multiply.  The lazy form stops
    // before the conditional subtraction.
    __device__ __forceinline__ uint32_t mul_add_lazy(uint32_t a, uint32_t b, uint32_t c) const {
        const uint64_t x = mad_u64_u32(a, b, c);
        return ((uint32_t)x & p) + (uint32_t)(x >> K);
    }
    __device__ __forceinline__ uint32_t mul_add(uint32_t a, uint32_t b, uint32_t c) const {
        const uint32_t s = mul_add_lazy(a, b, c);
        return min(s, s - p);
    }
    // The same with b and c given shifted left by SH = 32 - K (b_sh = b 2^SH,
    // c_sh = c 2^SH; a < p, b < p, c <= p): the product x 2^SH < 2^(K + 32)
    // splits at bit 32 into x >> K (high word) and (x mod 2^K) 2^SH (low
    // word), so the fold takes one shift instead of a funnel shift.
    template <int SH>
    __device__ __forceinline__ uint32_t mul_add_sh_lazy(uint32_t a, uint32_t b_sh, uint32_t c_sh) const {
        static_assert(SH == 32 - K, "operands shifted to the top of the word");
        const uint64_t x = mad_u64_u32(a, b_sh, c_sh);
        return ((uint32_t)x >> SH) + (uint32_t)(x >> 32);
    }
    template <int SH>
    __device__ __forceinline__ uint32_t mul_add_sh(uint32_t a, uint32_t b_sh, uint32_t c_sh) const {
        const uint32_t s = mul_add_sh_lazy<SH>(a, b_sh, c_sh);
        return min(s, s - p);
    }
};

// p = 2^K - c with c < 64 and c^2 < p (pseudo-Mersenne), K <= 32.  Every
// default prime (the largest prime below 2^K) has this form.  x = a*b + d (a, b, d < p)
// is below 2^(2K); with 2^K = c mod p, x = H 2^K + L folds to L + c H
// < (c + 1) 2^K, a second fold to L' + c H' < 2^K + c^2 < 2p, and one
// conditional subtraction ends it.  p is a literal, and both folds are
// multiply-adds.
template <int K, uint32_t CC>
struct FieldPM {
    static_assert(K >= 2 && K <= 32 && CC >= 1 && CC < 64 && (uint64_t)CC * CC < (1ull << K) - CC,
                  "pseudo-Mersenne 2^K - c with c^2 < p");
    using T = uint32_t;
    static constexpr bool kWrap = K == 32;   // p > 2^31: 32-bit sums can wrap
    static constexpr bool kDefault = true;   // the largest prime below 2^K
    static constexpr uint32_t p = (uint32_t)((1ull << K) - CC);
    static constexpr uint32_t LOW = (uint32_t)((1ull << K) - 1);
    static constexpr bool kLazy = K <= 30;   // the *_lazy forms: a value below 2p, 4p < 2^32
    __device__ __forceinline__ FieldPM vgpr() const { return *this; }
    __device__ __forceinline__ uint32_t mul(uint32_t a, uint32_t b) const { return mul_add(a, b, 0); }
    // Both folds, without the final conditional subtraction: below 2p (K < 32).
    __device__ __forceinline__ uint32_t mul_add_lazy(uint32_t a, uint32_t b, uint32_t d) const {
        static_assert(K < 32, "the 32-bit fold ends differently");
        if constexpr (K <= 12) {
            // x < p^2 < 2^24: every step in 32 bits with 24-bit multiply-adds
            const uint32_t x = __umul24(a, b) + d;
            const uint32_t t = __umul24(x >> K, CC) + (x & LOW);    // < (c + 1) 2^K
            return __umul24(t >> K, CC) + (t & LOW);                // < 2^K + c^2 < 2p
        } else {
            const uint64_t x = mad_u64_u32(a, b, d);
            const uint32_t H = __builtin_amdgcn_alignbit((uint32_t)(x >> 32), (uint32_t)x, K);   // x >> K
            const uint32_t L = (uint32_t)x & LOW;
            uint32_t H2, L2;
            if constexpr (K <= 24) {
                const uint32_t t = __umul24(H, CC) + L;            // < 2^(K + 6) <= 2^30
                H2 = t >> K;
                L2 = t & LOW;
            } else {
                const uint64_t t = mad_u64_u32(H, CC, L);           // < 2^(K + 6)
                H2 = __builtin_amdgcn_alignbit((uint32_t)(t >> 32), (uint32_t)t, K);
                L2 = (uint32_t)t & LOW;
            }
            return L2 + __umul24(H2, CC);                          // < 2^K + c^2 < 2p
        }
    }
    __device__ __forceinline__ uint32_t mul_add(uint32_t a, uint32_t b, uint32_t d) const {
        if constexpr (K < 32) {
            const uint32_t S = mul_add_lazy(a, b, d);
            return min(S, S - p);
        }
        // K = 32: 64-bit folds, and S = L2 + c H2 < 2^32 + c^2 may exceed 32
        // bits; S >= p exactly when S + c reaches 2^32, and then
        // S - p = (S + c) mod 2^32.
        const uint64_t x = mad_u64_u32(a, b, d);
        const uint64_t t = mad_u64_u32((uint32_t)(x >> 32), CC, (uint32_t)x);   // < 2^38
        const uint64_t S = (uint64_t)(uint32_t)t + __umul24((uint32_t)(t >> 32), CC);
        const uint64_t R = S + CC;
        return (R >> 32) ? (uint32_t)R : (uint32_t)S;
    }
    // mul_add with b and d given shifted left by SH = 32 - K (12 < K <= 24):
    // x 2^SH splits at bit 32 into H = x >> K and L 2^SH, L = x mod 2^K.
    template <int SH>
    __device__ __forceinline__ uint32_t mul_add_sh_lazy(uint32_t a, uint32_t b_sh, uint32_t d_sh) const {
        static_assert(SH == 32 - K && K > 12 && K <= 24, "operands shifted to the top of the word");
        const uint64_t x = mad_u64_u32(a, b_sh, d_sh);
        const uint32_t H = (uint32_t)(x >> 32), L = (uint32_t)x >> SH;
        const uint32_t t = __umul24(H, CC) + L;                    // < 2^(K + 6) <= 2^30
        return (t & LOW) + __umul24(t >> K, CC);                   // < 2^K + c^2 < 2p
    }
    template <int SH>
    __device__ __forceinline__ uint32_t mul_add_sh(uint32_t a, uint32_t b_sh, uint32_t d_sh) const {
        const uint32_t S = mul_add_sh_lazy<SH>(a, b_sh, d_sh);
        return min(S, S - p);
    }
};

// p = 2^33 - 9, the default prime of l_x = 32 (64-bit field elements).
// For a, b, d < p: split each at bit 32 (the high parts are single bits);
// then a*b + d = (a0 b0 + d0) + 2^32 (a1 b0 + a0 b1 + d1) + 2^64 a1 b1, and
// with 2^33 = 9 and 2^64 = 9 * 2^31 (mod p) each part folds below 2^36; their
// sum (< 2^37) folds once more below 2^33 + 144 < 2p.  Three 32x32 multiply-
// adds, no fp64 and no 64x64 product.
struct FieldPM33 {
    using T = uint64_t;
    static constexpr bool kWrap = false;
    static constexpr bool kDefault = true;    // the largest prime below 2^33
    static constexpr uint64_t p = (1ull << 33) - 9;
    static constexpr uint64_t LOW33 = (1ull << 33) - 1;
    __device__ __forceinline__ FieldPM33 vgpr() const { return *this; }
    __device__ __forceinline__ uint64_t mul(uint64_t a, uint64_t b) const { return mul_add(a, b, 0); }
    __device__ __forceinline__ uint64_t mul_add(uint64_t a, uint64_t b, uint64_t d) const {
        const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
        const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
        const uint32_t d0 = (uint32_t)d, d1 = (uint32_t)(d >> 32);
        const uint64_t t0 = mad_u64_u32(a0, b0, d0);                                   // < 2^64
        const uint64_t A = mad_u64_u32((uint32_t)(t0 >> 33), 9u, t0 & LOW33);          // < 2^35
        const uint64_t C = (uint64_t)(a1 ? b0 : 0u) + (b1 ? a0 : 0u) + d1;             // < 2^33 - 18
        const uint64_t Cm = mad_u64_u32((uint32_t)(C >> 1), 9u, (C & 1) << 32);        // C 2^32 mod-folded
        const uint64_t U = A + Cm + ((a1 & b1) ? (9ull << 31) : 0ull);                 // < 2^37
        const uint64_t R = (U & LOW33) + 9u * (uint32_t)(U >> 33);                      // < 2p
        return R >= p ? R - p : R;
    }
};

// 2^K minus the largest prime below 2^K, for K = lx + 1 in 2..33 (the
// default primes; 0 where unused).  Checked against an independent
// primality search on the host.
constexpr uint32_t kPrimeDelta[34] = {0, 0, 1, 1, 3, 1, 3, 1, 5, 3, 3, 9, 3, 1, 3, 19, 15, 1,
                                      5, 1, 3, 9, 3, 15, 3, 39, 5, 39, 57, 3, 35, 1, 5, 9};

// p < 2^24, any prime.  a*b < 2^48 is exact in fp64; an fp64 quotient is
// within one of floor(x / p), and the remainder from an fma is exact.
struct Field24 {
    using T = uint32_t;
    static constexpr bool kWrap = false;
    static constexpr bool kDefault = false;   // any prime of its range
    uint32_t p;
    double pd, pinv;
    __device__ __forceinline__ Field24 vgpr() const { return Field24{in_vgpr(p), pd, pinv}; }
    __device__ __forceinline__ uint32_t mul(uint32_t a, uint32_t b) const {
        return reduce((double)a * (double)b);
    }
    // a, b, c < p: a*b + c < 2^48 is exact in one fp64 fma.
    __device__ __forceinline__ uint32_t mul_add(uint32_t a, uint32_t b, uint32_t c) const {
        return reduce(__builtin_fma((double)a, (double)b, (double)c));
    }
    __device__ __forceinline__ uint32_t reduce(double xd) const {   // integer xd < 2^48
        const double q = __builtin_floor(xd * pinv);
        double r = __builtin_fma(-q, pd, xd);
        r = r < 0.0 ? r + pd : r;
        r = r >= pd ? r - pd : r;
        return (uint32_t)r;
    }
};

// p < 2^32.  Barrett: mu = floor((2^64 - 1) / p); q = mulhi64(x, mu) is within
// two of floor(x / p).
struct Field32 {
    using T = uint32_t;
    static constexpr bool kWrap = true;   // p may exceed 2^31: a + b can wrap
    static constexpr bool kDefault = false;   // any prime of its range
    uint32_t p;
    uint64_t mu;
    __device__ __forceinline__ Field32 vgpr() const { return Field32{in_vgpr(p), mu}; }
    __device__ __forceinline__ uint32_t mul(uint32_t a, uint32_t b) const {
        return reduce((uint64_t)a * b);
    }
    // a, b, c < p < 2^32: a*b + c < 2^64, and the Barrett bound holds for any x < 2^64.
    __device__ __forceinline__ uint32_t mul_add(uint32_t a, uint32_t b, uint32_t c) const {
        return reduce((uint64_t)a * b + c);
    }
    __device__ __forceinline__ uint32_t reduce(uint64_t x) const {
        const uint64_t q = __umul64hi(x, mu);
        uint64_t r = x - q * p;
        r = r >= p ? r - p : r;
        r = r >= p ? r - p : r;
        return (uint32_t)r;
    }
};

// 2^32 < p < 2^34 (l_x = 32).  x = a*b < 2^68 as a 128-bit product; an fp64
// quotient of x / p (< 2^34, relative error 2^-51) is within one of the floor.
struct Field64 {
    using T = uint64_t;
    static constexpr bool kWrap = false;
    static constexpr bool kDefault = false;   // any prime of its range
    uint64_t p;
    double pd, pinv;
    __device__ __forceinline__ Field64 vgpr() const { return *this; }
    __device__ __forceinline__ uint64_t mul(uint64_t a, uint64_t b) const {
        const uint64_t lo = a * b;
        const uint64_t hi = __umul64hi(a, b);
        const double xd = __builtin_fma((double)hi, 18446744073709551616.0, (double)lo);
        const double qd = __builtin_floor(xd * pinv);
        const uint64_t q = (uint64_t)qd;
        int64_t r = (int64_t)(lo - q * p);   // true remainder in (-p, 2p): exact mod 2^64
        r = r < 0 ? r + (int64_t)p : r;
        r = r >= (int64_t)p ? r - (int64_t)p : r;
        return (uint64_t)r;
    }
    __device__ __forceinline__ uint64_t mul_add(uint64_t a, uint64_t b, uint64_t c) const {
        const uint64_t m = mul(a, b);
        const uint64_t s = m + c;          // < 2p < 2^35
        return s >= p ? s - p : s;
    }
};

// a < p, b <= p.  When p may exceed 2^31 the 32-bit sum can wrap; a wrapped
// sum is >= 2^32 > p, so it also takes the subtraction (exact mod 2^32).
template <typename F>
__device__ __forceinline__ typename F::T addmod(typename F::T a, typename F::T b, const F& f) {
    using FT = typename F::T;
    const FT s = a + b;
    if constexpr (F::kWrap) return (s < a || s >= f.p) ? s - f.p : s;
    return min(s, (FT)(s - f.p));         // s < p: s - p wraps above s
}

// a, b < p: (a - b) mod p.  Without wrap (2p <= 2^bits) the wrapped
// difference plus p is the answer exactly when a < b, and it is then the
// smaller of the two: one subtraction, one addition and one min.
template <typename F>
__device__ __forceinline__ typename F::T submod(typename F::T a, typename F::T b, const F& f) {
    using FT = typename F::T;
    const FT d = a - b;
    if constexpr (F::kWrap) return a < b ? d + f.p : d;
    return min(d, (FT)(d + f.p));
}

// Orders one wave's LDS accesses across its lanes: the lanes of a wave run
// in lockstep and the LDS serves a wave's instructions in order, so only the
// compiler must be kept from moving accesses across this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// r_s in Z_p^* and z_s in Z_p by multiply-shift of uniform 32-bit words
// (p < 2^32): r = 1 + floor(R (p - 1) / 2^32), z = floor(Z p / 2^32).
__device__ __forceinline__ uint32_t draw_r(uint32_t R, uint32_t p) { return 1u + __umulhi(R, p - 1u); }
__device__ __forceinline__ uint32_t draw_z(uint32_t Z, uint32_t p) { return __umulhi(Z, p); }

}  // namespace bc
