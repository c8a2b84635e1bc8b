// Fused Bicoptor 2.0 DReLU (Alg. 7) and UBL ReLU (Alg. 8) kernel.
//
// One thread owns one element and plays P0, P1 and P2 for it, in the order
// of Alg. 7:
//   P0/P1  flip     both shares negated when the seed_01 bit t is set
//          windows  l_x + 1 windows trc(x, k_lo + i, l - l_x - k_lo - i)
//          sums     adjacent sums v_i = u_i + u_{i+1} - 1 (P0 adds the -1)
//          switch   modulo switch to Z_p (Alg. 6)
//          shuffle  slot s takes position sigma(s) of a seed_01 Fisher-Yates
//                   shuffle run in the thread's slice of LDS
//          mask     multiply by r_s in Z_p^*, reshare by +-z_s
//   P2     test     reconstruct every slot, D' = [some slot is 0]
//          reply    reshare D' with rho from seed_02 (DReLU)
//   P0/P1  unflip   t + (1 - 2t) [D']
// ReLU replaces the reply and the unflip by the Beaver product of Alg. 8
// with the triple generated from seed_02 / seed_12 and the unflipped input
// shares.
//
// The l_x + 1 window values never leave VGPRs.  Kernels are instantiated
// per window count N = l_x + 1, so every loop over windows is unrolled.  The
// shuffle is applied by computing, for slot s, the window of the position
// sigma(s) read back from LDS: the message in slot s is v_{sigma(s)} r_s + z_s,
// exactly the array that the shuffle and mask produce.  With a capture
// pointer the same code also stores both parties' round-1 messages.
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
    uint64_t ncap;        // elements of the whole call (the capture's P1 half starts at ncap * N)
    uint64_t elem_base;
    uint64_t ring_mask;   // 2^l - 1
    uint64_t in_mask;     // 2^l_in - 1 of the input ring (l_in = l + k_in)
    uint32_t k_lo, k_in;  // k_in > 0: Alg. 5 truncation of the inputs by k_in bits first
    Stream s01, s02, s12;
};

// The share already shifted down by k_lo (pos <= l_x), shifted down by pos:
// bits [0, l_x] are the window, bits above it are left for the caller to
// mask.  With 64-bit shares: when bits [0, 2 l_x] fit in 32 bits a 32-bit
// shift of the low word, else (windows of at most 32 bits) one
// v_alignbit_b32 of the two halves does the variable shift.
template <typename T, int N, typename FT>
__device__ __forceinline__ FT window_low(T a, uint32_t pos) {
    if constexpr (sizeof(T) == 8 && 2 * N - 1 <= 32)     // bits [0, 2 l_x] fit in the low word
        return (FT)((uint32_t)a >> pos);
    else if constexpr (sizeof(T) == 8 && N <= 32)
        return (FT)__builtin_amdgcn_alignbit((uint32_t)(a >> 32), (uint32_t)a, pos);
    else
        return (FT)(a >> pos);
}

// Bits [pos, pos + l_x] of a share already shifted down by k_lo (pos <= l_x).
template <typename T, int N, typename FT>
__device__ __forceinline__ FT window(T a, uint32_t pos) {
    constexpr FT WIN1 = (FT)((2ull << (N - 1)) - 1);     // l_x + 1 bits
    return window_low<T, N, FT>(a, pos) & WIN1;
}

// a * b + c in Z_p with b and c given shifted left by SH bits (SH = 0: the
// plain values; see MaskDraws).  LAZY: a value below 2p congruent to it
// (the field's form without the final conditional subtraction).
template <int SH, typename F, bool LAZY = false>
__device__ __forceinline__ typename F::T field_mul_add(const F& f, typename F::T a, typename F::T b, typename F::T c) {
    if constexpr (LAZY) {
        if constexpr (SH == 0)
            return f.mul_add_lazy(a, b, c);
        else
            return f.template mul_add_sh_lazy<SH>(a, b, c);
    } else if constexpr (SH == 0) {
        return f.mul_add(a, b, c);
    } else {
        return f.template mul_add_sh<SH>(a, b, c);
    }
}

// P1's reshare addend p - z, kept shifted by SH like z, from a z whose low
// SH bits may carry stray bits (stream_draws): they are masked first.
template <int SH, typename F>
__device__ __forceinline__ typename F::T reshare_neg(const F& f, typename F::T z) {
    using FT = typename F::T;
    constexpr FT KEEP = (FT)~(((FT)1 << SH) - 1);
    return (FT)((f.p << SH) - (FT)(z & KEEP));
}

// Whether field F offers the lazy forms (a value below 2p with 4p < 2^32).
template <typename F, typename = void>
struct HasLazy : std::false_type {};
template <typename F>
struct HasLazy<F, std::void_t<decltype(F::kLazy)>> : std::integral_constant<bool, F::kLazy> {};

// v_min3_u32 written out: the compiler would otherwise re-associate P2's
// running minimum into a tree over all slots, which defers every slot's
// fold to the end and keeps all the products live at once.
__device__ __forceinline__ uint32_t min3_in_order(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t d;
    asm("v_min3_u32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// P2's running minimum over the slots of w0 + w1 mod p (a slot is zero
// exactly when its reconstruction is 0): without wrap, min(least, s, s - p)
// is one three-operand minimum, taken slot after slot.
template <typename F>
__device__ __forceinline__ typename F::T p2_least(typename F::T least, typename F::T w0, typename F::T w1, const F& f) {
    using FT = typename F::T;
    if constexpr (F::kWrap) {
        const FT w = addmod(w0, w1, f);
        FT m = w < least ? w : least;
        asm("" : "+v"(m));                          // slot by slot, as min3_in_order does
        return m;
    } else if constexpr (sizeof(FT) == 4) {
        const FT s = w0 + w1;
        return min3_in_order(least, s, s - f.p);
    } else {
        const FT s = w0 + w1;
        FT m = min(least, min(s, (FT)(s - f.p)));
        asm("" : "+v"(m));                          // slot by slot, as min3_in_order does
        return m;
    }
}

// P2's running minimum from two lazy messages w0, w1 < 2p (4p < 2^32): their
// sum t < 4p, u = t mod 2p by one conditional subtraction, then u and u - p
// into the minimum as in p2_least; u is 0 or p exactly when t is 0 mod p.
template <typename F>
__device__ __forceinline__ uint32_t p2_least_lazy(uint32_t least, uint32_t w0, uint32_t w1, const F& f) {
    const uint32_t t = w0 + w1;
    const uint32_t u = min(t, t - 2 * f.p);
    return min3_in_order(least, u, u - f.p);
}

// Windows through P2's reconstruction (Alg. 7) for one slot: the window
// position `pos` (sigma of the slot), the slot's mask r and reshare z (both
// shifted left by SH bits, see MaskDraws); returns both parties' messages
// and folds P2's reconstruction w0 + w1 mod p into its running minimum
// `least` (some slot is zero exactly when the minimum ends at 0).
// a0 and nb1 are P0's share and P1's negated share, both shifted down by k_lo.
// Every select is written as masks and adds so that it stays on the
// full-rate VOP2 forms (no compare / cndmask pairs).  With LAZY (callers
// that only test the slot, not capture its messages) and a field that has
// the lazy forms, w0 and w1 are left below 2p, one congruent value each, and
// P2 reduces their sum once.
// `next_w` is the width of u_{i+1}: l_x, or 0 when pos = l_x (u_{l_x+1} :=
// 0); the overload without it derives it from pos.
template <typename T, int N, typename F, int SH = 0, bool LAZY = false>
__device__ __forceinline__ void slot_messages(T a0, T nb1, uint32_t pos, uint32_t next_w, typename F::T r,
                                              typename F::T z, const F& f, typename F::T& w0, typename F::T& w1,
                                              typename F::T& least) {
    using FT = typename F::T;
    constexpr int LX = N - 1;
    constexpr FT TWO_LX = (FT)1 << LX;                   // 2^l_x mod p = 2^l_x
    constexpr FT WIN = TWO_LX - 1;                       // Z_{2^l_x}
    // W: bits [k_lo + pos, k_lo + pos + l_x] in bits [0, l_x]; with 32-bit
    // field elements the bits above are left in place, since u_{i+1} reads
    // bits [1, 1 + next_w) only and everything after is reduced mod 2^l_x
    FT W0, W1, u0n, u1n;                                 // u_{i+1}, and u_{l_x+1} := 0
    if constexpr (sizeof(FT) == 4) {
        W0 = window_low<T, N, FT>(a0, pos);
        W1 = window_low<T, N, FT>(nb1, pos);
        u0n = __builtin_amdgcn_ubfe(W0, 1, next_w);
        u1n = __builtin_amdgcn_ubfe(W1, 1, next_w);
    } else {
        W0 = window<T, N, FT>(a0, pos);
        W1 = window<T, N, FT>(nb1, pos);
        const FT more = (FT)0 - (FT)(next_w != 0);
        u0n = (W0 >> 1) & more;
        u1n = (W1 >> 1) & more;
    }
    // adjacent sum and modulo switch (Alg. 6) for P0: v0 = u_i + u_{i+1} - 1 in Z_{2^l_x},
    // s0 = v0, or 2^l_x when v0 = 0, which is ((v0 - 1) mod 2^l_x) + 1.
    const FT s0 = ((W0 + u0n - 2) & WIN) + 1;
    // P1: v1 = -(cut_i + cut_{i+1}) in Z_{2^l_x} and s1 = v1 + p - 2^l_x,
    // which is (p - 1) - ((cut_i + cut_{i+1} - 1) mod 2^l_x)
    const FT s1 = (f.p - 1) - ((W1 + u1n - 1) & WIN);
    if constexpr (LAZY && HasLazy<F>::value) {
        w0 = field_mul_add<SH, F, true>(f, s0, r, z);
        w1 = field_mul_add<SH, F, true>(f, s1, r, reshare_neg<SH>(f, z));
        least = p2_least_lazy(least, w0, w1, f);
    } else {
        w0 = field_mul_add<SH>(f, s0, r, z);                           // mask, reshare
        w1 = field_mul_add<SH>(f, s1, r, reshare_neg<SH>(f, z));       // P1: s1 r - z
        least = p2_least(least, w0, w1, f);                            // P2 reconstructs and tests
    }
}

template <typename T, int N, typename F, int SH = 0, bool LAZY = false>
__device__ __forceinline__ void slot_messages(T a0, T nb1, uint32_t pos, typename F::T r, typename F::T z, const F& f,
                                              typename F::T& w0, typename F::T& w1, typename F::T& least) {
    const uint32_t more_mask = (uint32_t)((int32_t)(pos - (uint32_t)(N - 1)) >> 31);   // all ones unless pos = l_x
    slot_messages<T, N, F, SH, LAZY>(a0, nb1, pos, (uint32_t)(N - 1) & more_mask, r, z, f, w0, w1, least);
}

// (-1)^t v mod 2^l for v < 2^l (Alg. 7's flip).  A select: the select-free
// form (v ^ -t) + t compiled to 36 more instructions and 74 VGPRs in the
// N = 19 DReLU kernel.
template <typename T>
__device__ __forceinline__ T flip_by(T v, uint32_t t, T mask) {
    return t ? (T)((T)0 - v) & mask : v;
}

// The shares a DReLU/ReLU works on, from the loaded ones: with k_in > 0 the
// loaded shares are of Z_{2^(l + k_in)} (in_mask) and each party first
// truncates its own by k_in bits (Alg. 5); with k_in = 0 and in_mask = mask
// the same expressions are the plain shares.  P0 holds in0 = cut(x0, k_in);
// P1 holds -n1 with n1 = cut(-x1, k_in), and n1, its negated share, is what it
// cuts the windows from (Alg. 7).
template <typename T>
__device__ __forceinline__ void input_shares(T x0, T x1, T mask, T in_mask, uint32_t k_in, T& in0, T& n1) {
    if (k_in == 0) {                                  // the plain shares (in_mask = mask): a uniform branch
        in0 = x0 & mask;
        n1 = (T)((T)0 - x1) & mask;
    } else {
        in0 = (T)((x0 & in_mask) >> k_in) & mask;
        n1 = (T)((((T)0 - x1) & in_mask) >> k_in) & mask;
    }
}

// DReLU's end (Alg. 7): P2's fresh sharing (rho, D' - rho), then the unflip:
// y0 = t + (1 - 2t) rho, y1 = (1 - 2t)(D' - rho), select-free with tm = -t
// (all ones when t = 1): (v ^ tm) - tm = (1 - 2t) v.  Each step keeps the low
// l bits a function of the low l bits, so rho may carry bits above l and one
// mask at the end reduces mod 2^l.
template <typename T>
__device__ __forceinline__ void drelu_finish(T dp, T rho, uint32_t t, T mask, T& y0, T& y1) {
    const T tm = (T)0 - (T)t;
    y0 = (T)((rho ^ tm) + (T)(2 * t)) & mask;          // t = 1: ~rho + 2 = 1 - rho
    y1 = (T)(((T)(dp - rho) ^ tm) - tm) & mask;
}

// Alg. 8's preprocessing draws of element g: [a]_0, [b]_0, [c]_0 from
// seed_02 (blocks 0 and 1 of TAG_BEAVER), [a]_1, [b]_1 from seed_12 (block 0);
// P2 forms [c]_1 = (a0 + a1)(b0 + b1) - c0 from them.
template <typename T>
__device__ __forceinline__ void beaver_shares(const Stream& s02, const Stream& s12, uint64_t g, T mask, T& ba0, T& bb0,
                                              T& bc0, T& ba1, T& bb1) {
    const StreamAt r02 = s02.at(g);
    const Words4 w0 = r02.block(TAG_BEAVER, 0);
    const Words4 w1 = r02.block(TAG_BEAVER, 1);
    const Words4 w2 = s12.block(g, TAG_BEAVER, 0);
    ba0 = (T)join64(w0.w0, w0.w1) & mask;
    bb0 = (T)join64(w0.w2, w0.w3) & mask;
    bc0 = (T)join64(w1.w0, w1.w1) & mask;
    ba1 = (T)join64(w2.w0, w2.w1) & mask;
    bb1 = (T)join64(w2.w2, w2.w3) & mask;
}

// Alg. 8 after the zero test: e = D' - b, d = x - a and the product, with
// the triple ([a]_j, [b]_j, [c]_j) and the unflipped inputs.
template <typename T>
__device__ __forceinline__ void relu_finish(T dp, T in0, T in1, T ba0, T bb0, T bc0, T ba1, T bb1, T bc1, uint32_t t,
                                            T mask, T& y0, T& y1) {
    const T ee = (T)(dp - (T)(bb0 + bb1)) & mask;                 // P2: e = D' - b
    const T dd = (T)((in0 - ba0) + (in1 - ba1)) & mask;           // P0, P1: d = x - a
    const T m0 = (T)(dd * ee + dd * bb0 + ee * ba0 + bc0) & mask; // de + d[b] + e[a] + [c]
    const T m1 = (T)(dd * bb1 + ee * ba1 + bc1) & mask;
    y0 = t ? (T)(in0 - m0) & mask : m0;                            // t[x] + (1 - 2t)[x D']
    y1 = t ? (T)(in1 - m1) & mask : m1;
}

// The flip bit t and the shuffle of one element, both from seed_01 (Alg. 7).
// N digits: t (radix 2), then j_i in [0, i] (radix i + 1) for i = 1..N-1, the
// choices of an inside-out Fisher-Yates shuffle: A[0] = 0, and for each i,
// A[i] = A[j_i], A[j_i] = i; slot s takes window position A[s].  The digits
// are cut from 64-bit chunks F of the TAG_SHUFFLE stream (chunk c: words
// 2 (c % 2) and 2 (c % 2) + 1 of block c / 2, low word first); a chunk takes
// digits in order while the product of their radices stays <= 2^32, and a
// digit of radix m is the part of F m above 2^64, F m mod 2^64 the next F.
template <int N>
struct ShufflePlan {
    int chunk[N];      // the chunk of digit k
    constexpr ShufflePlan() : chunk() {
        uint64_t prod = 1;
        int c = 0;
        for (int k = 0; k < N; ++k) {
            const uint64_t m = k == 0 ? 2 : (uint64_t)k + 1;
            if (prod * m > (1ull << 32)) {
                ++c;
                prod = 1;
            }
            prod *= m;
            chunk[k] = c;
        }
    }
};

// Runs the shuffle in this thread's slice of a per-block LDS array (blocks of
// at most 256 threads: every kernel is launched with __launch_bounds__(256))
// and returns the slice.  Entry A[k] is E bytes at byte k ROW of the slice,
// ROW = 256 E, so entry k of the 256 threads is one contiguous row and the
// address of a drawn index j is one multiply-add.  With E = 4 the 64 lanes of
// a wave touch 64 different banks whatever their k; E = 4 while 8 blocks of N
// rows fit the compute unit's 160 KiB of LDS (N <= 20), else E = 2.  Byte 0
// of an entry is the window position; its top byte is the width of the
// slot's next window u_{i+1}: 0 for the slot that received the top position
// l_x (u_{l_x+1} is 0; the last swap puts it at slot j_{N-1}, and nothing
// moves it after) and l_x for every other slot (shuffle_next_width).  The
// slice stays valid until the thread's next call.
template <int N>
struct ShuffleSlice {
    static constexpr int E = N <= 20 ? 4 : 2;               // bytes per entry
    static constexpr int ROW = 256 * E;
    using U = typename std::conditional<E == 4, uint32_t, uint16_t>::type;
    static constexpr U FLAG = (U)((U)(N - 1) << (8 * (E - 1)));  // top byte of a slot below l_x
};

template <int N>
__device__ __forceinline__ uint8_t* shuffle_fill(const StreamAt& r01, uint32_t& t) {
    using S = ShuffleSlice<N>;
    using U = typename S::U;
    constexpr ShufflePlan<N> plan{};
    __shared__ U lds[N * 256];
    uint8_t* A = reinterpret_cast<uint8_t*>(lds + threadIdx.x);
    Words4 w = {0, 0, 0, 0};
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int c = plan.chunk[k];
        if (k == 0 || plan.chunk[k > 0 ? k - 1 : 0] != c) {
            if (c % 2 == 0) w = r01.block(TAG_SHUFFLE, (uint32_t)(c / 2));
            lo = c % 2 ? w.w2 : w.w0;
            hi = c % 2 ? w.w3 : w.w1;
        }
        const uint32_t m = k == 0 ? 2u : (uint32_t)k + 1u;
        const uint64_t pl = (uint64_t)lo * m;
        const uint64_t ph = (uint64_t)hi * m + (uint32_t)(pl >> 32);
        lo = (uint32_t)pl;
        hi = (uint32_t)ph;
        uint32_t d = (uint32_t)(ph >> 32);                    // t, or j_k <= k
        if (k == 0) {
            t = d;
            *reinterpret_cast<U*>(A) = N == 1 ? (U)0 : S::FLAG;  // A[0] = 0
        } else {
            // d as a register of its own: the entry's address is then one
            // shift-add, where the compiler would otherwise cut d * ROW out
            // of the 64-bit product with an alignbit and a mask
            asm("" : "+v"(d));
            U* aj = reinterpret_cast<U*>(A + d * S::ROW);
            *reinterpret_cast<U*>(A + k * S::ROW) = *aj;        // A[k] = A[j_k]
            *aj = k == N - 1 ? (U)k : (U)(S::FLAG | (U)k);      // A[j_k] = k
        }
    }
    return A;
}

// The width of slot s's next window after shuffle_fill: l_x, or 0 for the
// slot of position l_x (the entry's top byte).
template <int N>
__device__ __forceinline__ uint32_t shuffle_next_width(const uint8_t* A, uint32_t s) {
    return A[s * ShuffleSlice<N>::ROW + ShuffleSlice<N>::E - 1];
}

// Window position of slot s after shuffle_fill.
template <int N>
__device__ __forceinline__ uint32_t shuffle_pos(const uint8_t* A, uint32_t s) {
    return A[s * ShuffleSlice<N>::ROW];
}

// The shuffle as words: byte q of perm[k] is the position of slot 4k + q
// (bytes past N zero).
template <int N>
__device__ __forceinline__ uint32_t shuffle_perm(const StreamAt& r01, uint32_t (&perm)[(N + 3) / 4]) {
    uint32_t t;
    const uint8_t* A = shuffle_fill<N>(r01, t);
#pragma unroll
    for (int k = 0; k < (N + 3) / 4; ++k) {
        uint32_t v = 0;
#pragma unroll
        for (int q = 0; q < 4 && 4 * k + q < N; ++q) v |= shuffle_pos<N>(A, (uint32_t)(4 * k + q)) << (8 * q);
        perm[k] = v;
    }
    return t;
}

// Layout of the masks r in Z_p^* and reshares z in Z_p of Alg. 7 in the
// seed_01 stream TAG_MASK, per window count N and field:
//  * the default prime at N >= 17 (STREAM): value v = 2s (r of slot s) or
//    2s + 1 (z of slot s) is the N-bit field at bits [N v, N v + N) of the
//    stream, whose bit i is bit i % 32 of word i / 32, word w being word
//    w % 4 of block w / 4; r = min(max(R, 1), p - 1), z = Z mod p.  Up to
//    N = 24 the kernels keep both shifted left by SH = 32 - N, which the
//    fields' mul_add_sh folds without a funnel shift.
//  * otherwise, p < 2^32: two slots to a block, words (0, 1) and (2, 3), by
//    32-bit multiply-shift; p > 2^32: one slot per block, 64-bit words.
template <int N, typename F>
struct MaskDraws {
    static constexpr bool WIDE = std::is_same<typename F::T, uint64_t>::value;
    static constexpr bool STREAM = F::kDefault && N >= 17;
    static constexpr int SPB = WIDE ? 1 : 2;                                            // slots per block otherwise
    static constexpr int NB = STREAM ? (2 * N * N + 127) / 128 : (N + SPB - 1) / SPB;   // blocks per element
    static constexpr int SH = STREAM && N <= 24 ? 32 - N : 0;                           // shift of the kept r and z
};

// r and z in the kept representation from the raw fields R, Z (STREAM,
// already shifted left by SH).
template <int N, typename F>
__device__ __forceinline__ void stream_draws(typename F::T R, typename F::T Z, typename F::T& r,
                                             typename F::T& z) {
    using FT = typename F::T;
    constexpr int SH = MaskDraws<N, F>::SH;
    constexpr FT KEEP = (FT)~(((FT)1 << SH) - 1);
    // r: clamp into Z_p^* (one v_med3); its low SH bits cleared, so that a
    // product r s has zero low SH bits.  z keeps whatever bits R and Z carry
    // below SH: an addend's low SH bits then stay below bit SH of a r + z
    // and never reach the folded value, and a subtraction from it masks them
    // first (reshare_neg).
    r = min(max((FT)(R & KEEP), (FT)((FT)1 << SH)), (FT)((FT)(F::p - 1) << SH));
    if constexpr (SH > 0 && F::p == (1ull << N) - 1)
        z = Z;                                      // Mersenne: Z <= p already stands for Z mod p
    else
        z = min(Z, (FT)(Z - ((FT)F::p << SH)));     // Z mod p (Z < 2p; the low SH bits decide nothing)
}

// Slot H's r and z of mask block w without STREAM (H < SPB, compile-time).
template <int N, typename F, int H>
__device__ __forceinline__ void block_draws(const Words4& w, const F& f, typename F::T& r, typename F::T& z) {
    if constexpr (MaskDraws<N, F>::WIDE) {
        r = 1 + __umul64hi(join64(w.w0, w.w1), f.p - 1);
        z = __umul64hi(join64(w.w2, w.w3), f.p);
    } else {
        r = draw_r(H ? w.w2 : w.w0, f.p);
        z = draw_z(H ? w.w3 : w.w1, f.p);
    }
}

// The masks of one element slot after slot (j compile-time after unrolling):
// with STREAM the block holding a field's last bit is fetched when the
// previous field ended in an earlier block, and that block's last word kept
// for a field that straddles the two (a field spans at most two words);
// otherwise block j / SPB is fetched at its first slot.  Every decision
// depends on j alone, so it folds away once the slot loop is unrolled.
template <int N, typename F>
struct MaskReader {
    using FT = typename F::T;
    using D = MaskDraws<N, F>;
    Words4 cur = {0, 0, 0, 0};
    uint32_t prev = 0;     // the last word of the block before cur

    // Word w of the stream, with block b current (w >= 4 b - 1).
    __device__ __forceinline__ uint32_t word(int w, int b) const {
        const int q = w - 4 * b;
        return q < 0 ? prev : q == 0 ? cur.w0 : q == 1 ? cur.w1 : q == 2 ? cur.w2 : cur.w3;
    }
    // The raw field of value v (shifted left by SH; with SH > 0 the low SH
    // bits are left as they come, see stream_draws).
    __device__ __forceinline__ FT field(const StreamAt& r01, int v) {
        const int o = N * v;
        const int b = (o + N - 1) / 128;                    // the block of the field's last bit
        if (o == 0 || (o - 1) / 128 != b) {                 // the previous field ended in an earlier block
            prev = cur.w3;
            cur = r01.block(TAG_MASK, (uint32_t)b);
        }
        if constexpr (D::SH > 0) {
            const int lo = o + N - 32;              // the field is the top of the word [lo, lo + 32)
            if (lo < 0) return word(0, b) << D::SH;
            const int k = lo / 32, s = lo % 32;
            if (s == 0) return word(k, b);
            return __builtin_amdgcn_alignbit(word(k + 1, b), word(k, b), s);
        } else if constexpr (D::WIDE) {
            const int k = o / 32, s = o % 32;       // 33 bits: always two words
            return (join64(word(k, b), word(k + 1, b)) >> s) & ((1ull << N) - 1);
        } else {
            const int k = o / 32, s = o % 32;
            constexpr uint32_t M = N >= 32 ? ~0u : (1u << N) - 1;
            if (s + N <= 32) return (word(k, b) >> s) & M;
            return __builtin_amdgcn_alignbit(word(k + 1, b), word(k, b), s) & M;
        }
    }
    __device__ __forceinline__ void slot(const StreamAt& r01, int j, const F& f, FT& r, FT& z) {
        if constexpr (D::STREAM) {
            const FT R = field(r01, 2 * j);
            const FT Z = field(r01, 2 * j + 1);
            stream_draws<N, F>(R, Z, r, z);
        } else {
            constexpr int SPB = D::SPB;
            if (j % SPB == 0) cur = r01.block(TAG_MASK, (uint32_t)(j / SPB));
            if (j % SPB == 0)
                block_draws<N, F, 0>(cur, f, r, z);
            else
                block_draws<N, F, (SPB > 1 ? 1 : 0)>(cur, f, r, z);
        }
    }
};

// The raw field of value v (STREAM) from a group's words in LDS: W[-1] and
// W[4 NB] are zero, so every read stays inside the array.
template <int N, typename F>
__device__ __forceinline__ typename F::T stream_field_at(const uint32_t* W, uint32_t v) {
    using D = MaskDraws<N, F>;
    const int o = N * (int)v;
    if constexpr (D::SH > 0) {
        const int lo = o + N - 32;                  // > -32
        const int k = ((lo + 32) >> 5) - 1;         // floor(lo / 32): -1 for v = 0
        return __builtin_amdgcn_alignbit(W[k + 1], W[k], (uint32_t)lo & 31u);   // low SH bits as they come
    } else if constexpr (D::WIDE) {
        const int k = o >> 5;
        return (join64(W[k], W[k + 1]) >> (o & 31)) & ((1ull << N) - 1);
    } else {
        const int k = o >> 5;
        constexpr uint32_t M = N >= 32 ? ~0u : (1u << N) - 1;
        return __builtin_amdgcn_alignbit(W[k + 1], W[k], (uint32_t)o & 31u) & M;
    }
}

// Plain canonical values of kept draws (the record of the precomputed mode).
template <int N, typename F>
__device__ __forceinline__ void plain_draws(const F& f, typename F::T& r, typename F::T& z) {
    constexpr int SH = MaskDraws<N, F>::SH;
    if constexpr (SH > 0) {
        r >>= SH;
        z >>= SH;
        z = min(z, z - f.p);                        // a Mersenne Z = p stands for 0
    }
}

// Alg. 7 from the flip through P2's zero test for one element: the 2-of-2
// input (in0, -n1) of Z_{2^l} (n1: P1's negated share, see input_shares),
// randomness of global index g.  Returns D'
// (1 when some slot reconstructs to 0) and the flip bit t.  With CAP the
// round-1 messages go to cap[e * N + slot] (P0) and cap[(ncap + e) * N +
// slot] (P1).
template <typename T, int N, typename F, bool CAP>
__device__ __forceinline__ T drelu_round1(T in0, T n1, uint64_t g, T mask, uint32_t k_lo, const Stream& s01,
                                          typename F::T* cap, uint64_t ncap, uint64_t e, const F& f,
                                          uint32_t& t_out) {
    using FT = typename F::T;
    constexpr bool WIDE = std::is_same<FT, uint64_t>::value;
    static_assert(WIDE == (N == 33), "64-bit field elements exactly when l_x = 32");

    // The flip bit t and the shuffle, both from seed_01.
    const StreamAt r01 = s01.at(g);
    uint32_t t;
    const uint8_t* A = shuffle_fill<N>(r01, t);

    // Flip: [x] := (-1)^t [x]  (both parties); P1 cuts its negated share
    // -(-1)^t [x]_1 = (-1)^t n1.
    const T a0 = flip_by(in0, t, mask);
    const T nb1 = flip_by(n1, t, mask);
    const T a0k = a0 >> k_lo, nb1k = nb1 >> k_lo;         // common low cut of every window

    FT least = f.p;                                        // P2: min over slots of w0 + w1 mod p
    MaskReader<N, F> masks;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        // Mask r and reshare z of slot j.
        FT r, z;
        masks.slot(r01, j, f, r, z);
        FT w0, w1;
        slot_messages<T, N, F, MaskDraws<N, F>::SH, !CAP>(a0k, nb1k, shuffle_pos<N>(A, j), shuffle_next_width<N>(A, j), r, z,
                                                          f, w0, w1, least);
        if constexpr (CAP) {
            cap[e * N + j] = w0;
            cap[(ncap + e) * N + j] = w1;
        }
    }
    t_out = t;
    return least == 0 ? 1 : 0;                             // D' = [some slot is 0]
}

// One element, all three parties.  N = l_x + 1 windows, fixed at compile
// time: every loop over windows and slots is unrolled and all window masks
// are constants.  From the loaded shares x0, x1 to the output shares y0,
// y1; the randomness belongs to global index g, and e is the element's
// index in the call (for the capture).  With CAP, the round-1 messages are captured
// (drelu_round1).  With k_in > 0 the inputs are shares of Z_{2^(l + k_in)}
// (in_mask) and are first truncated by k_in bits into Z_{2^l} (Alg. 5); with
// k_in = 0 and in_mask = mask the same expressions are the plain load.
template <typename T, int N, typename F, bool RELU, bool CAP>
__device__ __forceinline__ void drelu_element_of(T x0, T x1, T& y0, T& y1, typename F::T* cap, uint64_t ncap,
                                                 uint64_t e, uint64_t g, T mask, T in_mask, uint32_t k_in,
                                                 uint32_t k_lo, const Stream& s01, const Stream& s02,
                                                 const Stream& s12, const F& f) {
    T in0, n1;
    input_shares<T>(x0, x1, mask, in_mask, k_in, in0, n1);

    uint32_t t;
    const T dp = drelu_round1<T, N, F, CAP>(in0, n1, g, mask, k_lo, s01, cap, ncap, e, f, t);

    if constexpr (!RELU) {
        const Words4 w = s02.block(g, TAG_RESP, 0);               // rho from seed_02
        drelu_finish<T>(dp, (T)join64(w.w0, w.w1), t, mask, y0, y1);
    } else {
        const T in1 = (T)((T)0 - n1) & mask;
        // Alg. 8 preprocessing; P2 forms [c]_1 = (a0 + a1)(b0 + b1) - c0.
        T ba0, bb0, bc0, ba1, bb1;
        beaver_shares<T>(s02, s12, g, mask, ba0, bb0, bc0, ba1, bb1);
        const T bc1 = (T)((T)(ba0 + ba1) * (T)(bb0 + bb1) - bc0) & mask;
        relu_finish<T>(dp, in0, in1, ba0, bb0, bc0, ba1, bb1, bc1, t, mask, y0, y1);
    }
}

// drelu_element_of from X0[e], X1[e] to Y0[e], Y1[e].
template <typename T, int N, typename F, bool RELU, bool CAP>
__device__ __forceinline__ void drelu_element(const T* __restrict__ X0, const T* __restrict__ X1, T* Y0, T* Y1,
                                              typename F::T* cap, uint64_t ncap, uint64_t e, uint64_t g, T mask,
                                              T in_mask, uint32_t k_in, uint32_t k_lo, const Stream& s01,
                                              const Stream& s02, const Stream& s12, const F& f) {
    T y0, y1;
    drelu_element_of<T, N, F, RELU, CAP>(ld_nt(&X0[e]), ld_nt(&X1[e]), y0, y1, cap, ncap, e, g, mask, in_mask, k_in,
                                         k_lo, s01, s02, s12, f);
    st_nt(&Y0[e], y0);
    st_nt(&Y1[e], y1);
}

// Elements of one k_drelu launch: at most 2^28, so that element indices and
// byte offsets (and an index plus the grid's stride) stay in 32 bits; the
// host runs a larger call as launches over consecutive ranges, each with
// its own element offset, which gives the results of one launch.
constexpr uint64_t kLaunchElems = 1ull << 28;

// Element i of p, addressed as p plus a 32-bit byte offset (the load or
// store then takes p from scalar registers and the offset from one VGPR),
// nontemporal (ld_nt / st_nt).
template <typename T>
__device__ __forceinline__ T load_at(const T* p, uint32_t i) {
    return ld_nt(reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + (uint32_t)(i * (uint32_t)sizeof(T))));
}
template <typename T>
__device__ __forceinline__ void store_at(T* p, uint32_t i, T v) {
    st_nt(reinterpret_cast<T*>(reinterpret_cast<char*>(p) + (uint32_t)(i * (uint32_t)sizeof(T))), v);
}

// Element i of the buffer r (a raw buffer of 4- or 8-byte elements), loaded
// nontemporal; an element past the buffer's end reads as 0 without a memory
// access (the buffer's range check).
template <typename T>
__device__ __forceinline__ T load_buf(__amdgpu_buffer_rsrc_t r, uint32_t i) {
    constexpr int kNontemporal = 2;
    if constexpr (sizeof(T) == 8) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, i * 8u, 0, kNontemporal);
        return (T)w[0] | ((T)w[1] << 32);
    } else {
        return (T)__builtin_amdgcn_raw_buffer_load_b32(r, i * 4u, 0, kNontemporal);
    }
}

// A raw buffer over n elements of T at p (word 3: the gfx9 data format of
// raw, unswizzled buffers).
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const T* p, uint32_t n) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), (short)0, (int)(n * (uint32_t)sizeof(T)), 0x00020000);
}

// The loop of one k_drelu launch (see k_drelu), with the ring mask given.
template <typename T, int N, typename F, bool RELU, bool CAP>
__device__ __forceinline__ void drelu_launch_loop(const DreluKArgs& A, const F& f, T mask) {
    const T* X0 = static_cast<const T*>(A.x0);
    const T* X1 = static_cast<const T*>(A.x1);
    T* Y0 = static_cast<T*>(A.y0);
    T* Y1 = static_cast<T*>(A.y1);
    typename F::T* cap = static_cast<typename F::T*>(A.cap);
    const uint32_t n = (uint32_t)A.n;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const __amdgpu_buffer_rsrc_t B0 = buffer_of(X0, n), B1 = buffer_of(X1, n);
    T x0 = load_at(X0, e), x1 = load_at(X1, e);
    // Wait for the first shares before the loop: its head then waits on no
    // memory operation (later entries have only the last stores outstanding).
    asm volatile("" : "+v"(x0), "+v"(x1));
    for (;;) {
        const uint32_t en = e + stride;
        const T x0n = load_buf<T>(B0, en), x1n = load_buf<T>(B1, en);   // past the last: 0, no access
        T y0, y1;
        drelu_element_of<T, N, F, RELU, CAP>(x0, x1, y0, y1, cap, A.ncap, e, A.elem_base + e, mask, (T)A.in_mask,
                                             A.k_in, A.k_lo, A.s01, A.s02, A.s12, f);
        store_at(Y0, e, y0);
        store_at(Y1, e, y1);
        if (en >= n) break;
        e = en;
        x0 = x0n;
        x1 = x1n;
    }
}

// One launch: grid-stride over its n <= kLaunchElems elements of one share
// pair.  Each thread loads its next element's shares before computing the
// current one, so the loads have a whole element's work to land: with other
// traffic on the memory system (the truncation beside it), a load at the top
// of each element stalled the kernel.
template <typename T, int N, typename F, bool RELU, bool CAP>
__global__ BC_KERNEL_ATTRS void k_drelu(DreluKArgs A, F f_arg) {
    const F f = f_arg.vgpr();
    // A full-width ring (l = 64 in 64-bit storage, l = 32 in 32-bit) makes
    // every reduction mod 2^l a no-op: that loop runs with the mask as a
    // constant, so the compiler drops the masking instructions.
    if constexpr (!CAP) {
        if ((T)A.ring_mask == (T)~(T)0) {
            drelu_launch_loop<T, N, F, RELU, CAP>(A, f, (T)~(T)0);
            return;
        }
    }
    drelu_launch_loop<T, N, F, RELU, CAP>(A, f, in_vgpr((T)A.ring_mask));
}

// Lane groups for small calls: G consecutive lanes share one element, so a
// call of n elements still runs n * G threads.  Every lane of the group runs
// the whole shuffle in its own LDS slice.  Without STREAM lane l takes mask
// block kG + l in round k and its slots (two, or one when l_x = 32); with
// STREAM the lanes draw the blocks the same way into the group's words in
// LDS and lane l then takes slots kG + l, reading its fields from there.
// The group's P2 minimum is combined by lane shuffles; lane 0 finishes and
// writes.  Results are those of drelu_element: same draws, same slots, same
// messages.
template <typename T, int N, typename F, bool RELU, int G>
__device__ __forceinline__ void drelu_element_group(const T* __restrict__ X0, const T* __restrict__ X1, T* Y0, T* Y1,
                                                    uint64_t e, uint64_t g, uint32_t lane, T mask, T in_mask,
                                                    uint32_t k_in, uint32_t k_lo, const Stream& s01,
                                                    const Stream& s02, const Stream& s12, const F& f) {
    using FT = typename F::T;
    using D = MaskDraws<N, F>;
    constexpr bool WIDE = D::WIDE;
    constexpr int SPB = D::SPB;                             // slots per mask block without STREAM
    constexpr int SH = D::SH;
    constexpr int NB = D::NB;                               // mask blocks
    constexpr int ROUNDS = (NB + G - 1) / G;

    T in0, n1;
    input_shares<T>(ld_nt(&X0[e]), ld_nt(&X1[e]), mask, in_mask, k_in, in0, n1);

    const StreamAt r01 = s01.at(g);
    uint32_t t;
    const uint8_t* A = shuffle_fill<N>(r01, t);

    const T a0 = flip_by(in0, t, mask);                  // the flip, as in drelu_round1
    const T nb1 = flip_by(n1, t, mask);
    const T a0k = a0 >> k_lo, nb1k = nb1 >> k_lo;

    FT least = f.p;
    if constexpr (D::STREAM) {
        // The group's 4 NB stream words, with a zero word on either side.
        constexpr int STRIDE = 4 * NB + 2;
        __shared__ uint32_t mw[(256 / G) * STRIDE];
        uint32_t* W = mw + (threadIdx.x / G) * STRIDE + 1;
        if (lane == 0) {
            W[-1] = 0;
            W[4 * NB] = 0;
        }
#pragma unroll
        for (int k = 0; k < ROUNDS; ++k) {
            const uint32_t blk = (uint32_t)(k * G) + lane;
            if (blk < (uint32_t)NB) {
                const Words4 w = r01.block(TAG_MASK, blk);
                W[4 * blk] = w.w0;
                W[4 * blk + 1] = w.w1;
                W[4 * blk + 2] = w.w2;
                W[4 * blk + 3] = w.w3;
            }
        }
        wave_sync();                                        // the group's words before its reads
#pragma unroll
        for (int k = 0; k < (N + G - 1) / G; ++k) {
            const uint32_t j = (uint32_t)(k * G) + lane;
            const bool valid = j < (uint32_t)N;
            const uint32_t js = valid ? j : 0u;             // past the last slot: any slot, not counted
            FT r, z;
            stream_draws<N, F>(stream_field_at<N, F>(W, 2 * js), stream_field_at<N, F>(W, 2 * js + 1), r, z);
            FT w0, w1, v = f.p;
            slot_messages<T, N, F, SH, true>(a0k, nb1k, shuffle_pos<N>(A, js), shuffle_next_width<N>(A, js), r, z, f, w0, w1,
                                             v);
            least = (valid && v < least) ? v : least;
        }
        wave_sync();                                        // every read before the next element's words
    } else {
#pragma unroll
        for (int k = 0; k < ROUNDS; ++k) {
            const uint32_t blk = (uint32_t)(k * G) + lane;  // this lane's mask block
            const Words4 w = r01.block(TAG_MASK, blk);
#pragma unroll
            for (int h = 0; h < SPB; ++h) {
                // slot j = SPB * blk + h (past the last slot: any slot, its message is not counted)
                const bool valid = SPB * blk + h < (uint32_t)N;
                const uint32_t js = valid ? SPB * blk + h : 0u;
                const uint32_t pos = shuffle_pos<N>(A, js);
                FT r, z;
                if (h == 0)
                    block_draws<N, F, 0>(w, f, r, z);
                else
                    block_draws<N, F, (SPB > 1 ? 1 : 0)>(w, f, r, z);
                FT w0, w1, v = f.p;
                slot_messages<T, N, F, SH, true>(a0k, nb1k, pos, shuffle_next_width<N>(A, js), r, z, f, w0, w1, v);
                least = (valid && v < least) ? v : least;
            }
        }
    }
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        if constexpr (WIDE) {
            const uint32_t lo = __shfl_xor((uint32_t)least, o, G), hi = __shfl_xor((uint32_t)(least >> 32), o, G);
            const FT other = join64(lo, hi);
            least = other < least ? other : least;
        } else {
            const FT other = (FT)__shfl_xor((uint32_t)least, o, G);
            least = other < least ? other : least;
        }
    }
    const T dp = least == 0 ? 1 : 0;

    T y0, y1;
    if constexpr (!RELU) {
        const Words4 w = s02.block(g, TAG_RESP, 0);
        drelu_finish<T>(dp, (T)join64(w.w0, w.w1), t, mask, y0, y1);
    } else {
        const T in1 = (T)((T)0 - n1) & mask;
        const StreamAt r02 = s02.at(g);
        const Words4 w0 = r02.block(TAG_BEAVER, 0);
        const Words4 w1 = r02.block(TAG_BEAVER, 1);
        const Words4 w2 = s12.block(g, TAG_BEAVER, 0);
        const T ba0 = (T)join64(w0.w0, w0.w1) & mask;
        const T bb0 = (T)join64(w0.w2, w0.w3) & mask;
        const T bc0 = (T)join64(w1.w0, w1.w1) & mask;
        const T ba1 = (T)join64(w2.w0, w2.w1) & mask;
        const T bb1 = (T)join64(w2.w2, w2.w3) & mask;
        const T bc1 = (T)((T)(ba0 + ba1) * (T)(bb0 + bb1) - bc0) & mask;
        relu_finish<T>(dp, in0, in1, ba0, bb0, bc0, ba1, bb1, bc1, t, mask, y0, y1);
    }
    if (lane == 0) {
        st_nt(&Y0[e], y0);
        st_nt(&Y1[e], y1);
    }
}

// Lane-group launch: thread t serves element t / G as lane t % G.  Every lane
// of a group is active or inactive together (the loop bound is per element),
// so the shuffles only read lanes that take part.
template <typename T, int N, typename F, bool RELU, int G>
__global__ BC_KERNEL_ATTRS void k_drelu_group(DreluKArgs A, F f_arg) {
    static_assert(G >= 2 && (G & (G - 1)) == 0 && 256 % G == 0, "G: a power of two dividing the block");
    const F f = f_arg.vgpr();
    const T* X0 = static_cast<const T*>(A.x0);
    const T* X1 = static_cast<const T*>(A.x1);
    T* Y0 = static_cast<T*>(A.y0);
    T* Y1 = static_cast<T*>(A.y1);
    const T mask = in_vgpr((T)A.ring_mask);
    const uint32_t lane = threadIdx.x & (G - 1);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t total = A.n * G;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const uint64_t e = t / G;
        drelu_element_group<T, N, F, RELU, G>(X0, X1, Y0, Y1, e, A.elem_base + e, lane, mask, (T)A.in_mask, A.k_in,
                                              A.k_lo, A.s01, A.s02, A.s12, f);
    }
}

// Host helpers: field parameters for each prime size.
inline FieldSmall make_field_small(uint64_t p) { return FieldSmall{(uint32_t)p, 1.0f / (float)p}; }
inline Field24 make_field24(uint64_t p) { return Field24{(uint32_t)p, (double)p, 1.0 / (double)p}; }
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
    A.ncap = L.n;
    A.elem_base = L.elem_base;
    A.ring_mask = L.ell >= 64 ? ~0ull : ((1ull << L.ell) - 1);
    A.in_mask = L.ell + L.k_in >= 64 ? ~0ull : ((1ull << (L.ell + L.k_in)) - 1);
    A.k_lo = L.k_lo;
    A.k_in = L.k_in;
    A.s01 = Stream{L.s01.k0, L.s01.k1, L.s01.n0, L.s01.n1};
    A.s02 = Stream{L.s02.k0, L.s02.k1, L.s02.n0, L.s02.n1};
    A.s12 = Stream{L.s12.k0, L.s12.k1, L.s12.n0, L.s12.n1};
    return A;
}

template <typename T, int N, typename F, bool RELU>
hipError_t launch_field(const DreluLaunch& L, const F& f, hipStream_t st) {
    const DreluKArgs A = make_kargs(L);
    if (L.group == 8)
        hipLaunchKernelGGL((k_drelu_group<T, N, F, RELU, 8>), dim3(L.grid), dim3(L.block), 0, st, A, f);
    else if (L.group == 4)
        hipLaunchKernelGGL((k_drelu_group<T, N, F, RELU, 4>), dim3(L.grid), dim3(L.block), 0, st, A, f);
    else {
        // consecutive ranges of at most kLaunchElems elements
        for (uint64_t off = 0; off < L.n; off += kLaunchElems) {
            DreluKArgs R = A;
            R.n = L.n - off < kLaunchElems ? L.n - off : kLaunchElems;
            R.x0 = static_cast<const T*>(A.x0) + off;
            R.x1 = static_cast<const T*>(A.x1) + off;
            R.y0 = static_cast<T*>(A.y0) + off;
            R.y1 = static_cast<T*>(A.y1) + off;
            R.elem_base = A.elem_base + off;
            if (L.cap) {
                R.cap = static_cast<typename F::T*>(A.cap) + off * N;
                hipLaunchKernelGGL((k_drelu<T, N, F, RELU, true>), dim3(L.grid), dim3(L.block), 0, st, R, f);
            } else {
                hipLaunchKernelGGL((k_drelu<T, N, F, RELU, false>), dim3(L.grid), dim3(L.block), 0, st, R, f);
            }
            const hipError_t err = hipGetLastError();
            if (err != hipSuccess) return err;
        }
        return hipSuccess;
    }
    return hipGetLastError();
}

constexpr bool mersenne_exponent(int k) { return k == 13 || k == 17 || k == 19; }   // 2^k - 1 prime, 12 < k <= 24

// Calls fn(field) with the Z_p arithmetic for N = l_x + 1 (p has N bits):
// for the default primes the Mersenne fold (2^13 - 1, 2^17 - 1, 2^19 - 1)
// or the pseudo-Mersenne folds (every other default prime up to 2^33); for
// any other prime fp32-quotient 24-bit products (p < 2^12), an fp64
// quotient (p < 2^24), Barrett (p < 2^32), or the 128-bit product with an
// fp64 quotient (l_x = 32).
template <int N, typename Fn>
hipError_t with_field(uint64_t p, Fn&& fn) {
    if constexpr (N <= 12) {
        if (p == (1ull << N) - kPrimeDelta[N]) return fn(FieldPM<N, kPrimeDelta[N]>{});
        return fn(make_field_small(p));
    } else if constexpr (N <= 32) {
        if constexpr (mersenne_exponent(N)) {
            if (p == (1ull << N) - 1) return fn(FieldMersenne<N>{});
        } else {
            if (p == (1ull << N) - kPrimeDelta[N]) return fn(FieldPM<N, kPrimeDelta[N]>{});
        }
        if constexpr (N <= 24)
            return fn(make_field24(p));
        else
            return fn(make_field32(p));
    } else {
        if (p == (1ull << 33) - kPrimeDelta[33]) return fn(FieldPM33{});
        return fn(make_field64(p));
    }
}

// The field type follows from N = l_x + 1 (p has N bits), and from p itself
// when p is a Mersenne prime.
template <typename T, int N, bool RELU>
hipError_t launch_exact(const DreluLaunch& L, hipStream_t st) {
    return with_field<N>(L.p, [&](auto f) { return launch_field<T, N, decltype(f), RELU>(L, f, st); });
}

template <typename T, bool RELU, int NLO, int NHI>
hipError_t launch_range(const DreluLaunch& L, hipStream_t st) {
    if constexpr (NLO > NHI) {
        return hipErrorInvalidValue;
    } else {
        if (L.npos == (uint32_t)NLO) return launch_exact<T, NLO, RELU>(L, st);
        return launch_range<T, RELU, NLO + 1, NHI>(L, st);
    }
}

}  // namespace bc
