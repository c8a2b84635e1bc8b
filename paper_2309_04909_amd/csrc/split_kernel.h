// The DReLU (Alg. 7) with the parties apart: each party's part as its own
// kernel, the round-1 messages bit-packed as they would cross a link.
//
//   k_send<P>   P0 or P1 alone, from its own share: flip, windows, adjacent
//               sums, modulo switch, shuffle, mask and reshare (the same
//               draws and slot arithmetic as the fused kernel), then the N
//               slot values of N bits each packed into ceil(N^2 / 32) words:
//               bit b of slot s is bit s N + b of the element's string, word
//               k holds bits 32k .. 32k + 31, stored word-major (msg[k n + i])
//               so that every word plane is one coalesced stream.
//   k_reply     P2: unpacks both messages, reconstructs every slot, D' = [some
//               slot is 0], and writes its reply shares (rho, D' - rho).
//   k_finish<P> P0 or P1 unflips its reply share with t.
// Every step before P2 uses one share only, so k_send reads one array.
#pragma once

#include "drelu_kernel.h"

namespace bc {

struct SplitKArgs {
    const void* in0;      // send: the party's share; reply: P0's message; finish: the reply share
    const void* in1;      // reply: P1's message
    void* out0;           // send: the message; reply: P0's reply share; finish: the output share
    void* out1;           // reply: P1's reply share
    uint64_t n, elem_base, ring_mask;
    uint32_t k_lo;
    Stream s01, s02;
};

// One party's message for one slot (the P0 or P1 half of slot_messages).
// ak: the party's flipped share (P1: its negation) shifted down by k_lo; r
// and z in the kept representation of MaskDraws (shifted left by SH).
template <typename T, int N, typename F, int PARTY, int SH = MaskDraws<N, F>::SH>
__device__ __forceinline__ typename F::T party_message(T ak, uint32_t pos, typename F::T r, typename F::T z,
                                                       const F& f) {
    using FT = typename F::T;
    constexpr int LX = N - 1;
    constexpr FT TWO_LX = (FT)1 << LX;
    constexpr FT WIN = TWO_LX - 1;
    const FT Wv = window<T, N, FT>(ak, pos);
    const FT more = (FT)(int64_t)((int32_t)(pos - (uint32_t)LX) >> 31);
    const FT un = (Wv >> 1) & more;                                   // u_{i+1}, u_{l_x+1} := 0
    if constexpr (PARTY == 0) {
        const FT s0 = ((Wv + un - 2) & WIN) + 1;                     // v0, or 2^l_x when v0 = 0
        return field_mul_add<SH>(f, s0, r, z);
    } else {
        const FT s1 = (f.p - 1) - ((Wv + un - 1) & WIN);             // v1 + p - 2^l_x, v1 = -(Wv + un)
        return field_mul_add<SH>(f, s1, r, reshare_neg<SH>(f, z));
    }
}

template <int N>
struct Packing {
    static constexpr int W = (N * N + 31) / 32;
};

// OR an N-bit value into the element's words at bit offset j N (j constant
// after unrolling, so every index and shift is too).
template <int N>
__device__ __forceinline__ void pack_slot(uint32_t (&w)[Packing<N>::W], int j, uint64_t v) {
    const int off = j * N, wi = off >> 5, sh = off & 31;
    w[wi] |= (uint32_t)(v << sh);
    if (sh + N > 32 && wi + 1 < Packing<N>::W) w[wi + 1] |= (uint32_t)(v >> (32 - sh));
}

template <int N>
__device__ __forceinline__ uint64_t unpack_slot(const uint32_t (&w)[Packing<N>::W], int j) {
    const int off = j * N, wi = off >> 5, sh = off & 31;
    uint64_t v = (uint64_t)w[wi] >> sh;
    if (sh + N > 32 && wi + 1 < Packing<N>::W) v |= (uint64_t)w[wi + 1] << (32 - sh);
    return v & ((1ull << N) - 1);
}

template <typename T, int N, typename F, int PARTY>
__global__ BC_KERNEL_ATTRS void k_send(SplitKArgs A, F f_arg) {
    using FT = typename F::T;
    constexpr int W = Packing<N>::W;
    const F f = f_arg.vgpr();
    const T* X = static_cast<const T*>(A.in0);
    uint32_t* M = static_cast<uint32_t*>(A.out0);
    const T mask = in_vgpr((T)A.ring_mask);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < A.n; e += stride) {
        const uint64_t g = A.elem_base + e;
        const T x = X[e] & mask;
        const StreamAt r01 = A.s01.at(g);
        uint32_t t;
        const uint8_t* sig = shuffle_fill<N>(r01, t);
        // the flipped share (-1)^t x; P1 cuts its negation (-1)^(t+1) x
        const T ak = flip_by(x, PARTY == 0 ? t : t ^ 1u, mask) >> A.k_lo;
        uint32_t words[W];
#pragma unroll
        for (int k = 0; k < W; ++k) words[k] = 0;
        MaskReader<N, F> masks;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            FT r, z;
            masks.slot(r01, j, f, r, z);
            pack_slot<N>(words, j, (uint64_t)party_message<T, N, F, PARTY>(ak, shuffle_pos<N>(sig, j), r, z, f));
        }
#pragma unroll
        for (int k = 0; k < W; ++k) st_nt(&M[(uint64_t)k * A.n + e], words[k]);
    }
}

template <typename T, int N, typename F>
__global__ BC_KERNEL_ATTRS void k_reply(SplitKArgs A, F f_arg) {
    using FT = typename F::T;
    constexpr int W = Packing<N>::W;
    const F f = f_arg.vgpr();
    const uint32_t* M0 = static_cast<const uint32_t*>(A.in0);
    const uint32_t* M1 = static_cast<const uint32_t*>(A.in1);
    T* D0 = static_cast<T*>(A.out0);
    T* D1 = static_cast<T*>(A.out1);
    const T mask = in_vgpr((T)A.ring_mask);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < A.n; e += stride) {
        uint32_t w0[W], w1[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            w0[k] = ld_nt(&M0[(uint64_t)k * A.n + e]);
            w1[k] = ld_nt(&M1[(uint64_t)k * A.n + e]);
        }
        FT least = f.p;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const FT v = addmod((FT)unpack_slot<N>(w0, j), (FT)unpack_slot<N>(w1, j), f);
            least = v < least ? v : least;
        }
        const T dp = least == 0 ? 1 : 0;                              // D'
        const Words4 w = A.s02.block(A.elem_base + e, TAG_RESP, 0);    // rho from seed_02
        const T rho = (T)join64(w.w0, w.w1) & mask;
        st_nt(&D0[e], rho);
        st_nt(&D1[e], (T)((T)(dp - rho) & mask));
    }
}

template <typename T, int PARTY>
__global__ __launch_bounds__(256) void k_finish(SplitKArgs A) {
    const T* D = static_cast<const T*>(A.in0);
    T* Y = static_cast<T*>(A.out0);
    const T mask = (T)A.ring_mask;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < A.n; e += stride) {
        // t is the shuffle's first digit (radix 2) of chunk 0: the top bit of its high word
        const uint32_t t = A.s01.block(A.elem_base + e, TAG_SHUFFLE, 0).w1 >> 31;
        const T d = D[e] & mask;
        if constexpr (PARTY == 0)
            Y[e] = (T)((d ^ ((T)0 - (T)t)) + (T)(2 * t)) & mask;      // t + (1 - 2t) d
        else
            Y[e] = flip_by(d, t, mask);                              // (1 - 2t) d
    }
}

inline SplitKArgs make_split_kargs(const SplitLaunch& L) {
    SplitKArgs A;
    A.in0 = L.in0;
    A.in1 = L.in1;
    A.out0 = L.out0;
    A.out1 = L.out1;
    A.n = L.n;
    A.elem_base = L.elem_base;
    A.ring_mask = L.ell >= 64 ? ~0ull : ((1ull << L.ell) - 1);
    A.k_lo = L.k_lo;
    A.s01 = Stream{L.s01.k0, L.s01.k1, L.s01.n0, L.s01.n1};
    A.s02 = Stream{L.s02.k0, L.s02.k1, L.s02.n0, L.s02.n1};
    return A;
}

template <typename T, int N>
hipError_t launch_split_exact(const SplitLaunch& L, hipStream_t st) {
    const SplitKArgs A = make_split_kargs(L);
    return with_field<N>(L.p, [&](auto f) {
        using F = decltype(f);
        if (L.kind == SplitLaunch::SEND && L.party == 0)
            hipLaunchKernelGGL((k_send<T, N, F, 0>), dim3(L.grid), dim3(256), 0, st, A, f);
        else if (L.kind == SplitLaunch::SEND)
            hipLaunchKernelGGL((k_send<T, N, F, 1>), dim3(L.grid), dim3(256), 0, st, A, f);
        else
            hipLaunchKernelGGL((k_reply<T, N, F>), dim3(L.grid), dim3(256), 0, st, A, f);
        return hipGetLastError();
    });
}

template <typename T, int NLO, int NHI>
hipError_t launch_split_range(const SplitLaunch& L, hipStream_t st) {
    if constexpr (NLO > NHI) {
        return hipErrorInvalidValue;
    } else {
        if (L.npos == (uint32_t)NLO) return launch_split_exact<T, NLO>(L, st);
        return launch_split_range<T, NLO + 1, NHI>(L, st);
    }
}

}  // namespace bc
