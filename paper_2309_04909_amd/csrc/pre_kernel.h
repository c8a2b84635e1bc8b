// Precomputed-randomness form of the DReLU (Alg. 7) and ReLU (Alg. 8) kernels.
//
// Everything the parties draw from their seeds is independent of the input,
// so it can be expanded ahead of time (an offline phase) and kept resident.
// The record keeps what would cost the online phase its shuffle, its mask
// draws or a message: P0/P1's flip t and shuffle and the masks from seed_01,
// and for the ReLU P2's [c]_1 of the Beaver triple (Alg. 8's preprocessing,
// sent to P1).  What a party draws from seed_02 or seed_12 alone (P2's
// response share rho, the triple shares [a]_0 [b]_0 [c]_0 and [a]_1 [b]_1)
// it regenerates online from its seed, one to three Philox blocks, as
// holders of a triple's seeds would.  The online kernel streams the shares
// plus the record and does flip, windows, sums, modulo switch, mask and zero
// test and the finish; it reuses the slot arithmetic of the fused kernel, so
// both give bit-identical results and messages.
//
// Record of a call on n elements, structure of arrays (each array [.][n]):
//   perm  uint32[ceil(N/4)][n]: byte q of word k is sigma(4k + q); bit 7 of
//         byte 0 of word 0 is t
//   rz    uint64[rz_words(N)][n]: the values r_0, z_0, r_1, z_1, ... (value
//         v = 2j for r_j, 2j + 1 for z_j) in N-bit fields (p < 2^N),
//         floor(64 / N) to a word: value v is bits N (v % K) .. of word
//         v / K, K = floor(64 / N).  N == 33: one value per word.
//   tail  ReLU only: T[n] = [c]_1
// Sections start at 256-byte boundaries.
#pragma once

#include "drelu_kernel.h"

namespace bc {

struct PreKArgs {
    const void* x0;
    const void* x1;
    void* y0;
    void* y1;
    void* cap;
    const uint32_t* perm;
    const void* rz;
    const void* tail;
    uint64_t n;
    uint64_t elem_base;
    uint64_t ring_mask;
    uint32_t k_lo, pad;
    Stream s02, s12;
};

struct ExpandKArgs {
    uint32_t* perm;
    void* rz;
    void* tail;
    uint64_t n;
    uint64_t elem_base;
    uint64_t ring_mask;
    Stream s01, s02, s12;
};

template <int N>
struct RzLayout {
    static constexpr bool WIDE = N == 33;
    static constexpr int K = WIDE ? 1 : 64 / N;          // values per word
    static constexpr uint64_t FIELD = WIDE ? ~0ull : (1ull << N) - 1;
};

// Offline: expand the seeds of n elements into the record.
template <typename T, int N, typename F, bool RELU>
__global__ BC_KERNEL_ATTRS void k_expand(ExpandKArgs A, F f) {
    const T mask = (T)A.ring_mask;
    const uint64_t n = A.n;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const uint64_t g = A.elem_base + e;
        const StreamAt r01 = A.s01.at(g);
        uint32_t perm[(N + 3) / 4];
        const uint32_t t = shuffle_perm<N>(r01, perm);
#pragma unroll
        for (int k = 0; k < (N + 3) / 4; ++k) st_nt(&A.perm[(uint64_t)k * n + e], k == 0 ? perm[0] | t << 7 : perm[k]);
        MaskReader<N, F> masks;
        uint64_t* rz = static_cast<uint64_t*>(A.rz);
        constexpr int K = RzLayout<N>::K;
        uint64_t acc = 0;                                  // the word being filled
#pragma unroll
        for (int j = 0; j < N; ++j) {
            typename F::T r, z;
            masks.slot(r01, j, f, r, z);
            plain_draws<N, F>(f, r, z);                   // the record keeps plain values
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int v = 2 * j + h;
                acc |= (uint64_t)(h ? z : r) << (N * (v % K) % 64);
                if (v % K == K - 1 || v == 2 * N - 1) {
                    st_nt(&rz[(uint64_t)(v / K) * n + e], acc);
                    acc = 0;
                }
            }
        }
        if constexpr (RELU) {
            T ba0, bb0, bc0, ba1, bb1;
            beaver_shares<T>(A.s02, A.s12, g, mask, ba0, bb0, bc0, ba1, bb1);
            st_nt(&static_cast<T*>(A.tail)[e], (T)((T)((T)(ba0 + ba1) * (T)(bb0 + bb1) - bc0) & mask));   // P2's [c]_1
        }
    }
}

// The sections of a record on n elements (rand_offsets).
template <typename T>
struct RecordView {
    const uint32_t* perm;
    const uint64_t* rz;
    const T* tail;
    uint64_t n;
};

template <typename T>
__device__ __forceinline__ RecordView<T> record_view(const void* rand, uint32_t npos, bool relu, uint64_t n) {
    const RandOffsets o = rand_offsets(npos, relu, sizeof(T), n);
    const uint8_t* base = static_cast<const uint8_t*>(rand);
    return RecordView<T>{reinterpret_cast<const uint32_t*>(base + o.perm), reinterpret_cast<const uint64_t*>(base + o.rz),
                         reinterpret_cast<const T*>(base + o.tail), n};
}

// Online: the input-dependent part of Alg. 7 (and of Alg. 8) for element e,
// reading its draws from the record.  Reads X0[e], X1[e] (with k_in > 0,
// shares of Z_{2^(l + k_in)} truncated by k_in bits first, Alg. 5, as in
// drelu_element) and writes Y0[e], Y1[e]; with CAP the round-1 messages go
// to cap[e * N + slot] and cap[(R.n + e) * N + slot].
template <typename T, int N, typename F, bool RELU, bool CAP>
__device__ __forceinline__ void drelu_pre_element(const T* __restrict__ X0, const T* __restrict__ X1, T* Y0, T* Y1,
                                                  typename F::T* cap, const RecordView<T>& R, uint64_t e, uint64_t g,
                                                  T mask, T in_mask, uint32_t k_in, uint32_t k_lo, const Stream& s02,
                                                  const Stream& s12, const F& f) {
    using FT = typename F::T;
    const uint64_t n = R.n;
    T in0, n1;
    input_shares<T>(ld_nt(&X0[e]), ld_nt(&X1[e]), mask, in_mask, k_in, in0, n1);
    uint32_t perm[(N + 3) / 4];
#pragma unroll
    for (int k = 0; k < (N + 3) / 4; ++k) perm[k] = ld_nt(&R.perm[(uint64_t)k * n + e]);
    const uint32_t t = (perm[0] >> 7) & 1u;
    const T a0 = flip_by(in0, t, mask);                // the flip, as in drelu_round1
    const T nb1 = flip_by(n1, t, mask);
    const T a0k = a0 >> k_lo, nb1k = nb1 >> k_lo;
    FT least = f.p;
    constexpr int K = RzLayout<N>::K;
    uint64_t cur = 0;                                  // the word being read
#pragma unroll
    for (int j = 0; j < N; ++j) {
        FT rv[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int v = 2 * j + h;
            if (v % K == 0) cur = ld_nt(&R.rz[(uint64_t)(v / K) * n + e]);
            rv[h] = (FT)((cur >> (N * (v % K) % 64)) & RzLayout<N>::FIELD);
        }
        const FT r = rv[0], z = rv[1];
        const uint32_t pos = (perm[j >> 2] >> (8 * (j & 3))) & 63u;
        FT w0, w1;
        slot_messages<T, N, F, 0, !CAP>(a0k, nb1k, pos, r, z, f, w0, w1, least);
        if constexpr (CAP) {
            cap[e * N + j] = w0;
            cap[(n + e) * N + j] = w1;
        }
    }
    const T dp = least == 0 ? 1 : 0;
    T y0, y1;
    if constexpr (!RELU) {
        const Words4 w = s02.block(g, TAG_RESP, 0);                 // rho, regenerated from seed_02
        drelu_finish<T>(dp, (T)join64(w.w0, w.w1), t, mask, y0, y1);
    } else {
        const T in1 = (T)((T)0 - n1) & mask;
        T ba0, bb0, bc0, ba1, bb1;                                  // the parties' triple shares, regenerated
        beaver_shares<T>(s02, s12, g, mask, ba0, bb0, bc0, ba1, bb1);
        relu_finish<T>(dp, in0, in1, ba0, bb0, bc0, ba1, bb1, ld_nt(&R.tail[e]), t, mask, y0, y1);
    }
    st_nt(&Y0[e], y0);
    st_nt(&Y1[e], y1);
}

// Online call: grid-stride over the n elements of one share pair.
template <typename T, int N, typename F, bool RELU, bool CAP>
__device__ __forceinline__ void drelu_pre_loop(const PreKArgs& A, const F& f, T mask) {
    const T* X0 = static_cast<const T*>(A.x0);
    const T* X1 = static_cast<const T*>(A.x1);
    T* Y0 = static_cast<T*>(A.y0);
    T* Y1 = static_cast<T*>(A.y1);
    typename F::T* cap = static_cast<typename F::T*>(A.cap);
    const RecordView<T> R{A.perm, static_cast<const uint64_t*>(A.rz), static_cast<const T*>(A.tail), A.n};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < A.n; e += stride)
        drelu_pre_element<T, N, F, RELU, CAP>(X0, X1, Y0, Y1, cap, R, e, A.elem_base + e, mask, mask, 0, A.k_lo,
                                              A.s02, A.s12, f);
}

// On a full-width ring the loop runs with the ring mask as a constant (see
// k_drelu).
template <typename T, int N, typename F, bool RELU, bool CAP>
__global__ BC_KERNEL_ATTRS void k_drelu_pre(PreKArgs A, F f_arg) {
    const F f = f_arg.vgpr();
    if constexpr (!CAP) {
        if ((T)A.ring_mask == (T)~(T)0) {
            drelu_pre_loop<T, N, F, RELU, CAP>(A, f, (T)~(T)0);
            return;
        }
    }
    drelu_pre_loop<T, N, F, RELU, CAP>(A, f, in_vgpr((T)A.ring_mask));
}

template <typename T, int N, typename F>
hipError_t launch_pre_field(const PreLaunch& L, const F& f, hipStream_t st) {
    const uint64_t mask = L.ell >= 64 ? ~0ull : ((1ull << L.ell) - 1);
    const RandOffsets o = rand_offsets(N, L.relu, sizeof(T), L.n);
    uint8_t* base = static_cast<uint8_t*>(L.rand);
    if (L.expand) {
        ExpandKArgs A;
        A.perm = reinterpret_cast<uint32_t*>(base + o.perm);
        A.rz = base + o.rz;
        A.tail = base + o.tail;
        A.n = L.n;
        A.elem_base = L.elem_base;
        A.ring_mask = mask;
        A.s01 = Stream{L.s01.k0, L.s01.k1, L.s01.n0, L.s01.n1};
        A.s02 = Stream{L.s02.k0, L.s02.k1, L.s02.n0, L.s02.n1};
        A.s12 = Stream{L.s12.k0, L.s12.k1, L.s12.n0, L.s12.n1};
        if (L.relu)
            hipLaunchKernelGGL((k_expand<T, N, F, true>), dim3(L.grid), dim3(256), 0, st, A, f);
        else
            hipLaunchKernelGGL((k_expand<T, N, F, false>), dim3(L.grid), dim3(256), 0, st, A, f);
        return hipGetLastError();
    }
    PreKArgs A;
    A.x0 = L.x0;
    A.x1 = L.x1;
    A.y0 = L.y0;
    A.y1 = L.y1;
    A.cap = L.cap;
    A.perm = reinterpret_cast<const uint32_t*>(base + o.perm);
    A.rz = base + o.rz;
    A.tail = base + o.tail;
    A.n = L.n;
    A.elem_base = L.elem_base;
    A.ring_mask = mask;
    A.k_lo = L.k_lo;
    A.pad = 0;
    A.s02 = Stream{L.s02.k0, L.s02.k1, L.s02.n0, L.s02.n1};
    A.s12 = Stream{L.s12.k0, L.s12.k1, L.s12.n0, L.s12.n1};
    if (L.relu) {
        if (L.cap) hipLaunchKernelGGL((k_drelu_pre<T, N, F, true, true>), dim3(L.grid), dim3(256), 0, st, A, f);
        else hipLaunchKernelGGL((k_drelu_pre<T, N, F, true, false>), dim3(L.grid), dim3(256), 0, st, A, f);
    } else {
        if (L.cap) hipLaunchKernelGGL((k_drelu_pre<T, N, F, false, true>), dim3(L.grid), dim3(256), 0, st, A, f);
        else hipLaunchKernelGGL((k_drelu_pre<T, N, F, false, false>), dim3(L.grid), dim3(256), 0, st, A, f);
    }
    return hipGetLastError();
}

template <typename T, int N>
hipError_t launch_pre_exact(const PreLaunch& L, hipStream_t st) {
    return with_field<N>(L.p, [&](auto f) { return launch_pre_field<T, N, decltype(f)>(L, f, st); });
}

template <typename T, int NLO, int NHI>
hipError_t launch_pre_range(const PreLaunch& L, hipStream_t st) {
    if constexpr (NLO > NHI) {
        return hipErrorInvalidValue;
    } else {
        if (L.npos == (uint32_t)NLO) return launch_pre_exact<T, NLO>(L, st);
        return launch_pre_range<T, NLO + 1, NHI>(L, st);
    }
}

}  // namespace bc
