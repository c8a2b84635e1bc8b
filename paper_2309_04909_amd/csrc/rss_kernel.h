// Replicated-sharing (RSS) Bicoptor 2.0 DReLU (Alg. drelu2) and ReLU (the
// RSS ReLU of the appendix: one more product of replicated shares).
//
// x = [x]_0 + [x]_1 + [x]_2 mod 2^l and P_j holds ([x]_j, [x]_{j+1}),
// indices mod 3; on one GPU each share is stored once, in its own array.
// One thread owns one element and plays all three parties:
//   preprocessing  [t] = (a0 - a2, a1 - a0 + t, a2 - a1) from the seed_012
//                  alphas and the seed_01 flip bit t (the same t as Alg. 7);
//                  [s] = (s - s1 - s2, s1, s2) with [s]_1 from seed_012,
//                  [s]_2 from seed_12 and P2's bit s from seed_2;
//                  [s xor t] = [s] + [t] - 2 [s][t]
//   round 1        P0 enters [x]_0 + [x]_1 and P1 enters [x]_2 into Alg. 7
//                  up to their messages; P2's zero test gives D'
//   round 2        P2 publishes D'' = s xor D'
//   finish         [DReLU] = D'' + [s xor t] - 2 D'' [s xor t], the public
//                  D'' on share 0 (held by P0 and P2)
//   ReLU           the product [x][DReLU(x)] with the full-precision x
// A product of replicated shares: P_j forms u_j v_j + u_j v_{j+1} +
// u_{j+1} v_j plus the zero share g_j = a'_j - a'_{j-1} (fresh seed_012
// alphas) and sends it to P_{j-1}; these sums are the product's shares.
//
// Draws: V_k = (w_{2k}, w_{2k+1}) of stream TAG_RSS under seed_012 (word
// 2k is word 2k % 4 of block 2k / 4), each mod 2^l: the alphas of [t]
// (V_0..V_2), [s]_1 (V_3), the zero sharing of [s][t] (V_4..V_6) and of the
// ReLU product (V_7..V_9).  [s]_2 = (w0, w1) of block 0 of TAG_RSS under
// seed_12; s = bit 0 of word 0 of block 0 of TAG_RSS under seed_2.
//
// Arithmetic in the storage width (2^64 or 2^32) reduces consistently mod
// 2^l, so only the Alg. 7 inputs and the stored outputs are masked.
#pragma once

#include "drelu_kernel.h"

namespace bc {

struct RssKArgs {
    const void* x0;
    const void* x1;
    const void* x2;
    void* y0;
    void* y1;
    void* y2;
    void* cap;
    uint64_t n;
    uint64_t elem_base;
    uint64_t ring_mask;
    uint32_t k_lo;
    Stream s01, s12, s012, s2;
};

// z = [u v] from replicated shares u, v and the zero sharing g.
template <typename T>
__device__ __forceinline__ void rss_product(const T (&u)[3], const T (&v)[3], const T (&g)[3], T (&z)[3]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int k = j == 2 ? 0 : j + 1;
        z[j] = (T)(u[j] * (T)(v[j] + v[k]) + u[k] * v[j] + g[j]);   // u_j v_j + u_j v_{j+1} + u_{j+1} v_j
    }
}

template <typename T>
__device__ __forceinline__ T word_pair(uint32_t lo, uint32_t hi) {
    return (T)join64(lo, hi);
}

template <typename T, int N, typename F, bool RELU, bool CAP>
__device__ __forceinline__ void rss_element(const RssKArgs& A, const T* __restrict__ X0, const T* __restrict__ X1,
                                            const T* __restrict__ X2, T* Y0, T* Y1, T* Y2,
                                            typename F::T* cap, uint64_t e, uint64_t g, T mask, const F& f) {
    const T x[3] = {ld_nt(&X0[e]), ld_nt(&X1[e]), ld_nt(&X2[e])};

    // round 1 and P2's zero test on the 2-of-2 input ([x]_0 + [x]_1, [x]_2),
    // whose second holder cuts its negated share -[x]_2
    uint32_t t;
    const T nx2 = (T)((T)0 - x[2]) & mask;
    const T dp = drelu_round1<T, N, F, CAP>((T)(x[0] + x[1]) & mask, nx2, g, mask, A.k_lo, A.s01, cap, A.n, e, f, t);

    // preprocessing: [t], [s], [s][t]
    const StreamAt r012 = A.s012.at(g);
    const Words4 b0 = r012.block(TAG_RSS, 0);
    const Words4 b1 = r012.block(TAG_RSS, 1);
    const Words4 b2 = r012.block(TAG_RSS, 2);
    const Words4 b3 = r012.block(TAG_RSS, 3);
    const Words4 c12 = A.s12.block(g, TAG_RSS, 0);
    const T s = (T)(A.s2.block(g, TAG_RSS, 0).w0 & 1u);
    const T al0 = word_pair<T>(b0.w0, b0.w1), al1 = word_pair<T>(b0.w2, b0.w3), al2 = word_pair<T>(b1.w0, b1.w1);
    const T s1 = word_pair<T>(b1.w2, b1.w3), s2 = word_pair<T>(c12.w0, c12.w1);
    const T ts[3] = {(T)(al0 - al2), (T)(al1 - al0 + (T)t), (T)(al2 - al1)};
    const T ss[3] = {(T)(s - s1 - s2), s1, s2};
    const T ga0 = word_pair<T>(b2.w0, b2.w1), ga1 = word_pair<T>(b2.w2, b2.w3), ga2 = word_pair<T>(b3.w0, b3.w1);
    const T gst[3] = {(T)(ga0 - ga2), (T)(ga1 - ga0), (T)(ga2 - ga1)};
    T st[3];
    rss_product<T>(ss, ts, gst, st);

    // P2's public reply and the finish: y_j = q_j - 2 D'' q_j (+ D'' on share 0)
    const T dpp = dp ^ s;
    T y[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const T q = (T)(ss[j] + ts[j] - (T)2 * st[j]);               // [s xor t]_j
        y[j] = dpp ? (T)((T)0 - q) : q;
    }
    y[0] = (T)(y[0] + dpp);

    if constexpr (RELU) {
        const Words4 b4 = r012.block(TAG_RSS, 4);
        const T gb0 = word_pair<T>(b3.w2, b3.w3), gb1 = word_pair<T>(b4.w0, b4.w1), gb2 = word_pair<T>(b4.w2, b4.w3);
        const T gr[3] = {(T)(gb0 - gb2), (T)(gb1 - gb0), (T)(gb2 - gb1)};
        T z[3];
        rss_product<T>(x, y, gr, z);
        st_nt(&Y0[e], (T)(z[0] & mask));
        st_nt(&Y1[e], (T)(z[1] & mask));
        st_nt(&Y2[e], (T)(z[2] & mask));
    } else {
        st_nt(&Y0[e], (T)(y[0] & mask));
        st_nt(&Y1[e], (T)(y[1] & mask));
        st_nt(&Y2[e], (T)(y[2] & mask));
    }
}

// One call: grid-stride over the n elements of one share triple.
template <typename T, int N, typename F, bool RELU, bool CAP>
__device__ __forceinline__ void rss_loop(const RssKArgs& A, const F& f, T mask) {
    const T* X0 = static_cast<const T*>(A.x0);
    const T* X1 = static_cast<const T*>(A.x1);
    const T* X2 = static_cast<const T*>(A.x2);
    T* Y0 = static_cast<T*>(A.y0);
    T* Y1 = static_cast<T*>(A.y1);
    T* Y2 = static_cast<T*>(A.y2);
    typename F::T* cap = static_cast<typename F::T*>(A.cap);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < A.n; e += stride)
        rss_element<T, N, F, RELU, CAP>(A, X0, X1, X2, Y0, Y1, Y2, cap, e, A.elem_base + e, mask, f);
}

// On a full-width ring the loop runs with the ring mask as a constant (see
// k_drelu).
template <typename T, int N, typename F, bool RELU, bool CAP>
__global__ BC_KERNEL_ATTRS void k_rss(RssKArgs A, F f_arg) {
    const F f = f_arg.vgpr();
    if constexpr (!CAP) {
        if ((T)A.ring_mask == (T)~(T)0) {
            rss_loop<T, N, F, RELU, CAP>(A, f, (T)~(T)0);
            return;
        }
    }
    rss_loop<T, N, F, RELU, CAP>(A, f, in_vgpr((T)A.ring_mask));
}

inline Stream stream_of(const StreamKey& k) { return Stream{k.k0, k.k1, k.n0, k.n1}; }

template <typename T, int N, bool RELU>
hipError_t launch_rss_exact(const RssLaunch& L, hipStream_t st) {
    RssKArgs A;
    A.x0 = L.x0;
    A.x1 = L.x1;
    A.x2 = L.x2;
    A.y0 = L.y0;
    A.y1 = L.y1;
    A.y2 = L.y2;
    A.cap = L.cap;
    A.n = L.n;
    A.elem_base = L.elem_base;
    A.ring_mask = L.ell >= 64 ? ~0ull : ((1ull << L.ell) - 1);
    A.k_lo = L.k_lo;
    A.s01 = stream_of(L.s01);
    A.s12 = stream_of(L.s12);
    A.s012 = stream_of(L.s012);
    A.s2 = stream_of(L.s2);
    return with_field<N>(L.p, [&](auto f) {
        using F = decltype(f);
        if (L.cap)
            hipLaunchKernelGGL((k_rss<T, N, F, RELU, true>), dim3(L.grid), dim3(256), 0, st, A, f);
        else
            hipLaunchKernelGGL((k_rss<T, N, F, RELU, false>), dim3(L.grid), dim3(256), 0, st, A, f);
        return hipGetLastError();
    });
}

template <typename T, int NLO, int NHI>
hipError_t launch_rss_range(const RssLaunch& L, hipStream_t st) {
    if constexpr (NLO > NHI) {
        return hipErrorInvalidValue;
    } else {
        if (L.npos == (uint32_t)NLO)
            return L.relu ? launch_rss_exact<T, NLO, true>(L, st) : launch_rss_exact<T, NLO, false>(L, st);
        return launch_rss_range<T, NLO + 1, NHI>(L, st);
    }
}

}  // namespace bc
