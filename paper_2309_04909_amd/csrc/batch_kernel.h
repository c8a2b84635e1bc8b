// Ragged batch of DReLU / ReLU segments (one setting, one persistent launch).
#pragma once

#include "pre_kernel.h"

namespace bc {

struct BatchKArgs {
    uint64_t total_tiles;
    uint64_t tile_elems;
    uint64_t ring_mask;
    uint32_t nseg, k_lo, ell;
    uint32_t k01a, k01b, k02a, k02b, k12a, k12b;
};

// The fused elements [e0, e1) of one tile (at most a tile's elements, so
// 32-bit offsets from the tile's start): each thread walks its elements with
// the next one's shares loaded before the current one is computed (raw
// buffer loads over the tile, which read 0 past its end), as k_drelu does.
template <typename T, int N, typename F, bool RELU>
__device__ __forceinline__ void tile_elements(const T* X0, const T* X1, T* Y0, T* Y1, uint64_t e0, uint64_t e1,
                                              uint64_t base, T mask, T in_mask, uint32_t k_in, uint32_t k_lo,
                                              const Stream& s01, const Stream& s02, const Stream& s12, const F& f) {
    const uint32_t m = (uint32_t)(e1 - e0);
    uint32_t i = threadIdx.x;
    if (i >= m) return;
    const T* x0 = X0 + e0;
    const T* x1 = X1 + e0;
    const __amdgpu_buffer_rsrc_t B0 = buffer_of(x0, m), B1 = buffer_of(x1, m);
    T a0 = load_at(x0, i), a1 = load_at(x1, i);
    for (;;) {
        const uint32_t in = i + blockDim.x;
        const T a0n = load_buf<T>(B0, in), a1n = load_buf<T>(B1, in);
        T y0, y1;
        drelu_element_of<T, N, F, RELU, false>(a0, a1, y0, y1, nullptr, 0, e0 + i, base + e0 + i, mask, in_mask, k_in,
                                               k_lo, s01, s02, s12, f);
        store_at(Y0 + e0, i, y0);
        store_at(Y1 + e0, i, y1);
        if (in >= m) break;
        i = in;
        a0 = a0n;
        a1 = a1n;
    }
}

// Ragged batch: a persistent grid walks the tiles of every segment.  Tile t
// belongs to the segment s with tile_begin[s] <= t < tile_begin[s + 1]; each
// segment has its own op, nonce and global element offset, so every element
// gets exactly the randomness (and result) of a single call on its segment.
// A segment with a precomputed record runs the online element (the draws
// come from the record, as in bc_drelu_pre / bc_relu_pre), with the same
// per-segment input truncation.
// Each block takes tiles blockIdx.x, blockIdx.x + gridDim.x, ... until
// total_tiles: every wave reaches the exit.  This is the walk, with the ring
// mask given; k_batch below calls it.
template <typename T, int N, typename F>
__device__ __forceinline__ void batch_walk(const bc_segment* __restrict__ segs,
                                           const uint64_t* __restrict__ tile_begin, const BatchKArgs& A, const F& f,
                                           T mask) {
    const uint32_t nseg = A.nseg;
    const uint64_t total = A.total_tiles;
    const uint64_t tile = A.tile_elems;
    for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) {
        // segment of tile t: largest s with tile_begin[s] <= t (uniform search)
        uint32_t lo = 0, hi = nseg;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (tile_begin[mid] <= t) lo = mid; else hi = mid;
        }
        const bc_segment& S = segs[lo];
        const T* X0 = static_cast<const T*>(S.x0);
        const T* X1 = static_cast<const T*>(S.x1);
        T* Y0 = static_cast<T*>(S.y0);
        T* Y1 = static_cast<T*>(S.y1);
        const uint64_t e0 = (t - tile_begin[lo]) * tile;
        const uint64_t e1 = e0 + tile < S.n ? e0 + tile : S.n;
        const uint32_t n0 = (uint32_t)S.nonce, n1 = (uint32_t)(S.nonce >> 32);
        const Stream s01{A.k01a, A.k01b, n0, n1}, s02{A.k02a, A.k02b, n0, n1}, s12{A.k12a, A.k12b, n0, n1};
        const uint64_t base = S.elem_base;
        // the segment's input ring l + k_in (Alg. 5 by k_in first; 0 = the plain load)
        const uint32_t k_in = S.k_in, lin = A.ell + k_in;
        const T in_mask = lin >= 8 * sizeof(T) ? (T)~(T)0 : (T)(((T)1 << lin) - 1);
        if (S.rand) {
            // precomputed randomness: the segment's record replaces its seed_01
            // draws (and holds P2's [c]_1); seed_02 / seed_12 draws are regenerated
            const bool relu = S.op == BC_OP_RELU;
            const RecordView<T> R = record_view<T>(S.rand, (uint32_t)N, relu, S.n);
            if (relu) {
                for (uint64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x)
                    drelu_pre_element<T, N, F, true, false>(X0, X1, Y0, Y1, nullptr, R, e, base + e, mask, in_mask,
                                                            k_in, A.k_lo, s02, s12, f);
            } else {
                for (uint64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x)
                    drelu_pre_element<T, N, F, false, false>(X0, X1, Y0, Y1, nullptr, R, e, base + e, mask, in_mask,
                                                             k_in, A.k_lo, s02, s12, f);
            }
        } else if (S.op == BC_OP_RELU) {
            tile_elements<T, N, F, true>(X0, X1, Y0, Y1, e0, e1, base, mask, in_mask, k_in, A.k_lo, s01, s02, s12, f);
        } else {
            tile_elements<T, N, F, false>(X0, X1, Y0, Y1, e0, e1, base, mask, in_mask, k_in, A.k_lo, s01, s02, s12, f);
        }
    }
}

// A full-width ring (l = 64 in 64-bit storage, l = 32 in 32-bit) walks the
// tiles with the ring mask as a constant (see k_drelu).
template <typename T, int N, typename F>
__global__ BC_KERNEL_ATTRS void k_batch(const BatchPlanHeader* __restrict__ hdr,
                                               const bc_segment* __restrict__ segs,
                                               const uint64_t* __restrict__ tile_begin, BatchKArgs A, F f_arg) {
    // The device plan must still be the one this launch was built from: a
    // plan whose memory was freed and reused fails these checks, and then no
    // block walks it.
    if (hdr->magic != kBatchMagic || hdr->nseg != A.nseg || hdr->total_tiles != A.total_tiles) return;
    const F f = f_arg.vgpr();
    if ((T)A.ring_mask == (T)~(T)0)
        batch_walk<T, N, F>(segs, tile_begin, A, f, (T)~(T)0);
    else
        batch_walk<T, N, F>(segs, tile_begin, A, f, in_vgpr((T)A.ring_mask));
}

template <typename T, int N, typename F>
hipError_t launch_batch_field(const BatchLaunch& L, const F& f, hipStream_t st) {
    BatchKArgs A;
    A.total_tiles = L.total_tiles;
    A.tile_elems = L.tile_elems;
    A.ring_mask = L.ell >= 64 ? ~0ull : ((1ull << L.ell) - 1);
    A.nseg = L.nseg;
    A.k_lo = L.k_lo;
    A.ell = L.ell;
    A.k01a = L.s01.k0;
    A.k01b = L.s01.k1;
    A.k02a = L.s02.k0;
    A.k02b = L.s02.k1;
    A.k12a = L.s12.k0;
    A.k12b = L.s12.k1;
    hipLaunchKernelGGL((k_batch<T, N, F>), dim3(L.grid), dim3(256), 0, st, L.hdr, L.segs, L.tile_begin, A, f);
    return hipGetLastError();
}

template <typename T, int N>
hipError_t launch_batch_exact(const BatchLaunch& L, hipStream_t st) {
    return with_field<N>(L.p, [&](auto f) { return launch_batch_field<T, N, decltype(f)>(L, f, st); });
}

template <typename T, int NLO, int NHI>
hipError_t launch_batch_range(const BatchLaunch& L, hipStream_t st) {
    if constexpr (NLO > NHI) {
        return hipErrorInvalidValue;
    } else {
        if (L.npos == (uint32_t)NLO) return launch_batch_exact<T, NLO>(L, st);
        return launch_batch_range<T, NLO + 1, NHI>(L, st);
    }
}

}  // namespace bc
