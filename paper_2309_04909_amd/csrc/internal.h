// Host-side declarations shared by the C-ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bicop.h"

namespace bc {

// Counter-based stream handle passed by value to kernels (key and nonce).
struct StreamKey {
    uint32_t k0, k1, n0, n1;
};

// Fully validated DReLU/ReLU launch description.
struct DreluLaunch {
    const void* x0;
    const void* x1;
    void* y0;
    void* y1;
    void* cap;
    uint64_t n;
    uint64_t elem_base;
    uint32_t ell, lx, k_lo, npos;
    uint32_t k_in;        // > 0: inputs are shares of Z_{2^(ell + k_in)}, truncated first (Alg. 5)
    uint64_t p;
    StreamKey s01, s02, s12;
    int grid;
    int block;
    int group;            // lanes per element: 1, or 4 / 8 (lane-group kernel, no capture)
};

// Device plan of a ragged batch: this header, then nseg bc_segment records,
// then nseg + 1 uint64 tile offsets.
struct BatchPlanHeader {
    uint32_t magic;        // kBatchMagic
    uint32_t nseg;
    uint32_t ell, lx, k_lo, tile_elems;
    uint64_t p;
    uint64_t total_tiles;
    uint64_t total_elems;
    uint32_t reserved[4];
};
static_assert(sizeof(BatchPlanHeader) == 64, "plan header is 64 bytes");
static_assert(sizeof(bc_segment) == 80, "segment record is 80 bytes");
constexpr uint32_t kBatchMagic = 0x4C504342u;   // "BCPL"

struct BatchLaunch {
    const BatchPlanHeader* hdr;      // device
    const bc_segment* segs;          // device
    const uint64_t* tile_begin;      // device
    uint64_t total_tiles, tile_elems, p;
    uint32_t ell, k_lo, npos, nseg;
    StreamKey s01, s02, s12;
    int grid;
};

hipError_t launch_batch_u64_lo(const BatchLaunch& L, hipStream_t st);    // N 2..12
hipError_t launch_batch_u64_mid(const BatchLaunch& L, hipStream_t st);   // N 13..24
hipError_t launch_batch_u64_hi(const BatchLaunch& L, hipStream_t st);    // N 25..33
hipError_t launch_batch_u32(const BatchLaunch& L, hipStream_t st);       // N 2..17

// Enqueues on `st` the copy of a host plan of `bytes` bytes (a multiple of 8,
// at most BC_STATIC_PLAN_BYTES) into the current device's fixed plan area,
// and returns that area's device address in *dev_plan.  Allocates nothing.
hipError_t static_plan_upload(const void* host_plan, uint64_t bytes, hipStream_t st, void** dev_plan);

// Precomputed-randomness calls: the offline expansion (expand = true, writes
// `rand`) or the online DReLU/ReLU (reads `rand`).
struct PreLaunch {
    const void* x0;
    const void* x1;
    void* y0;
    void* y1;
    void* cap;
    void* rand;
    uint64_t n, elem_base, p;
    uint32_t ell, k_lo, npos;
    bool relu, expand;
    StreamKey s01, s02, s12;
    int grid;
};

// Byte offsets of the sections of a randomness record on n elements
// (each section starts at a 256-byte boundary).
struct RandOffsets {
    uint64_t perm, rz, tail, total;
};

__host__ __device__ inline uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

// 64-bit words per element of a record's r/z section: the 2 npos values of
// npos bits (p < 2^npos) packed floor(64 / npos) to a word; npos = 33 keeps
// one value per word.
__host__ __device__ constexpr uint32_t rz_words(uint32_t npos) {
    return npos >= 33 ? 2 * npos : (2 * npos + 64 / npos - 1) / (64 / npos);
}

__host__ __device__ inline RandOffsets rand_offsets(uint32_t npos, bool relu, uint32_t ring_width, uint64_t n) {
    RandOffsets o;
    o.perm = 0;
    const uint64_t perm_bytes = 4ull * ((npos + 3) / 4) * n;
    o.rz = align256(perm_bytes);
    const uint64_t rz_bytes = n * 8ull * rz_words(npos);
    o.tail = align256(o.rz + rz_bytes);
    o.total = o.tail + (relu ? (uint64_t)ring_width * n : 0);   // the ReLU's [c]_1
    return o;
}

// Fully validated replicated-sharing DReLU/ReLU launch (Alg. drelu2).
struct RssLaunch {
    const void* x0;
    const void* x1;
    const void* x2;
    void* y0;
    void* y1;
    void* y2;
    void* cap;
    uint64_t n, elem_base, p;
    uint32_t ell, lx, k_lo, npos;
    bool relu;
    StreamKey s01, s12, s012, s2;
    int grid;
};

hipError_t launch_rss_u64_lo(const RssLaunch& L, hipStream_t st);    // N 2..12
hipError_t launch_rss_u64_mid(const RssLaunch& L, hipStream_t st);   // N 13..24
hipError_t launch_rss_u64_hi(const RssLaunch& L, hipStream_t st);    // N 25..33
hipError_t launch_rss_u32(const RssLaunch& L, hipStream_t st);       // N 2..17

// Validated launch of one party's part of the DReLU with the parties apart.
struct SplitLaunch {
    enum Kind { SEND, REPLY, FINISH };
    Kind kind;
    uint32_t party;       // SEND, FINISH: 0 (P0) or 1 (P1)
    const void* in0;
    const void* in1;
    void* out0;
    void* out1;
    uint64_t n, elem_base, p;
    uint32_t ell, lx, k_lo, npos;
    StreamKey s01, s02;
    int grid;
};

hipError_t launch_split_u64_lo(const SplitLaunch& L, hipStream_t st);   // SEND / REPLY, N 2..17
hipError_t launch_split_u64_hi(const SplitLaunch& L, hipStream_t st);   // SEND / REPLY, N 18..33
hipError_t launch_split_u32(const SplitLaunch& L, hipStream_t st);      // SEND / REPLY, N 2..17
hipError_t launch_split_finish(const SplitLaunch& L, hipStream_t st);   // FINISH, any ring

// Validated elementwise product with truncation (Alg. linear / multiply-then-truncate).
struct MulLaunch {
    const void* x0;
    const void* x1;
    const void* y0;
    const void* y1;
    void* z0;
    void* z1;
    uint64_t n, elem_base;
    uint32_t ell, kx, ky, kz;   // Alg. 1 shifts of the factors (kx, ky) and of the product (kz)
    StreamKey s02, s12;
    int grid_cap;
};

hipError_t launch_mul(const MulLaunch& L, hipStream_t st);

// Elementwise Z_p multiply-add with the kernels' field arithmetic (diagnostic).
struct ZpLaunch {
    const uint64_t* a;
    const uint64_t* b;
    const uint64_t* d;
    uint64_t* out;
    uint64_t n;
    uint64_t p;
    uint32_t npos;
    int grid;
};
hipError_t launch_zp_mul_add(const ZpLaunch& L, hipStream_t st);

hipError_t launch_pre_u64_lo(const PreLaunch& L, hipStream_t st);    // N 2..12
hipError_t launch_pre_u64_mid(const PreLaunch& L, hipStream_t st);   // N 13..24
hipError_t launch_pre_u64_hi(const PreLaunch& L, hipStream_t st);    // N 25..33
hipError_t launch_pre_u32(const PreLaunch& L, hipStream_t st);       // N 2..17

// Kernel launchers, one per op, storage width and range of N = l_x + 1 (the
// split only spreads compilation over several files).  Each returns
// hipErrorInvalidValue when L.npos is outside its range.
hipError_t launch_drelu_u64_lo(const DreluLaunch& L, hipStream_t st);    // N 2..12
hipError_t launch_drelu_u64_mid(const DreluLaunch& L, hipStream_t st);   // N 13..24
hipError_t launch_drelu_u64_hi(const DreluLaunch& L, hipStream_t st);    // N 25..33
hipError_t launch_relu_u64_lo(const DreluLaunch& L, hipStream_t st);
hipError_t launch_relu_u64_mid(const DreluLaunch& L, hipStream_t st);
hipError_t launch_relu_u64_hi(const DreluLaunch& L, hipStream_t st);
hipError_t launch_drelu_u32(const DreluLaunch& L, hipStream_t st);       // N 2..17
hipError_t launch_relu_u32(const DreluLaunch& L, hipStream_t st);

hipError_t launch_trunc_det(const void* x0, const void* x1, void* y0, void* y1, uint64_t n,
                            uint32_t ell, uint32_t k1, uint32_t k2, int grid, hipStream_t st);
hipError_t launch_trunc_prob(const void* x0, const void* x1, void* y0, void* y1, uint64_t n,
                             uint32_t ell, uint32_t k, int grid, hipStream_t st);
hipError_t launch_mod_switch(const void* x0, const void* x1, void* y0, void* y1, uint64_t n,
                             uint32_t ell_in, uint64_t p, int grid, hipStream_t st);
hipError_t launch_prg_blocks(uint32_t* out, uint64_t n, uint32_t nblocks, StreamKey key, uint32_t tag,
                             uint64_t elem_base, int grid, hipStream_t st);

// Number of compute units of the current device (cached per device).
int device_cus();

}  // namespace bc
