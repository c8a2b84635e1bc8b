// HBM-streaming share kernels: deterministic truncation (Alg. 4 / Alg. 5),
// SecureML truncation (Alg. 1), modulo switch (Alg. 6), and a raw dump of
// Philox blocks for checking the generator.
//
// Each thread reads V consecutive elements of both input shares with one
// vector load per share, computes both parties' outputs, and writes them back
// with one vector store per share; V makes the wider of the two vectors 16
// bytes.
// The grid strides over vectors; a scalar loop finishes the ragged tail.
#include "bc_device.h"
#include "internal.h"

namespace bc {

// Alg. 4 / Alg. 5: P0 cut(x0, k1, k2), P1 -cut(-x1, k1, k2), in Z_{2^(l-k1-k2)}.
template <typename TI, typename TO>
struct OpTruncDet {
    TI imask;
    TO omask;
    uint32_t k1;
    __device__ __forceinline__ void operator()(TI a, TI b, TO& c, TO& d) const {
        a &= imask;
        const TI nb = (TI)((TI)0 - (b & imask)) & imask;
        c = (TO)(a >> k1) & omask;
        d = (TO)((TO)0 - (TO)(nb >> k1)) & omask;
    }
};

// Alg. 1: P0 cut(x0, k), P1 -cut(-x1, k), in Z_{2^l}.
template <typename T>
struct OpTruncProb {
    T mask;
    uint32_t k;
    __device__ __forceinline__ void operator()(T a, T b, T& c, T& d) const {
        a &= mask;
        const T nb = (T)((T)0 - (b & mask)) & mask;
        c = a >> k;
        d = (T)((T)0 - (nb >> k)) & mask;
    }
};

// Alg. 6 with 2^l' < p < 2^(l'+1): an input share x < 2^l' is already < p and
// 2^l' mod p = 2^l', so P0 outputs x0 (or 2^l' when x0 = 0) and P1 outputs
// x1 + p - 2^l' (< p).
template <typename TI, typename TO>
struct OpModSwitch {
    TI imask;
    TO two;        // 2^l'
    TO p_minus;    // p - 2^l'
    __device__ __forceinline__ void operator()(TI a, TI b, TO& c, TO& d) const {
        a &= imask;
        c = a ? (TO)a : two;
        d = (TO)(b & imask) + p_minus;
    }
};

template <typename TI, typename TO, int V, typename Op>
__global__ __launch_bounds__(256) void k_map2(const TI* x0, const TI* x1, TO* y0, TO* y1, uint64_t n, Op op) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t nv = n / V;
    for (uint64_t v = tid; v < nv; v += stride) {
        const vec_t<TI, V> a = ld_nt(reinterpret_cast<const vec_t<TI, V>*>(x0 + v * V));
        const vec_t<TI, V> b = ld_nt(reinterpret_cast<const vec_t<TI, V>*>(x1 + v * V));
        vec_t<TO, V> c, d;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            TO ck, dk;
            op(a[k], b[k], ck, dk);
            c[k] = ck;
            d[k] = dk;
        }
        st_nt(reinterpret_cast<vec_t<TO, V>*>(y0 + v * V), c);
        st_nt(reinterpret_cast<vec_t<TO, V>*>(y1 + v * V), d);
    }
    for (uint64_t i = nv * V + tid; i < n; i += stride) {
        TO c, d;
        op(x0[i], x1[i], c, d);
        y0[i] = c;
        y1[i] = d;
    }
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

template <typename TI, typename TO, typename Op>
static hipError_t launch_map2(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, const Op& op,
                              int grid_cap, hipStream_t st) {
    constexpr int V = 16 / (int)(sizeof(TI) > sizeof(TO) ? sizeof(TI) : sizeof(TO));
    const bool vec = aligned16(x0) && aligned16(x1) && aligned16(y0) && aligned16(y1);
    const uint64_t work = vec ? (n + V - 1) / V : n;
    uint64_t grid = (work + 255) / 256;
    if (grid > (uint64_t)grid_cap) grid = (uint64_t)grid_cap;
    if (grid == 0) grid = 1;
    const TI* a = static_cast<const TI*>(x0);
    const TI* b = static_cast<const TI*>(x1);
    TO* c = static_cast<TO*>(y0);
    TO* d = static_cast<TO*>(y1);
    if (vec)
        hipLaunchKernelGGL((k_map2<TI, TO, V, Op>), dim3((unsigned)grid), dim3(256), 0, st, a, b, c, d, n, op);
    else
        hipLaunchKernelGGL((k_map2<TI, TO, 1, Op>), dim3((unsigned)grid), dim3(256), 0, st, a, b, c, d, n, op);
    return hipGetLastError();
}

static uint64_t low_mask(uint32_t bits) { return bits >= 64 ? ~0ull : ((1ull << bits) - 1); }

hipError_t launch_trunc_det(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, uint32_t ell,
                            uint32_t k1, uint32_t k2, int grid, hipStream_t st) {
    const uint32_t m = ell - k1 - k2;
    const uint64_t im = low_mask(ell), om = low_mask(m);
    if (ell > 32) {
        if (m > 32)
            return launch_map2<uint64_t, uint64_t>(x0, x1, y0, y1, n, OpTruncDet<uint64_t, uint64_t>{im, om, k1}, grid, st);
        return launch_map2<uint64_t, uint32_t>(x0, x1, y0, y1, n, OpTruncDet<uint64_t, uint32_t>{im, (uint32_t)om, k1},
                                               grid, st);
    }
    return launch_map2<uint32_t, uint32_t>(x0, x1, y0, y1, n, OpTruncDet<uint32_t, uint32_t>{(uint32_t)im, (uint32_t)om, k1},
                                           grid, st);
}

hipError_t launch_trunc_prob(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, uint32_t ell, uint32_t k,
                             int grid, hipStream_t st) {
    const uint64_t m = low_mask(ell);
    if (ell > 32) return launch_map2<uint64_t, uint64_t>(x0, x1, y0, y1, n, OpTruncProb<uint64_t>{m, k}, grid, st);
    return launch_map2<uint32_t, uint32_t>(x0, x1, y0, y1, n, OpTruncProb<uint32_t>{(uint32_t)m, k}, grid, st);
}

hipError_t launch_mod_switch(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, uint32_t ell_in,
                             uint64_t p, int grid, hipStream_t st) {
    const uint64_t im = low_mask(ell_in);
    const uint64_t two = 1ull << ell_in;
    if (ell_in > 32)
        return launch_map2<uint64_t, uint64_t>(x0, x1, y0, y1, n, OpModSwitch<uint64_t, uint64_t>{im, two, p - two}, grid, st);
    if (p >= (1ull << 32))   // l' = 32: 32-bit input shares, 64-bit field elements
        return launch_map2<uint32_t, uint64_t>(x0, x1, y0, y1, n, OpModSwitch<uint32_t, uint64_t>{(uint32_t)im, two, p - two},
                                               grid, st);
    return launch_map2<uint32_t, uint32_t>(x0, x1, y0, y1, n,
                                           OpModSwitch<uint32_t, uint32_t>{(uint32_t)im, (uint32_t)two, (uint32_t)(p - two)},
                                           grid, st);
}

__global__ __launch_bounds__(256) void k_prg_blocks(uint32_t* out, uint64_t n, uint32_t nblocks, Stream s, uint32_t tag,
                                                    uint64_t elem_base) {
    const uint64_t total = n * nblocks;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        const uint64_t i = idx / nblocks;
        const uint32_t b = (uint32_t)(idx - i * nblocks);
        const Words4 w = s.block(elem_base + i, tag, b);
        out[idx * 4 + 0] = w.w0;
        out[idx * 4 + 1] = w.w1;
        out[idx * 4 + 2] = w.w2;
        out[idx * 4 + 3] = w.w3;
    }
}

hipError_t launch_prg_blocks(uint32_t* out, uint64_t n, uint32_t nblocks, StreamKey key, uint32_t tag, uint64_t elem_base,
                             int grid_cap, hipStream_t st) {
    const uint64_t total = n * nblocks;
    uint64_t grid = (total + 255) / 256;
    if (grid > (uint64_t)grid_cap) grid = (uint64_t)grid_cap;
    if (grid == 0) grid = 1;
    const Stream s{key.k0, key.k1, key.n0, key.n1};
    hipLaunchKernelGGL(k_prg_blocks, dim3((unsigned)grid), dim3(256), 0, st, out, n, nblocks, s, tag, elem_base);
    return hipGetLastError();
}

}  // namespace bc
