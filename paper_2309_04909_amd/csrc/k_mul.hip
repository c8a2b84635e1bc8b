// Elementwise product of 2-of-2 shares with the SecureML truncation (Alg. 1)
// of the factors first (truncate-then-multiply, Alg. linear) or of the
// product after (multiply-then-truncate), all three parties in one kernel.
//
// Per element: P0 and P1 truncate their factor shares locally by kx and ky
// bits (0 = none); the Beaver triple [a]_0, [b]_0, [c]_0 comes from seed_02
// and [a]_1, [b]_1 from seed_12 (stream TAG_MUL, the block layout of Alg. 8's
// triple), P2 forms [c]_1 = (a0 + a1)(b0 + b1) - c0; d = x - a and e = y - b
// are opened; [z]_0 = de + d[b]_0 + e[a]_0 + [c]_0, [z]_1 = d[b]_1 + e[a]_1
// + [c]_1; then both truncate the product shares by kz bits.
//
// Each thread handles V consecutive elements with one 16-byte vector load
// per input share and one vector store per output share; the grid strides
// over vectors and a scalar loop finishes the ragged tail.  Reads 32 B and
// writes 16 B per element at l = 64 against ~200 integer operations (three
// Philox blocks and the product), so HBM bounds it.
#include "bc_device.h"
#include "internal.h"

namespace bc {

struct MulKArgs {
    const void* x0;
    const void* x1;
    const void* y0;
    const void* y1;
    void* z0;
    void* z1;
    uint64_t n, elem_base, mask;
    uint32_t kx, ky, kz;
    Stream s02, s12;
};

// Alg. 1 on one share pair in Z_{2^l}: P0 cut(a, k), P1 -cut(-b, k).  With
// k = 0 this is the plain reduction of both shares.
template <typename T>
__device__ __forceinline__ void secureml(T& a, T& b, uint32_t k, T mask) {
    const T nb = (T)((T)0 - b) & mask;
    a = (T)(a & mask) >> k;
    b = (T)((T)0 - (T)(nb >> k)) & mask;
}

template <typename T>
__device__ __forceinline__ void mul_element(T x0, T x1, T y0, T y1, uint64_t g, const MulKArgs& A, T mask, T& z0,
                                            T& z1) {
    secureml<T>(x0, x1, A.kx, mask);
    secureml<T>(y0, y1, A.ky, mask);
    const StreamAt r02 = A.s02.at(g);
    const Words4 w0 = r02.block(TAG_MUL, 0);
    const Words4 w1 = r02.block(TAG_MUL, 1);
    const Words4 w2 = A.s12.block(g, TAG_MUL, 0);
    const T a0 = (T)join64(w0.w0, w0.w1), b0 = (T)join64(w0.w2, w0.w3), c0 = (T)join64(w1.w0, w1.w1);
    const T a1 = (T)join64(w2.w0, w2.w1), b1 = (T)join64(w2.w2, w2.w3);
    const T c1 = (T)((T)(a0 + a1) * (T)(b0 + b1) - c0);                 // P2
    const T d = (T)(x0 - a0 + x1 - a1);                                  // opened x - a
    const T e = (T)(y0 - b0 + y1 - b1);                                  // opened y - b
    T p0 = (T)(d * (T)(e + b0) + e * a0 + c0);                          // de + d[b]_0 + e[a]_0 + [c]_0
    T p1 = (T)(d * b1 + e * a1 + c1);
    secureml<T>(p0, p1, A.kz, mask);
    z0 = p0;
    z1 = p1;
}

template <typename T, int V>
__global__ __launch_bounds__(256) void k_mul(MulKArgs A) {
    const T* X0 = static_cast<const T*>(A.x0);
    const T* X1 = static_cast<const T*>(A.x1);
    const T* Y0 = static_cast<const T*>(A.y0);
    const T* Y1 = static_cast<const T*>(A.y1);
    T* Z0 = static_cast<T*>(A.z0);
    T* Z1 = static_cast<T*>(A.z1);
    const T mask = (T)A.mask;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t nv = A.n / V;
    for (uint64_t v = tid; v < nv; v += stride) {
        const vec_t<T, V> a = ld_nt(reinterpret_cast<const vec_t<T, V>*>(X0 + v * V));
        const vec_t<T, V> b = ld_nt(reinterpret_cast<const vec_t<T, V>*>(X1 + v * V));
        const vec_t<T, V> c = ld_nt(reinterpret_cast<const vec_t<T, V>*>(Y0 + v * V));
        const vec_t<T, V> d = ld_nt(reinterpret_cast<const vec_t<T, V>*>(Y1 + v * V));
        vec_t<T, V> o0, o1;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            T r0, r1;
            mul_element<T>(a[k], b[k], c[k], d[k], A.elem_base + v * V + k, A, mask, r0, r1);
            o0[k] = r0;
            o1[k] = r1;
        }
        st_nt(reinterpret_cast<vec_t<T, V>*>(Z0 + v * V), o0);
        st_nt(reinterpret_cast<vec_t<T, V>*>(Z1 + v * V), o1);
    }
    for (uint64_t i = nv * V + tid; i < A.n; i += stride) {
        T r0, r1;
        mul_element<T>(X0[i], X1[i], Y0[i], Y1[i], A.elem_base + i, A, mask, r0, r1);
        Z0[i] = r0;
        Z1[i] = r1;
    }
}

template <typename T>
static hipError_t launch_mul_t(const MulLaunch& L, hipStream_t st) {
    constexpr int V = 16 / (int)sizeof(T);
    const bool vec = (((uintptr_t)L.x0 | (uintptr_t)L.x1 | (uintptr_t)L.y0 | (uintptr_t)L.y1 | (uintptr_t)L.z0 |
                       (uintptr_t)L.z1) & 15u) == 0;
    MulKArgs A;
    A.x0 = L.x0;
    A.x1 = L.x1;
    A.y0 = L.y0;
    A.y1 = L.y1;
    A.z0 = L.z0;
    A.z1 = L.z1;
    A.n = L.n;
    A.elem_base = L.elem_base;
    A.mask = L.ell >= 64 ? ~0ull : ((1ull << L.ell) - 1);
    A.kx = L.kx;
    A.ky = L.ky;
    A.kz = L.kz;
    A.s02 = Stream{L.s02.k0, L.s02.k1, L.s02.n0, L.s02.n1};
    A.s12 = Stream{L.s12.k0, L.s12.k1, L.s12.n0, L.s12.n1};
    const uint64_t work = vec ? (L.n + V - 1) / V : L.n;
    uint64_t grid = (work + 255) / 256;
    if (grid > (uint64_t)L.grid_cap) grid = (uint64_t)L.grid_cap;
    if (grid == 0) grid = 1;
    if (vec)
        hipLaunchKernelGGL((k_mul<T, V>), dim3((unsigned)grid), dim3(256), 0, st, A);
    else
        hipLaunchKernelGGL((k_mul<T, 1>), dim3((unsigned)grid), dim3(256), 0, st, A);
    return hipGetLastError();
}

hipError_t launch_mul(const MulLaunch& L, hipStream_t st) {
    return L.ell > 32 ? launch_mul_t<uint64_t>(L, st) : launch_mul_t<uint32_t>(L, st);
}

}  // namespace bc
