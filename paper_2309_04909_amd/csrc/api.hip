// C ABI of libbicop.so (declared in include/bicop.h): argument validation,
// parameter derivation, message accounting and kernel launches.  Every check
// runs on the host before anything is enqueued; no exception crosses the ABI.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>

#include "internal.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(BC_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// ---------------------------------------------------------------- primes

uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }

uint64_t powmod64(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod64(r, a, m);
        a = mulmod64(a, a, m);
        e >>= 1;
    }
    return r;
}

// Deterministic Miller-Rabin: these twelve bases decide every n < 3.3e24.
bool is_prime64(uint64_t n) {
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (uint64_t q : bases)
        if (n % q == 0) return n == q;
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        ++s;
    }
    for (uint64_t a : bases) {
        uint64_t x = powmod64(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < s; ++i) {
            x = mulmod64(x, x, n);
            if (x == n - 1) {
                comp = false;
                break;
            }
        }
        if (comp) return false;
    }
    return true;
}

// Computed once per l_x (Miller-Rabin on every call would dominate the host
// cost of a small DReLU call).
uint64_t default_prime(uint32_t lx) {
    if (lx < 1 || lx > 32) return 0;
    static std::atomic<uint64_t> cache[33];
    uint64_t c = cache[lx].load(std::memory_order_relaxed);
    if (c) return c;
    c = (1ull << (lx + 1)) - 1;
    while (!is_prime64(c)) --c;
    cache[lx].store(c, std::memory_order_relaxed);
    return c;
}

// is_prime64 with a one-entry memo of the last explicit prime that passed.
bool is_prime_cached(uint64_t p) {
    static std::atomic<uint64_t> last{0};
    if (p != 0 && last.load(std::memory_order_relaxed) == p) return true;
    if (!is_prime64(p)) return false;
    last.store(p, std::memory_order_relaxed);
    return true;
}

// ------------------------------------------------------------ validation

uint32_t width_of_ring(uint32_t ell) { return ell <= 32 ? 4u : 8u; }

bool aligned(const void* p, uint32_t w) { return ((uintptr_t)p % w) == 0; }

int check_params(const bc_drelu_params* prm, bc_drelu_params* out) {
    if (!prm) return fail(BC_ERR_NULL, "params is NULL");
    if (prm->reserved != 0) return fail(BC_ERR_ARG, "params.reserved must be 0");
    if (prm->ell < 1 || prm->ell > 64) return fail(BC_ERR_RING, "ell = %u outside [1, 64]", prm->ell);
    if (prm->lx < 1 || prm->lx > 32) return fail(BC_ERR_WINDOW, "lx = %u outside [1, 32]", prm->lx);
    if ((uint64_t)prm->k_lo + 2ull * prm->lx > prm->ell)
        return fail(BC_ERR_WINDOW, "k_lo + 2 lx = %u exceeds ell = %u", prm->k_lo + 2 * prm->lx, prm->ell);
    const uint64_t dp = default_prime(prm->lx);
    uint64_t p = prm->p ? prm->p : dp;
    const uint64_t lo = 1ull << prm->lx, hi = 1ull << (prm->lx + 1);
    if (!(lo < p && p < hi) || (p != dp && !is_prime_cached(p)))
        return fail(BC_ERR_PRIME, "p = %llu is not a prime in (2^%u, 2^%u)", (unsigned long long)p, prm->lx, prm->lx + 1);
    if (out) {
        *out = *prm;
        out->p = p;
    }
    return BC_OK;
}

// A record's description against the op, resolved setting and n of the call
// that reads it.
int check_desc(const bc_rand_desc* d, uint32_t op, const bc_drelu_params& r, uint64_t n, uint64_t nonce,
               uint64_t elem_base) {
    if (!d) return fail(BC_ERR_NULL, "record description is NULL");
    if (d->magic != BC_RAND_MAGIC) return fail(BC_ERR_ARG, "record description was not filled by bc_rand_expand");
    if (d->op != op || d->prm.ell != r.ell || d->prm.lx != r.lx || d->prm.k_lo != r.k_lo || d->prm.p != r.p ||
        d->n != n)
        return fail(BC_ERR_ARG,
                    "record was expanded for op %u, l = %u, l_x = %u, k_lo = %u, p = %llu, n = %llu; the call has op "
                    "%u, l = %u, l_x = %u, k_lo = %u, p = %llu, n = %llu",
                    d->op, d->prm.ell, d->prm.lx, d->prm.k_lo, (unsigned long long)d->prm.p,
                    (unsigned long long)d->n, op, r.ell, r.lx, r.k_lo, (unsigned long long)r.p,
                    (unsigned long long)n);
    if (d->nonce != nonce || d->elem_base != elem_base)
        return fail(BC_ERR_ARG, "record was expanded for nonce %llu, elem_base %llu; the call has %llu, %llu",
                    (unsigned long long)d->nonce, (unsigned long long)d->elem_base, (unsigned long long)nonce,
                    (unsigned long long)elem_base);
    const uint64_t need = bc::rand_offsets(r.lx + 1, op == BC_OP_RELU, width_of_ring(r.ell), n).total;
    if (d->bytes < need)
        return fail(BC_ERR_WORKSPACE, "record holds %llu of %llu bytes", (unsigned long long)d->bytes,
                    (unsigned long long)need);
    return BC_OK;
}

int account(uint32_t op, const bc_drelu_params& r, uint64_t n, bc_msg_acct* a) {
    memset(a, 0, sizeof(*a));
    const uint64_t npos = r.lx + 1;
    const uint64_t pbits = 64 - (uint64_t)__builtin_clzll(r.p);      // ceil(log2 p) = l_x + 1
    const uint64_t wbits = npos * pbits;                              // (l_x + 1)^2
    const uint64_t pbytes = r.p < (1ull << 32) ? 4 : 8;
    const uint64_t rbytes = width_of_ring(r.ell);
    a->bits[0] = a->bits[1] = wbits * n;
    a->stored_bytes[0] = a->stored_bytes[1] = npos * pbytes * n;
    a->bits[2] = a->bits[3] = (uint64_t)r.ell * n;
    a->stored_bytes[2] = a->stored_bytes[3] = rbytes * n;
    if (op == BC_OP_RELU) {
        a->bits[3] += (uint64_t)r.ell * n;                           // [c]_1, preprocessing
        a->stored_bytes[3] += rbytes * n;
        a->bits[4] = a->bits[5] = (uint64_t)r.ell * n;                // d-shares
        a->stored_bytes[4] = a->stored_bytes[5] = rbytes * n;
    }
    a->rounds = 2;
    if (op == BC_OP_RSS_DRELU || op == BC_OP_RSS_RELU) {
        // links 2, 3 already carry D''; P2 also sends [s]_0 to P0.  Every
        // product of replicated shares ([s][t], and the ReLU's) reshares z_j
        // from P_j to P_{j-1}: P0->P2, P1->P0, P2->P1.
        const uint64_t prods = op == BC_OP_RSS_RELU ? 2 : 1;
        a->bits[2] += (uint64_t)r.ell * n;
        a->stored_bytes[2] += rbytes * n;
        for (int l : {0, 5, 3}) {
            a->bits[l] += prods * r.ell * n;
            a->stored_bytes[l] += prods * rbytes * n;
        }
        if (op == BC_OP_RSS_RELU) a->rounds = 3;
    }
    return BC_OK;
}

bc::StreamKey stream_key(uint64_t seed, uint64_t nonce) {
    return bc::StreamKey{(uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)nonce, (uint32_t)(nonce >> 32)};
}

constexpr uint64_t kMaxIndex = 1ull << 48;

// Element i of a call has global index elem_base + i, which must stay below
// 2^48 (the counter layout of the draws).
int check_indices(uint64_t n, uint64_t elem_base) {
    if (elem_base > kMaxIndex || n > kMaxIndex - elem_base)
        return fail(BC_ERR_ARG, "element indices must stay below 2^48");
    return BC_OK;
}

int grid_cap(int per_cu) { return bc::device_cus() * per_cu; }

// Schedule table: blocks per compute unit of the grid, per kernel kind, window
// count, storage width (4 or 8 bytes) and op (DReLU or ReLU), 0 = the
// built-in default.  Written by bc_set_schedule.  Settings that share a
// window count but not a ring width or an op run different kernels, so each
// keeps its own entry.
constexpr int kKinds = 7;
std::atomic<uint32_t> g_sched[kKinds][34][2][2];
// blocks per CU of each kind; for BC_SCHED_GROUP the largest lanes per element,
// for BC_SCHED_GROUP_FILL the waves per SIMD lane groups may fill
constexpr uint32_t kDefaultBpc[kKinds] = {16, 8, 16, 16, 8, 8, 1};

uint32_t sched_value(uint32_t kind, uint32_t npos, uint32_t width, bool relu) {
    const uint32_t v =
        g_sched[kind][npos < 34 ? npos : 0][width == 4 ? 0 : 1][relu ? 1 : 0].load(std::memory_order_relaxed);
    return v ? v : kDefaultBpc[kind];
}

// Lanes per element of a DReLU/ReLU call: calls too small to give every SIMD
// `fill` waves at one lane per element (BC_SCHED_GROUP_FILL, default one)
// spread each element over 8 or 4 lanes (up to the group schedule's limit)
// while the grid stays within `fill` waves per SIMD; beyond that the lanes'
// repeated shuffle costs more than the latency it hides (measured
// on MI355X per window count; the tuner sets both limits).  Capturing calls
// keep one lane per element.
int lanes_per_element(uint32_t npos, uint32_t width, bool relu, uint64_t n, bool capture) {
    if (capture) return 1;
    const uint32_t gmax = sched_value(BC_SCHED_GROUP, npos, width, relu);
    const uint64_t fill = sched_value(BC_SCHED_GROUP_FILL, npos, width, relu);
    const uint64_t target = (uint64_t)bc::device_cus() * 4 * 64 * fill;   // `fill` waves on each of 4 SIMDs per CU
    if (gmax >= 8 && n * 8 <= target) return 8;
    if (gmax >= 4 && n * 4 <= target) return 4;
    return 1;
}

uint64_t sched_grid(uint32_t kind, uint32_t npos, uint32_t width, bool relu, uint64_t work_blocks) {
    const uint64_t cap = (uint64_t)grid_cap((int)sched_value(kind, npos, width, relu));
    const uint64_t g = work_blocks < cap ? work_blocks : cap;
    return g ? g : 1;
}

int drelu_common(uint32_t op, const void* x0, const void* x1, void* y0, void* y1, uint64_t n,
                 const bc_drelu_params* prm, const bc_seeds* seeds, uint64_t elem_base, void* capture,
                 bc_msg_acct* acct, void* stream, uint32_t ell_in = 0, uint32_t k_in = 0) {
    bc_drelu_params r;
    int rc = check_params(prm, &r);
    if (rc) return rc;
    if (k_in) {
        if (ell_in < 2 || ell_in > 64 || (uint64_t)r.ell + k_in != ell_in)
            return fail(BC_ERR_RING, "truncation must map Z_2^%u onto the ring of params (ell = %u, k1 = %u)", ell_in,
                        r.ell, k_in);
        if (width_of_ring(ell_in) != width_of_ring(r.ell))
            return fail(BC_ERR_RING, "input ring %u and output ring %u must share a storage width", ell_in, r.ell);
    }
    if (!seeds) return fail(BC_ERR_NULL, "seeds is NULL");
    if (int rc_i = check_indices(n, elem_base)) return rc_i;
    if (acct) account(op, r, n, acct);
    if (n == 0) return BC_OK;
    if (!x0 || !x1 || !y0 || !y1) return fail(BC_ERR_NULL, "share pointer is NULL");
    const uint32_t w = width_of_ring(r.ell);
    if (!aligned(x0, w) || !aligned(x1, w) || !aligned(y0, w) || !aligned(y1, w))
        return fail(BC_ERR_ALIGN, "share pointers must be %u-byte aligned", w);
    if (capture && !aligned(capture, r.p < (1ull << 32) ? 4 : 8))
        return fail(BC_ERR_ALIGN, "capture buffer misaligned");
    bc::DreluLaunch L;
    L.x0 = x0;
    L.x1 = x1;
    L.y0 = y0;
    L.y1 = y1;
    L.cap = capture;
    L.n = n;
    L.elem_base = elem_base;
    L.ell = r.ell;
    L.lx = r.lx;
    L.k_lo = r.k_lo;
    L.npos = r.lx + 1;
    L.k_in = k_in;
    L.p = r.p;
    L.s01 = stream_key(seeds->seed01, seeds->nonce);
    L.s02 = stream_key(seeds->seed02, seeds->nonce);
    L.s12 = stream_key(seeds->seed12, seeds->nonce);
    L.block = 256;
    L.group = lanes_per_element(L.npos, w, op == BC_OP_RELU, n, capture != nullptr);
    L.grid = (int)sched_grid(BC_SCHED_FUSED, L.npos, w, op == BC_OP_RELU, (n * (uint64_t)L.group + 255) / 256);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    const bool relu = op == BC_OP_RELU;
    if (r.ell > 32) {
        if (L.npos <= 12)
            e = relu ? bc::launch_relu_u64_lo(L, st) : bc::launch_drelu_u64_lo(L, st);
        else if (L.npos <= 24)
            e = relu ? bc::launch_relu_u64_mid(L, st) : bc::launch_drelu_u64_mid(L, st);
        else
            e = relu ? bc::launch_relu_u64_hi(L, st) : bc::launch_drelu_u64_hi(L, st);
    } else {
        e = relu ? bc::launch_relu_u32(L, st) : bc::launch_drelu_u32(L, st);
    }
    if (e != hipSuccess) return hip_fail(e, op == BC_OP_RELU ? "relu launch" : "drelu launch");
    return BC_OK;
}

int rss_common(bool relu, const void* x0, const void* x1, const void* x2, void* y0, void* y1, void* y2, uint64_t n,
               const bc_drelu_params* prm, const bc_rss_seeds* seeds, uint64_t elem_base, void* capture,
               bc_msg_acct* acct, void* stream) {
    bc_drelu_params r;
    int rc = check_params(prm, &r);
    if (rc) return rc;
    if (!seeds) return fail(BC_ERR_NULL, "seeds is NULL");
    if (int rc_i = check_indices(n, elem_base)) return rc_i;
    if (acct) account(relu ? BC_OP_RSS_RELU : BC_OP_RSS_DRELU, r, n, acct);
    if (n == 0) return BC_OK;
    if (!x0 || !x1 || !x2 || !y0 || !y1 || !y2) return fail(BC_ERR_NULL, "share pointer is NULL");
    const uint32_t w = width_of_ring(r.ell);
    if (!aligned(x0, w) || !aligned(x1, w) || !aligned(x2, w) || !aligned(y0, w) || !aligned(y1, w) ||
        !aligned(y2, w))
        return fail(BC_ERR_ALIGN, "share pointers must be %u-byte aligned", w);
    if (capture && !aligned(capture, r.p < (1ull << 32) ? 4 : 8))
        return fail(BC_ERR_ALIGN, "capture buffer misaligned");
    bc::RssLaunch L;
    L.x0 = x0;
    L.x1 = x1;
    L.x2 = x2;
    L.y0 = y0;
    L.y1 = y1;
    L.y2 = y2;
    L.cap = capture;
    L.n = n;
    L.elem_base = elem_base;
    L.p = r.p;
    L.ell = r.ell;
    L.lx = r.lx;
    L.k_lo = r.k_lo;
    L.npos = r.lx + 1;
    L.relu = relu;
    L.s01 = stream_key(seeds->seed01, seeds->nonce);
    L.s12 = stream_key(seeds->seed12, seeds->nonce);
    L.s012 = stream_key(seeds->seed012, seeds->nonce);
    L.s2 = stream_key(seeds->seed2, seeds->nonce);
    L.grid = (int)sched_grid(BC_SCHED_FUSED, L.npos, w, relu, (n + 255) / 256);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (r.ell > 32)
        e = L.npos <= 12 ? bc::launch_rss_u64_lo(L, st)
                         : (L.npos <= 24 ? bc::launch_rss_u64_mid(L, st) : bc::launch_rss_u64_hi(L, st));
    else
        e = bc::launch_rss_u32(L, st);
    if (e != hipSuccess) return hip_fail(e, relu ? "rss relu launch" : "rss drelu launch");
    return BC_OK;
}

int split_common(bc::SplitLaunch::Kind kind, uint32_t party, const void* in0, const void* in1, void* out0, void* out1,
                 uint64_t n, const bc_drelu_params* prm, const bc_seeds* seeds, uint64_t elem_base, void* stream) {
    bc_drelu_params r;
    int rc = check_params(prm, &r);
    if (rc) return rc;
    if (!seeds) return fail(BC_ERR_NULL, "seeds is NULL");
    if (int rc_i = check_indices(n, elem_base)) return rc_i;
    if (n == 0) return BC_OK;
    const bool reply = kind == bc::SplitLaunch::REPLY;
    if (!in0 || !out0 || (reply && (!in1 || !out1))) return fail(BC_ERR_NULL, "array pointer is NULL");
    const uint32_t w = width_of_ring(r.ell);
    // send reads a share and writes words; reply reads words and writes shares; finish shares to shares
    const uint32_t win = kind == bc::SplitLaunch::REPLY ? 4 : w;
    const uint32_t wout = kind == bc::SplitLaunch::SEND ? 4 : w;
    if (!aligned(in0, win) || (in1 && !aligned(in1, win)) || !aligned(out0, wout) || (out1 && !aligned(out1, wout)))
        return fail(BC_ERR_ALIGN, "arrays must be aligned to their element size");
    bc::SplitLaunch L;
    L.kind = kind;
    L.party = party;
    L.in0 = in0;
    L.in1 = in1;
    L.out0 = out0;
    L.out1 = out1;
    L.n = n;
    L.elem_base = elem_base;
    L.p = r.p;
    L.ell = r.ell;
    L.lx = r.lx;
    L.k_lo = r.k_lo;
    L.npos = r.lx + 1;
    L.s01 = stream_key(seeds->seed01, seeds->nonce);
    L.s02 = stream_key(seeds->seed02, seeds->nonce);
    L.grid = (int)sched_grid(kind == bc::SplitLaunch::FINISH ? BC_SCHED_STREAM : BC_SCHED_FUSED,
                             kind == bc::SplitLaunch::FINISH ? 0 : L.npos, w, false, (n + 255) / 256);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (kind == bc::SplitLaunch::FINISH)
        e = bc::launch_split_finish(L, st);
    else if (r.ell > 32)
        e = L.npos <= 17 ? bc::launch_split_u64_lo(L, st) : bc::launch_split_u64_hi(L, st);
    else
        e = bc::launch_split_u32(L, st);
    if (e != hipSuccess) return hip_fail(e, "split drelu launch");
    return BC_OK;
}

int batch_plan(const bc_segment* segs, uint32_t nseg, const bc_drelu_params* prm, uint32_t tile_elems, void* plan,
               uint64_t plan_bytes) {
    if (!segs || !plan) return fail(BC_ERR_NULL, "segments or plan is NULL");
    if (nseg < 1 || nseg > (1u << 20)) return fail(BC_ERR_ARG, "nseg = %u outside [1, 2^20]", nseg);
    if (plan_bytes < bc_batch_plan_bytes(nseg)) return fail(BC_ERR_WORKSPACE, "plan buffer too small");
    bc_drelu_params r;
    int rc = check_params(prm, &r);
    if (rc) return rc;
    if (tile_elems == 0) tile_elems = 1024;
    if (tile_elems > (1u << 20)) return fail(BC_ERR_ARG, "tile_elems = %u above 2^20", tile_elems);
    const uint32_t w = width_of_ring(r.ell);
    uint8_t* base = static_cast<uint8_t*>(plan);
    bc::BatchPlanHeader* h = reinterpret_cast<bc::BatchPlanHeader*>(base);
    bc_segment* out = reinterpret_cast<bc_segment*>(base + sizeof(bc::BatchPlanHeader));
    uint64_t* tb = reinterpret_cast<uint64_t*>(base + sizeof(bc::BatchPlanHeader) + sizeof(bc_segment) * nseg);
    uint64_t tiles = 0, elems = 0;
    for (uint32_t i = 0; i < nseg; ++i) {
        const bc_segment& s = segs[i];
        if (s.op != BC_OP_DRELU && s.op != BC_OP_RELU) return fail(BC_ERR_ARG, "segment %u: unknown op %u", i, s.op);
        if (s.k_in && (r.ell + s.k_in > 64 || width_of_ring(r.ell + s.k_in) != w))
            return fail(BC_ERR_RING, "segment %u: input ring %u + %u must share the storage width of %u", i, r.ell,
                        s.k_in, r.ell);
        if (s.elem_base > kMaxIndex || s.n > kMaxIndex - s.elem_base)
            return fail(BC_ERR_ARG, "segment %u: element indices must stay below 2^48", i);
        if (s.n && (!s.x0 || !s.x1 || !s.y0 || !s.y1)) return fail(BC_ERR_NULL, "segment %u: NULL share pointer", i);
        if (s.n && (!aligned(s.x0, w) || !aligned(s.x1, w) || !aligned(s.y0, w) || !aligned(s.y1, w)))
            return fail(BC_ERR_ALIGN, "segment %u: share pointers must be %u-byte aligned", i, w);
        if (s.rand) {
            if (!aligned(s.rand, 16)) return fail(BC_ERR_ALIGN, "segment %u: record must be 16-byte aligned", i);
            if (int rc_d = check_desc(s.rand_desc, s.op, r, s.n, s.nonce, s.elem_base)) {
                const int rc_seg = rc_d;
                char why[sizeof(g_err)];
                snprintf(why, sizeof(why), "%s", g_err);
                return fail(rc_seg, "segment %u: %s", i, why);
            }
        }
        out[i] = s;
        tb[i] = tiles;
        tiles += (s.n + tile_elems - 1) / tile_elems;
        elems += s.n;
    }
    tb[nseg] = tiles;
    memset(h, 0, sizeof(*h));
    h->magic = bc::kBatchMagic;
    h->nseg = nseg;
    h->ell = r.ell;
    h->lx = r.lx;
    h->k_lo = r.k_lo;
    h->tile_elems = tile_elems;
    h->p = r.p;
    h->total_tiles = tiles;
    h->total_elems = elems;
    return BC_OK;
}

int batch_run(const void* dev_plan, const void* host_plan, const bc_seeds* seeds, uint32_t grid, void* stream) {
    if (!dev_plan || !host_plan || !seeds) return fail(BC_ERR_NULL, "plan or seeds is NULL");
    const bc::BatchPlanHeader* h = static_cast<const bc::BatchPlanHeader*>(host_plan);
    if (h->magic != bc::kBatchMagic) return fail(BC_ERR_ARG, "host_plan is not a plan from bc_batch_plan");
    if (!aligned(dev_plan, 8)) return fail(BC_ERR_ALIGN, "dev_plan must be 8-byte aligned");
    if (h->total_tiles == 0) return BC_OK;
    const uint8_t* base = static_cast<const uint8_t*>(dev_plan);
    bc::BatchLaunch L;
    L.hdr = reinterpret_cast<const bc::BatchPlanHeader*>(base);
    L.segs = reinterpret_cast<const bc_segment*>(base + sizeof(bc::BatchPlanHeader));
    L.tile_begin = reinterpret_cast<const uint64_t*>(base + sizeof(bc::BatchPlanHeader) + sizeof(bc_segment) * h->nseg);
    L.total_tiles = h->total_tiles;
    L.tile_elems = h->tile_elems;
    L.p = h->p;
    L.ell = h->ell;
    L.k_lo = h->k_lo;
    L.npos = h->lx + 1;
    L.nseg = h->nseg;
    L.s01 = stream_key(seeds->seed01, 0);
    L.s02 = stream_key(seeds->seed02, 0);
    L.s12 = stream_key(seeds->seed12, 0);
    uint64_t g = grid ? grid : sched_grid(BC_SCHED_BATCH, L.npos, width_of_ring(h->ell), false, h->total_tiles);
    if (g > h->total_tiles) g = h->total_tiles;
    L.grid = (int)g;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (h->ell > 32) {
        if (L.npos <= 12) e = bc::launch_batch_u64_lo(L, st);
        else if (L.npos <= 24) e = bc::launch_batch_u64_mid(L, st);
        else e = bc::launch_batch_u64_hi(L, st);
    } else {
        e = bc::launch_batch_u32(L, st);
    }
    return e == hipSuccess ? BC_OK : hip_fail(e, "batch launch");
}

// The offline expansion (expand: writes `rand`, rand_bytes is its size, the
// description goes to desc_out when given) or the online call (reads `rand`,
// whose description desc_in must match the call).
int pre_common(bool expand, uint32_t op, const void* x0, const void* x1, void* y0, void* y1, uint64_t n,
               const bc_drelu_params* prm, const bc_seeds* seeds, uint64_t elem_base, void* rand, uint64_t rand_bytes,
               const bc_rand_desc* desc_in, bc_rand_desc* desc_out, void* capture, bc_msg_acct* acct, void* stream) {
    if (op != BC_OP_DRELU && op != BC_OP_RELU) return fail(BC_ERR_ARG, "unknown op %u", op);
    bc_drelu_params r;
    int rc = check_params(prm, &r);
    if (rc) return rc;
    if (!seeds) return fail(BC_ERR_NULL, "seeds is NULL");
    if (int rc_i = check_indices(n, elem_base)) return rc_i;
    const uint32_t w = width_of_ring(r.ell);
    const bc::RandOffsets o = bc::rand_offsets(r.lx + 1, op == BC_OP_RELU, w, n);
    if (!expand) {
        if (int rc_d = check_desc(desc_in, op, r, n, seeds->nonce, elem_base)) return rc_d;
        rand_bytes = desc_in->bytes;
    }
    if (acct) account(op, r, n, acct);
    if (expand && desc_out) {
        if (rand_bytes < o.total) return fail(BC_ERR_WORKSPACE, "randomness buffer holds %llu of %llu bytes",
                                              (unsigned long long)rand_bytes, (unsigned long long)o.total);
        memset(desc_out, 0, sizeof(*desc_out));
        desc_out->magic = BC_RAND_MAGIC;
        desc_out->op = op;
        desc_out->prm = r;
        desc_out->n = n;
        desc_out->bytes = o.total;
        desc_out->nonce = seeds->nonce;
        desc_out->elem_base = elem_base;
    }
    if (n == 0) return BC_OK;
    if (!rand) return fail(BC_ERR_NULL, "randomness buffer is NULL");
    if (!aligned(rand, 16)) return fail(BC_ERR_ALIGN, "randomness buffer must be 16-byte aligned");
    if (rand_bytes < o.total) return fail(BC_ERR_WORKSPACE, "randomness buffer holds %llu of %llu bytes",
                                          (unsigned long long)rand_bytes, (unsigned long long)o.total);
    if (!expand) {
        if (!x0 || !x1 || !y0 || !y1) return fail(BC_ERR_NULL, "share pointer is NULL");
        if (!aligned(x0, w) || !aligned(x1, w) || !aligned(y0, w) || !aligned(y1, w))
            return fail(BC_ERR_ALIGN, "share pointers must be %u-byte aligned", w);
        if (capture && !aligned(capture, r.p < (1ull << 32) ? 4 : 8))
            return fail(BC_ERR_ALIGN, "capture buffer misaligned");
    }
    bc::PreLaunch L;
    L.x0 = x0;
    L.x1 = x1;
    L.y0 = y0;
    L.y1 = y1;
    L.cap = expand ? nullptr : capture;
    L.rand = rand;
    L.n = n;
    L.elem_base = elem_base;
    L.p = r.p;
    L.ell = r.ell;
    L.k_lo = r.k_lo;
    L.npos = r.lx + 1;
    L.relu = op == BC_OP_RELU;
    L.expand = expand;
    const bc_seeds& sd = *seeds;
    L.s01 = stream_key(sd.seed01, sd.nonce);
    L.s02 = stream_key(sd.seed02, sd.nonce);
    L.s12 = stream_key(sd.seed12, sd.nonce);
    L.grid = (int)sched_grid(expand ? BC_SCHED_EXPAND : BC_SCHED_PRE, L.npos, w, L.relu, (n + 255) / 256);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (r.ell > 32) {
        if (L.npos <= 12) e = bc::launch_pre_u64_lo(L, st);
        else if (L.npos <= 24) e = bc::launch_pre_u64_mid(L, st);
        else e = bc::launch_pre_u64_hi(L, st);
    } else {
        e = bc::launch_pre_u32(L, st);
    }
    return e == hipSuccess ? BC_OK : hip_fail(e, expand ? "expand launch" : "online launch");
}

}  // namespace

namespace bc {

int device_cus() {
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lk(mu);
    if (!cache[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cache[dev] = v;
    }
    return cache[dev];
}

}  // namespace bc

extern "C" {

const char* bc_version(void) { return "bicop 0.1 (gfx950)"; }

const char* bc_strerror(int code) {
    switch (code) {
        case BC_OK: return "ok";
        case BC_ERR_NULL: return "null pointer";
        case BC_ERR_RING: return "invalid ring (l outside [1,64] or k1 + k2 >= l)";
        case BC_ERR_WINDOW: return "invalid window (l_x outside [1,32] or k_lo + 2 l_x > l)";
        case BC_ERR_PRIME: return "invalid prime (not prime or outside (2^l', 2^(l'+1)))";
        case BC_ERR_ALIGN: return "misaligned pointer";
        case BC_ERR_HIP: return "HIP error";
        case BC_ERR_WORKSPACE: return "workspace too small";
        case BC_ERR_ARG: return "invalid argument";
        default: return "unknown error";
    }
}

const char* bc_last_error(void) { return g_err; }

uint64_t bc_default_prime(uint32_t lx) { return default_prime(lx); }

int bc_set_schedule(uint32_t kind, uint32_t npos, uint32_t ring_width, uint32_t op, uint32_t blocks_per_cu) {
    if (kind >= (uint32_t)kKinds) return fail(BC_ERR_ARG, "unknown schedule kind %u", kind);
    if (npos > 33) return fail(BC_ERR_ARG, "npos = %u outside [0, 33]", npos);
    if (ring_width != 4 && ring_width != 8 && ring_width != BC_SCHED_ALL)
        return fail(BC_ERR_ARG, "ring_width = %u: 4, 8 or BC_SCHED_ALL", ring_width);
    if (op != BC_OP_DRELU && op != BC_OP_RELU && op != BC_SCHED_ALL)
        return fail(BC_ERR_ARG, "op = %u: BC_OP_DRELU, BC_OP_RELU or BC_SCHED_ALL", op);
    if (blocks_per_cu > 1024) return fail(BC_ERR_ARG, "blocks_per_cu = %u above 1024", blocks_per_cu);
    for (int wi = 0; wi < 2; ++wi) {
        if (ring_width != BC_SCHED_ALL && (ring_width == 4 ? 0 : 1) != wi) continue;
        for (int oi = 0; oi < 2; ++oi) {
            if (op != BC_SCHED_ALL && (int)op != oi) continue;
            g_sched[kind][npos][wi][oi].store(blocks_per_cu, std::memory_order_relaxed);
        }
    }
    return BC_OK;
}

uint32_t bc_get_schedule(uint32_t kind, uint32_t npos, uint32_t ring_width, uint32_t op) {
    if (kind >= (uint32_t)kKinds || npos > 33) return 0;
    if ((ring_width != 4 && ring_width != 8) || (op != BC_OP_DRELU && op != BC_OP_RELU)) return 0;
    return sched_value(kind, npos, ring_width, op == BC_OP_RELU);
}

int bc_check_params(const bc_drelu_params* prm, bc_drelu_params* resolved) { return check_params(prm, resolved); }

int bc_keybit_params(uint32_t ell, uint32_t f, uint32_t int_bits, uint32_t frac_bits, bc_drelu_params* out) {
    if (!out) return fail(BC_ERR_NULL, "out is NULL");
    if (frac_bits > f) return fail(BC_ERR_WINDOW, "frac_bits = %u exceeds f = %u", frac_bits, f);
    if (int_bits > 64 || frac_bits > 64) return fail(BC_ERR_WINDOW, "window bits above 64");
    bc_drelu_params q{};
    q.ell = ell;
    q.lx = int_bits + frac_bits;
    q.k_lo = f - frac_bits;
    return check_params(&q, out);
}

uint32_t bc_keybit_int_bits(uint64_t bound, uint32_t f) {
    uint32_t c = 0;                                   // ceil(log2(bound)): smallest c with bound <= 2^c
    while (c < 64 && (bound > (1ull << c))) ++c;
    if (bound > (1ull << 63)) c = 64;
    const int64_t i = (int64_t)c - (int64_t)f + 1;
    return i < 1 ? 1u : (uint32_t)i;
}

int bc_msg_account(uint32_t op, const bc_drelu_params* prm, uint64_t n, bc_msg_acct* acct) {
    if (!acct) return fail(BC_ERR_NULL, "acct is NULL");
    if (op > BC_OP_RSS_RELU) return fail(BC_ERR_ARG, "unknown op %u", op);
    bc_drelu_params r;
    int rc = check_params(prm, &r);
    if (rc) return rc;
    return account(op, r, n, acct);
}

int bc_prg_blocks(uint32_t* out, uint64_t n, uint32_t nblocks, uint64_t seed, uint64_t nonce, uint32_t tag,
                  uint64_t elem_base, void* stream) {
    if (nblocks < 1 || nblocks > 256) return fail(BC_ERR_ARG, "nblocks = %u outside [1, 256]", nblocks);
    if (tag > 255) return fail(BC_ERR_ARG, "tag = %u outside [0, 255]", tag);
    if (int rc_i = check_indices(n, elem_base)) return rc_i;
    if (n == 0) return BC_OK;
    if (!out) return fail(BC_ERR_NULL, "out is NULL");
    if (!aligned(out, 4)) return fail(BC_ERR_ALIGN, "out misaligned");
    hipError_t e = bc::launch_prg_blocks(out, n, nblocks, stream_key(seed, nonce), tag, elem_base, grid_cap(16),
                                         (hipStream_t)stream);
    return e == hipSuccess ? BC_OK : hip_fail(e, "prg launch");
}

int bc_zp_mul_add(const uint64_t* a, const uint64_t* b, const uint64_t* d, uint64_t* out, uint64_t n, uint32_t lx,
                  uint64_t p, void* stream) {
    bc_drelu_params q{64, lx, 0, 0, p};
    bc_drelu_params r;
    int rc = check_params(&q, &r);
    if (rc) return rc;
    if (n > kMaxIndex) return fail(BC_ERR_ARG, "n must stay below 2^48");
    if (n == 0) return BC_OK;
    if (!a || !b || !d || !out) return fail(BC_ERR_NULL, "array pointer is NULL");
    if (!aligned(a, 8) || !aligned(b, 8) || !aligned(d, 8) || !aligned(out, 8))
        return fail(BC_ERR_ALIGN, "arrays must be 8-byte aligned");
    bc::ZpLaunch L{a, b, d, out, n, r.p, r.lx + 1, (int)sched_grid(BC_SCHED_STREAM, 0, 8, false, (n + 255) / 256)};
    hipError_t e = bc::launch_zp_mul_add(L, (hipStream_t)stream);
    return e == hipSuccess ? BC_OK : hip_fail(e, "zp_mul_add launch");
}

int bc_trunc_det(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, uint32_t ell, uint32_t k1, uint32_t k2,
                 void* stream) {
    if (ell < 1 || ell > 64) return fail(BC_ERR_RING, "ell = %u outside [1, 64]", ell);
    if ((uint64_t)k1 + k2 >= ell) return fail(BC_ERR_RING, "k1 + k2 = %u must be < ell = %u", k1 + k2, ell);
    if (n == 0) return BC_OK;
    if (!x0 || !x1 || !y0 || !y1) return fail(BC_ERR_NULL, "share pointer is NULL");
    const uint32_t wi = width_of_ring(ell), wo = width_of_ring(ell - k1 - k2);
    if (!aligned(x0, wi) || !aligned(x1, wi) || !aligned(y0, wo) || !aligned(y1, wo))
        return fail(BC_ERR_ALIGN, "share pointers misaligned");
    hipError_t e = bc::launch_trunc_det(x0, x1, y0, y1, n, ell, k1, k2, (int)sched_grid(BC_SCHED_STREAM, 0, wi, false, ~0ull),
                                        (hipStream_t)stream);
    return e == hipSuccess ? BC_OK : hip_fail(e, "trunc_det launch");
}

int bc_trunc_prob(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, uint32_t ell, uint32_t k,
                  void* stream) {
    if (ell < 1 || ell > 64) return fail(BC_ERR_RING, "ell = %u outside [1, 64]", ell);
    if (k >= ell) return fail(BC_ERR_RING, "k = %u must be < ell = %u", k, ell);
    if (n == 0) return BC_OK;
    if (!x0 || !x1 || !y0 || !y1) return fail(BC_ERR_NULL, "share pointer is NULL");
    const uint32_t w = width_of_ring(ell);
    if (!aligned(x0, w) || !aligned(x1, w) || !aligned(y0, w) || !aligned(y1, w))
        return fail(BC_ERR_ALIGN, "share pointers misaligned");
    hipError_t e = bc::launch_trunc_prob(x0, x1, y0, y1, n, ell, k, (int)sched_grid(BC_SCHED_STREAM, 0, w, false, ~0ull),
                                         (hipStream_t)stream);
    return e == hipSuccess ? BC_OK : hip_fail(e, "trunc_prob launch");
}

int bc_mod_switch(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, uint32_t ell_in, uint64_t p,
                  void* stream) {
    if (ell_in < 1 || ell_in > 63) return fail(BC_ERR_RING, "ell_in = %u outside [1, 63]", ell_in);
    const uint64_t lo = 1ull << ell_in;
    const uint64_t hi = ell_in == 63 ? ~0ull : (1ull << (ell_in + 1));
    if (!(lo < p && (p < hi || (ell_in == 63))) || !is_prime_cached(p))
        return fail(BC_ERR_PRIME, "p = %llu is not a prime in (2^%u, 2^%u)", (unsigned long long)p, ell_in, ell_in + 1);
    if (n == 0) return BC_OK;
    if (!x0 || !x1 || !y0 || !y1) return fail(BC_ERR_NULL, "share pointer is NULL");
    const uint32_t wi = width_of_ring(ell_in), wo = p < (1ull << 32) ? 4u : 8u;
    if (!aligned(x0, wi) || !aligned(x1, wi) || !aligned(y0, wo) || !aligned(y1, wo))
        return fail(BC_ERR_ALIGN, "share pointers misaligned");
    hipError_t e = bc::launch_mod_switch(x0, x1, y0, y1, n, ell_in, p, (int)sched_grid(BC_SCHED_STREAM, 0, wi, false, ~0ull),
                                         (hipStream_t)stream);
    return e == hipSuccess ? BC_OK : hip_fail(e, "mod_switch launch");
}

int bc_drelu(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, const bc_drelu_params* prm,
             const bc_seeds* seeds, uint64_t elem_base, void* capture, bc_msg_acct* acct, void* stream) {
    return drelu_common(BC_OP_DRELU, x0, x1, y0, y1, n, prm, seeds, elem_base, capture, acct, stream);
}

uint64_t bc_batch_plan_bytes(uint32_t nseg) {
    return sizeof(bc::BatchPlanHeader) + (uint64_t)sizeof(bc_segment) * nseg + 8ull * (nseg + 1ull);
}

int bc_batch_plan(const bc_segment* segs, uint32_t nseg, const bc_drelu_params* prm, uint32_t tile_elems, void* plan,
                  uint64_t plan_bytes) {
    return batch_plan(segs, nseg, prm, tile_elems, plan, plan_bytes);
}

int bc_batch_run(const void* dev_plan, const void* host_plan, const bc_seeds* seeds, uint32_t grid, void* stream) {
    return batch_run(dev_plan, host_plan, seeds, grid, stream);
}

int bc_batch_run_static(const void* host_plan, const bc_seeds* seeds, uint32_t grid, void* stream) {
    if (!host_plan || !seeds) return fail(BC_ERR_NULL, "plan or seeds is NULL");
    bc::BatchPlanHeader h;
    memcpy(&h, host_plan, sizeof(h));
    if (h.magic != bc::kBatchMagic) return fail(BC_ERR_ARG, "host_plan is not a plan from bc_batch_plan");
    const uint64_t bytes = bc_batch_plan_bytes(h.nseg);
    if (bytes > BC_STATIC_PLAN_BYTES)
        return fail(BC_ERR_WORKSPACE, "plan of %u segments needs %llu bytes; the fixed plan area holds %u (%u segments)",
                    h.nseg, (unsigned long long)bytes, (unsigned)BC_STATIC_PLAN_BYTES, (unsigned)BC_STATIC_MAX_SEGMENTS);
    if (h.total_tiles == 0) return BC_OK;
    void* dev_plan = nullptr;
    hipError_t e = bc::static_plan_upload(host_plan, bytes, (hipStream_t)stream, &dev_plan);
    if (e != hipSuccess) return hip_fail(e, "static plan upload");
    return batch_run(dev_plan, host_plan, seeds, grid, stream);
}

uint64_t bc_rand_bytes(uint32_t op, const bc_drelu_params* prm, uint64_t n) {
    bc_drelu_params r;
    if (op != BC_OP_DRELU && op != BC_OP_RELU) return 0;
    if (check_params(prm, &r)) return 0;
    return bc::rand_offsets(r.lx + 1, op == BC_OP_RELU, width_of_ring(r.ell), n).total;
}

int bc_rand_expand(void* rand, uint64_t rand_bytes, uint64_t n, uint32_t op, const bc_drelu_params* prm,
                   const bc_seeds* seeds, uint64_t elem_base, bc_rand_desc* desc, void* stream) {
    return pre_common(true, op, nullptr, nullptr, nullptr, nullptr, n, prm, seeds, elem_base, rand, rand_bytes, nullptr,
                      desc, nullptr, nullptr, stream);
}

int bc_drelu_pre(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, const bc_drelu_params* prm,
                 const bc_seeds* seeds, uint64_t elem_base, const void* rand, const bc_rand_desc* desc, void* capture,
                 bc_msg_acct* acct, void* stream) {
    return pre_common(false, BC_OP_DRELU, x0, x1, y0, y1, n, prm, seeds, elem_base, const_cast<void*>(rand), 0, desc,
                      nullptr, capture, acct, stream);
}

int bc_relu_pre(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, const bc_drelu_params* prm,
                const bc_seeds* seeds, uint64_t elem_base, const void* rand, const bc_rand_desc* desc, void* capture,
                bc_msg_acct* acct, void* stream) {
    return pre_common(false, BC_OP_RELU, x0, x1, y0, y1, n, prm, seeds, elem_base, const_cast<void*>(rand), 0, desc,
                      nullptr, capture, acct, stream);
}

int bc_trunc_drelu(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, uint32_t ell_in, uint32_t k1,
                   const bc_drelu_params* prm, const bc_seeds* seeds, uint64_t elem_base, void* capture,
                   bc_msg_acct* acct, void* stream) {
    if (k1 == 0) return fail(BC_ERR_RING, "k1 must be > 0 (use bc_drelu)");
    return drelu_common(BC_OP_DRELU, x0, x1, y0, y1, n, prm, seeds, elem_base, capture, acct, stream, ell_in, k1);
}

int bc_trunc_relu(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, uint32_t ell_in, uint32_t k1,
                  const bc_drelu_params* prm, const bc_seeds* seeds, uint64_t elem_base, void* capture,
                  bc_msg_acct* acct, void* stream) {
    if (k1 == 0) return fail(BC_ERR_RING, "k1 must be > 0 (use bc_relu)");
    return drelu_common(BC_OP_RELU, x0, x1, y0, y1, n, prm, seeds, elem_base, capture, acct, stream, ell_in, k1);
}

uint32_t bc_msg_words(uint32_t npos) { return npos >= 2 && npos <= 33 ? (npos * npos + 31) / 32 : 0; }

int bc_drelu_send(uint32_t party, const void* x, uint32_t* msg, uint64_t n, const bc_drelu_params* prm,
                  const bc_seeds* seeds, uint64_t elem_base, void* stream) {
    if (party > 1) return fail(BC_ERR_ARG, "party = %u: the senders are 0 and 1", party);
    return split_common(bc::SplitLaunch::SEND, party, x, nullptr, msg, nullptr, n, prm, seeds, elem_base, stream);
}

int bc_drelu_reply(const uint32_t* msg0, const uint32_t* msg1, void* d0, void* d1, uint64_t n,
                   const bc_drelu_params* prm, const bc_seeds* seeds, uint64_t elem_base, void* stream) {
    return split_common(bc::SplitLaunch::REPLY, 0, msg0, msg1, d0, d1, n, prm, seeds, elem_base, stream);
}

int bc_drelu_finish(uint32_t party, const void* d, void* y, uint64_t n, const bc_drelu_params* prm,
                    const bc_seeds* seeds, uint64_t elem_base, void* stream) {
    if (party > 1) return fail(BC_ERR_ARG, "party = %u: the finishers are 0 and 1", party);
    return split_common(bc::SplitLaunch::FINISH, party, d, nullptr, y, nullptr, n, prm, seeds, elem_base, stream);
}

int bc_mul_trunc(const void* x0, const void* x1, const void* y0, const void* y1, void* z0, void* z1, uint64_t n,
                 uint32_t ell, uint32_t f, uint32_t order, const bc_seeds* seeds, uint64_t elem_base, void* stream) {
    if (ell < 1 || ell > 64) return fail(BC_ERR_RING, "ell = %u outside [1, 64]", ell);
    bc::MulLaunch L;
    L.kx = L.ky = L.kz = 0;
    if (order == BC_TRUNC_NONE) {
        if (f) return fail(BC_ERR_ARG, "f must be 0 without truncation");
    } else if (order == BC_TRUNC_AFTER) {
        if (f >= ell) return fail(BC_ERR_RING, "f = %u must be below ell = %u", f, ell);
        L.kz = f;
    } else if (order == BC_TRUNC_BEFORE) {
        if (f - f / 2 >= ell) return fail(BC_ERR_RING, "ceil(f/2) = %u must be below ell = %u", f - f / 2, ell);
        L.kx = f / 2;
        L.ky = f - f / 2;
    } else {
        return fail(BC_ERR_ARG, "unknown truncation order %u", order);
    }
    if (!seeds) return fail(BC_ERR_NULL, "seeds is NULL");
    if (int rc_i = check_indices(n, elem_base)) return rc_i;
    if (n == 0) return BC_OK;
    if (!x0 || !x1 || !y0 || !y1 || !z0 || !z1) return fail(BC_ERR_NULL, "share pointer is NULL");
    const uint32_t w = width_of_ring(ell);
    if (!aligned(x0, w) || !aligned(x1, w) || !aligned(y0, w) || !aligned(y1, w) || !aligned(z0, w) ||
        !aligned(z1, w))
        return fail(BC_ERR_ALIGN, "share pointers must be %u-byte aligned", w);
    L.x0 = x0;
    L.x1 = x1;
    L.y0 = y0;
    L.y1 = y1;
    L.z0 = z0;
    L.z1 = z1;
    L.n = n;
    L.elem_base = elem_base;
    L.ell = ell;
    L.s02 = stream_key(seeds->seed02, seeds->nonce);
    L.s12 = stream_key(seeds->seed12, seeds->nonce);
    L.grid_cap = (int)sched_grid(BC_SCHED_STREAM, 0, w, false, ~0ull);
    hipError_t e = bc::launch_mul(L, (hipStream_t)stream);
    return e == hipSuccess ? BC_OK : hip_fail(e, "mul launch");
}

int bc_rss_drelu(const void* x0, const void* x1, const void* x2, void* y0, void* y1, void* y2, uint64_t n,
                 const bc_drelu_params* prm, const bc_rss_seeds* seeds, uint64_t elem_base, void* capture,
                 bc_msg_acct* acct, void* stream) {
    return rss_common(false, x0, x1, x2, y0, y1, y2, n, prm, seeds, elem_base, capture, acct, stream);
}

int bc_rss_relu(const void* x0, const void* x1, const void* x2, void* y0, void* y1, void* y2, uint64_t n,
                const bc_drelu_params* prm, const bc_rss_seeds* seeds, uint64_t elem_base, void* capture,
                bc_msg_acct* acct, void* stream) {
    return rss_common(true, x0, x1, x2, y0, y1, y2, n, prm, seeds, elem_base, capture, acct, stream);
}

int bc_relu(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, const bc_drelu_params* prm,
            const bc_seeds* seeds, uint64_t elem_base, void* capture, bc_msg_acct* acct, void* stream) {
    return drelu_common(BC_OP_RELU, x0, x1, y0, y1, n, prm, seeds, elem_base, capture, acct, stream);
}

}  // extern "C"
