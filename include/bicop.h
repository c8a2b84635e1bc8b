/*
 * bicop.h -- C ABI of the Bicoptor 2.0 share-local DReLU/ReLU hot path on
 * AMD MI355X (gfx950).  Implemented by libbicop.so.
 *
 * Three parties are simulated on one GPU.  P0 holds share [x]_0, P1 holds
 * [x]_1, P2 is the helper.  The protocol calls take both share-holders'
 * arrays (the replicated-sharing calls all three shares), so P2's view
 * exists only inside the library; round-1 messages live in registers and
 * are counted in bytes (bc_msg_account), and a caller-provided capture
 * buffer can materialise them for inspection.  The parties-apart calls
 * (bc_drelu_send, bc_drelu_reply, bc_drelu_finish) run one party's part
 * each, with the messages bit-packed in device memory.
 *
 * Conventions for every entry point below:
 *  - Pointers named x*, y*, z*, d*, msg*, capture, rand and out are DEVICE
 *    pointers owned by the caller.  None of these calls allocates or frees
 *    device memory, and none retains a pointer after it returns.
 *  - Storage width follows the ring.  An element of Z_{2^l} is a uint32_t
 *    when l <= 32, else a uint64_t.  An element of Z_p is a uint32_t when
 *    p < 2^32, else a uint64_t.  Inputs are read modulo 2^l, so bits above
 *    l are ignored.  Outputs are canonical: each value is < the modulus.
 *  - Arrays are dense, element i at index i.  Every pointer must be aligned
 *    to its element size.
 *  - y may equal x (in place).  Partial overlap is not allowed.
 *  - Calls are asynchronous.  They validate arguments on the host, enqueue
 *    one kernel on `stream` (a hipStream_t; NULL is the null stream) and
 *    return.  n == 0 enqueues nothing and returns BC_OK.
 *  - Calls are stateless and thread-safe.  No C++ exception crosses the ABI.
 *  - Element indices: element i of a call has global index elem_base + i.
 *    It must be < 2^48.  All randomness of an element is a pure function of
 *    (seeds, nonce, global index).  The same element therefore gets the same
 *    result alone, inside a batch, or under any launch configuration.
 *
 * Interface choices, with their reasons:
 *  - Streams are `void*` holding a hipStream_t: this header then needs no HIP
 *    include, and bindings (ctypes) pass torch's raw stream handle through.
 *  - Alignment is to the element size, not 16 bytes: the streaming kernels
 *    take 16-byte vectors where the pointers allow and a scalar path
 *    otherwise, so views at any element offset are valid inputs.
 *  - Rings of 1..64 bits and windows of l_x >= 1: every step is defined and
 *    computed exactly there.  That the sign comes out right needs l_x >= 3
 *    and inputs in the guard-bit domain |x| < 2^(k_lo + l_x - 1), a property
 *    of the inputs that bc_keybit_int_bits sizes, not of the call.
 *  - The ragged batch is three calls (bc_batch_plan_bytes, bc_batch_plan on
 *    the host, bc_batch_run launching exactly one kernel) instead of one
 *    call with a workspace: the plan is validated and built once per batch
 *    shape, and every run is a single kernel a HIP graph can capture.
 */
#ifndef BICOP_H
#define BICOP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
#define BC_OK              0
#define BC_ERR_NULL       -1  /* a required pointer is NULL                      */
#define BC_ERR_RING       -2  /* l outside [1, 64], or k1 + k2 >= l              */
#define BC_ERR_WINDOW     -3  /* l_x outside [1, 32], or k_lo + 2 l_x > l        */
#define BC_ERR_PRIME      -4  /* p not prime, or p outside (2^l', 2^(l'+1))      */
#define BC_ERR_ALIGN      -5  /* a pointer is not aligned to its element size    */
#define BC_ERR_HIP        -6  /* a HIP call failed; bc_last_error() has detail   */
#define BC_ERR_WORKSPACE  -7  /* workspace / plan buffer too small               */
#define BC_ERR_ARG        -8  /* other invalid argument (op, n, index range)     */

#define BC_OP_DRELU     0u
#define BC_OP_RELU      1u
#define BC_OP_RSS_DRELU 2u   /* replicated sharing, Alg. drelu2 */
#define BC_OP_RSS_RELU  3u

/* DReLU/ReLU setting (Alg. 7 "Setting" plus the key-bit window of Sec. 6.1).
 *   ell  : ring bit length l, shares in Z_{2^l}, 1..64
 *   lx   : window width l_x, 1..32.  The protocol looks at n = l_x + 1
 *          windows of l_x bits.
 *   k_lo : low bits dropped below the key-bit window.  Window i (0..l_x) is
 *          the deterministic truncation trc(x, k_lo+i, l-l_x-k_lo-i)
 *          (Alg. 5).  Requires k_lo + 2 l_x <= l.
 *   p    : prime of the modulo switch (Alg. 6), 2^l_x < p < 2^(l_x+1).
 *          0 selects the largest prime below 2^(l_x+1) (bc_default_prime). */
typedef struct {
    uint32_t ell;
    uint32_t lx;
    uint32_t k_lo;
    uint32_t reserved;   /* must be 0 */
    uint64_t p;
} bc_drelu_params;

/* Pre-shared seeds (Sec. 2.1): seed01 of P0/P1, seed02 of P0/P2, seed12 of
 * P1/P2.  nonce separates calls that reuse the seeds; it is per call/job. */
typedef struct {
    uint64_t seed01;
    uint64_t seed02;
    uint64_t seed12;
    uint64_t nonce;
} bc_seeds;

/* Seeds of the replicated-sharing calls (the Setting of Alg. drelu2): the
 * fields of bc_seeds, then seed012 of all three parties and seed2 of P2
 * alone.  seed02 is not drawn from by these calls. */
typedef struct {
    uint64_t seed01;
    uint64_t seed02;
    uint64_t seed12;
    uint64_t nonce;
    uint64_t seed012;
    uint64_t seed2;
} bc_rss_seeds;

/* Links, in this order: P0->P2, P1->P2, P2->P0, P2->P1, P0->P1, P1->P0. */
#define BC_NLINKS 6
typedef struct {
    uint64_t bits[BC_NLINKS];          /* theoretical bits for the whole call  */
    uint64_t stored_bytes[BC_NLINKS];  /* bytes the values occupy in storage   */
    uint32_t rounds;                   /* online communication rounds          */
    uint32_t reserved;
} bc_msg_acct;

/* ----------------------------------------------------------- diagnostics */

/* Library version string (static storage). */
const char* bc_version(void);

/* Text of an error code (static storage). */
const char* bc_strerror(int code);

/* Detail of the last error raised in the calling thread (thread-local
 * storage, valid until the next call from that thread). */
const char* bc_last_error(void);

/* Largest prime below 2^(lx+1), for lx in [1, 32]; 0 otherwise.  This is
 * the reading of "a prime whose bit length is l_x + 1" (notation table). */
uint64_t bc_default_prime(uint32_t lx);

/* Validate a DReLU/ReLU setting.  If `resolved` is not NULL it receives
 * the setting with p filled in.  Returns BC_OK or the error code the
 * compute calls would return.  Host only. */
int bc_check_params(const bc_drelu_params* prm, bc_drelu_params* resolved);

/* Key-bit window of Sec. 6.1 (Tab. 5's "integer + fractional" notation)
 * for fixed-point values with f fractional bits: the DReLU keeps int_bits
 * integer bits (counting any guard bit) and frac_bits fractional bits, so
 * it drops the low k_lo = f - frac_bits bits and tests l_x = int_bits +
 * frac_bits bits above them.  Fills *out with (ell, l_x, k_lo, default p)
 * and validates it like bc_check_params; frac_bits > f is BC_ERR_WINDOW.
 * Host only. */
int bc_keybit_params(uint32_t ell, uint32_t f, uint32_t int_bits, uint32_t frac_bits, bc_drelu_params* out);

/* Integer bits of the key-bit window, guard bit included, for values with
 * |x| < bound at f fractional bits: the smallest i >= 1 with
 * bound <= 2^(f + i - 1), so that |x| < 2^(k_lo + l_x - 1) holds for any
 * frac_bits (the guard-bit domain on which the sign is exact outside
 * |x| < 2^k_lo).  Host only. */
uint32_t bc_keybit_int_bits(uint64_t bound, uint32_t f);

/* Message accounting for one call of `op` (BC_OP_*) on n elements.
 * Round 1: each of P0, P1 sends l_x + 1 values of Z_p, i.e. (l_x+1)^2 bits
 * per element (Tab. 1, Sec. 5.4).  DReLU round 2: one Z_{2^l} share to each
 * of P0 and P1 (P2's reply).  ReLU (Alg. 8): e to P0 and P1, [c]_1 to P1
 * (preprocessing), d-shares between P0 and P1.  RSS DReLU (Alg. drelu2):
 * round 1 as above; D'' (l bits) to P0 and P1; preprocessing [s]_0 to P0 and
 * the reshare of [s][t] on P0->P2, P1->P0, P2->P1.  RSS ReLU: one more such
 * reshare, in a third round.  Host only. */
int bc_msg_account(uint32_t op, const bc_drelu_params* prm, uint64_t n, bc_msg_acct* acct);

/* Raw Philox4x32-10 blocks, for checking the generator.  Writes
 * out[(i * nblocks + b) * 4 + w], the word w of block b of stream `tag` for
 * the element with global index elem_base + i, under key `seed` and
 * `nonce`.  The counter layout is the one used by the protocol kernels:
 * c0 = g mod 2^32, c1 = (g >> 32) | tag << 16 | b << 24, (c2, c3) = nonce.
 * nblocks in [1, 256], tag in [0, 255].  out is n * nblocks * 4 uint32_t. */
int bc_prg_blocks(uint32_t* out, uint64_t n, uint32_t nblocks, uint64_t seed,
                  uint64_t nonce, uint32_t tag, uint64_t elem_base, void* stream);

/* The Z_p multiply-add of the DReLU/ReLU kernels, elementwise, for checking
 * the field arithmetic (Alg. 7: the masked and reshared messages
 * v r + z).  For a setting (lx, p) as in bc_drelu_params (p = 0:
 * the default prime) it writes out[i] = (a[i] b[i] + d[i]) mod p using the
 * same field code as the kernels: fp32-quotient products, Mersenne or
 * pseudo-Mersenne folds (with b and d shifted to the top of the word, as the
 * kernels keep their masks for the default prime at l_x = 16..20), fp64
 * quotient, Barrett or the 128-bit product.
 * Requires a[i], b[i] < p and d[i] <= p (other values give unspecified
 * results).  Device arrays of n uint64, 8-byte aligned. */
int bc_zp_mul_add(const uint64_t* a, const uint64_t* b, const uint64_t* d, uint64_t* out, uint64_t n,
                  uint32_t lx, uint64_t p, void* stream);

/* ------------------------------------------------------------ schedules */

/* Kernel kinds of the schedule table. */
#define BC_SCHED_FUSED   0u   /* bc_drelu, bc_relu                       */
#define BC_SCHED_STREAM  1u   /* bc_trunc_det, bc_trunc_prob, bc_mod_switch */
#define BC_SCHED_PRE     2u   /* bc_drelu_pre, bc_relu_pre               */
#define BC_SCHED_EXPAND  3u   /* bc_rand_expand                          */
#define BC_SCHED_BATCH   4u   /* bc_batch_run with grid = 0              */
#define BC_SCHED_GROUP   5u   /* bc_drelu, bc_relu on small n: the value is
                                 the largest number of lanes per element
                                 (1 = off, 4, 8; default 8)                */
#define BC_SCHED_GROUP_FILL 6u /* bc_drelu, bc_relu: lane groups are used
                                 while n times the lanes per element stays
                                 within this many waves per SIMD (default 1) */

/* Wildcard of bc_set_schedule's ring_width and op. */
#define BC_SCHED_ALL 0xFFFFFFFFu

/* Process-wide launch schedule, keyed by (kind, npos, ring_width, op):
 *   npos        window count l_x + 1 (0..33; the streaming kernels use 0)
 *   ring_width  4 or 8, the storage width of the call's ring (the input
 *               ring for the streaming calls)
 *   op          BC_OP_DRELU or BC_OP_RELU (the replicated-sharing calls use
 *               the entry of their 2-of-2 counterpart; kinds without an op,
 *               the streaming kernels, the ragged batch and the parties-apart
 *               calls, use BC_OP_DRELU)
 * Settings that share a window count but not a width or an op run different
 * kernel instances, so each keeps its own entry.  The grid is capped at
 * blocks_per_cu blocks of 256 threads per compute unit; each thread then
 * handles n / (grid * 256) elements.  0 restores the built-in default.
 * BC_SCHED_ALL as ring_width or op sets every matching entry.  Results do
 * not depend on the schedule.  Set it before launching (the autotuner
 * paper_2309_04909_amd/tune.py writes a table the binding applies). */
int bc_set_schedule(uint32_t kind, uint32_t npos, uint32_t ring_width, uint32_t op, uint32_t blocks_per_cu);

/* The blocks per compute unit in effect for (kind, npos, ring_width, op),
 * ring_width 4 or 8 and op BC_OP_DRELU or BC_OP_RELU; 0 if invalid. */
uint32_t bc_get_schedule(uint32_t kind, uint32_t npos, uint32_t ring_width, uint32_t op);

/* --------------------------------------------------------- truncation */

/* Deterministic truncation, Alg. 4 (k2 = 0) and Alg. 5 (Sec. 5.1).
 * In  : x0, x1 -- n shares of Z_{2^ell} (width of ell).
 * Out : y0, y1 -- n shares of Z_{2^(ell-k1-k2)} (width of ell-k1-k2):
 *       P0: y0 = cut(x0, k1, k2) mod 2^(ell-k1-k2)
 *       P1: y1 = -cut(-x1 mod 2^ell, k1, k2) mod 2^(ell-k1-k2)
 *       They reconstruct to floor(x / 2^k1) + e0 in the smaller ring, with
 *       e0 in {0, 1} and no e1 term.
 * k1 low bits and k2 high bits are dropped; requires k1 + k2 < ell. */
int bc_trunc_det(const void* x0, const void* x1, void* y0, void* y1, uint64_t n,
                 uint32_t ell, uint32_t k1, uint32_t k2, void* stream);

/* SecureML probabilistic truncation, Alg. 1 (Sec. 2.4).
 * In/out shares of Z_{2^ell} (same width):
 *   P0: y0 = cut(x0, k) mod 2^ell;  P1: y1 = -cut(-x1 mod 2^ell, k) mod 2^ell.
 * Fails (the e1 term of Sec. 3) with probability |x| / 2^ell over the mask.
 * Requires k < ell. */
int bc_trunc_prob(const void* x0, const void* x1, void* y0, void* y1, uint64_t n,
                  uint32_t ell, uint32_t k, void* stream);

/* ------------------------------------------------------- modulo switch */

/* Modulo switch Z_{2^ell_in} -> Z_p, Alg. 6 (Sec. 5.3).
 * In  : x0, x1 -- n shares of Z_{2^ell_in}, ell_in in [1, 63].
 * Out : y0, y1 -- n shares of Z_p (uint32_t if p < 2^32, else uint64_t):
 *       P0: y0 = 2^ell_in mod p if x0 = 0, else x0 mod p
 *       P1: y1 = p + x1 - 2^ell_in mod p
 *       They reconstruct to 0 mod p exactly when x = 0 mod 2^ell_in.
 * p must be prime with 2^ell_in < p < 2^(ell_in+1). */
int bc_mod_switch(const void* x0, const void* x1, void* y0, void* y1, uint64_t n,
                  uint32_t ell_in, uint64_t p, void* stream);

/* ---------------------------------------------------------- DReLU / ReLU */

/* Bicoptor 2.0 DReLU, Alg. 7 (Sec. 5.4), all three parties in one kernel.
 * In  : x0, x1 -- n shares of x in Z_{2^ell}.
 * Out : y0, y1 -- n shares of DReLU(x) in Z_{2^ell}.  With k_lo = 0,
 *       DReLU(x) = [x > 0] for 0 < |x| < 2^(l_x-1), and DReLU(0) = t (the
 *       random flip).  With key bits, the band |x| < 2^k_lo follows the
 *       carry of the dropped bits.
 * Randomness: t and the shuffle from seed01, r_i in Z_p^* (mask) and z_i
 *       in Z_p (reshare) from seed01, P2's resharing of its bit from
 *       seed02.  Draws are documented with bc_prg_blocks.
 * capture: NULL, or a device buffer of 2 * n * (l_x + 1) elements of Z_p
 *       (uint32_t if p < 2^32, else uint64_t).  It receives the round-1
 *       messages [w]_0 then [w]_1, element-major, in slot (post-shuffle)
 *       order: capture[(party * n + i) * (l_x+1) + slot].
 * acct: NULL, or receives bc_msg_account(BC_OP_DRELU, prm, n). */
int bc_drelu(const void* x0, const void* x1, void* y0, void* y1, uint64_t n,
             const bc_drelu_params* prm, const bc_seeds* seeds, uint64_t elem_base,
             void* capture, bc_msg_acct* acct, void* stream);

/* UBL Bicoptor 2.0 ReLU, Alg. 8 (appendix): Alg. 7 up to P2's zero test, then the
 * Beaver multiplication x * DReLU(x).  [a]_0, [b]_0 and [c]_0 come from
 * seed02; [a]_1 and [b]_1 come from seed12; P2 forms [c]_1.  Outputs are
 * shares of x * DReLU(x) in Z_{2^ell}, with x at full precision.
 * Arguments as bc_drelu. */
int bc_relu(const void* x0, const void* x1, void* y0, void* y1, uint64_t n,
            const bc_drelu_params* prm, const bc_seeds* seeds, uint64_t elem_base,
            void* capture, bc_msg_acct* acct, void* stream);

/* Truncate, then DReLU / ReLU, in one pass.  x0, x1 are shares of
 * Z_{2^ell_in}; each party first applies the deterministic truncation of
 * Alg. 5 by k1 low bits (P0: cut(x0, k1), P1: -cut(-x1, k1)), giving shares
 * of Z_{2^(ell_in - k1)}, and the DReLU (Alg. 7) / ReLU (Alg. 8) of prm then
 * runs in that ring (prm->ell must equal ell_in - k1; both rings must have
 * the same storage width).  Outputs are shares of Z_{2^prm->ell}; the result
 * is bit-identical to bc_trunc_det followed by bc_drelu / bc_relu, with one
 * read and one write of the shares instead of two of each.  k1 > 0. */
int bc_trunc_drelu(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, uint32_t ell_in, uint32_t k1,
                   const bc_drelu_params* prm, const bc_seeds* seeds, uint64_t elem_base, void* capture,
                   bc_msg_acct* acct, void* stream);
int bc_trunc_relu(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, uint32_t ell_in, uint32_t k1,
                  const bc_drelu_params* prm, const bc_seeds* seeds, uint64_t elem_base, void* capture,
                  bc_msg_acct* acct, void* stream);

/* -------------------------------------------- DReLU with the parties apart */

/* 32-bit words per element of one party's packed round-1 message for
 * npos = l_x + 1 windows: ceil(npos^2 / 32); 0 if npos is outside [2, 33].
 * Host only. */
uint32_t bc_msg_words(uint32_t npos);

/* P0's (party 0) or P1's (party 1) part of Alg. 7's first round, alone: from
 * its own share x (n elements of Z_{2^ell}) the message it sends to P2, with
 * the same draws and values as bc_drelu's capture.  The N = l_x + 1 slot
 * values (each below p < 2^N) are bit-packed: bit b of slot s is bit s N + b
 * of the element's string, word k holds bits 32k .. 32k + 31, and word k of
 * element i is msg[k * n + i] (word-major); the spare high bits are 0.  msg
 * holds bc_msg_words(N) * n uint32_t, 4-byte aligned. */
int bc_drelu_send(uint32_t party, const void* x, uint32_t* msg, uint64_t n, const bc_drelu_params* prm,
                  const bc_seeds* seeds, uint64_t elem_base, void* stream);

/* P2's part: unpacks both parties' messages (as bc_drelu_send writes them),
 * sets D' = 1 when some slot reconstructs to 0 mod p, and writes its reply,
 * a fresh sharing of D' in Z_{2^ell}: d0 = rho (to P0, rho from seed02) and
 * d1 = D' - rho (to P1).  Slot values are not range-checked: a message with
 * a slot value >= p (not one bc_drelu_send wrote) gives an unspecified D'
 * for that element, and nothing else. */
int bc_drelu_reply(const uint32_t* msg0, const uint32_t* msg1, void* d0, void* d1, uint64_t n,
                   const bc_drelu_params* prm, const bc_seeds* seeds, uint64_t elem_base, void* stream);

/* P0's or P1's unflip of its reply share d with the flip bit t of seed01:
 * P0 y = t + (1 - 2t) d, P1 y = (1 - 2t) d, in Z_{2^ell}.  send, reply and
 * finish with the same arguments give bc_drelu's outputs.  y may equal d. */
int bc_drelu_finish(uint32_t party, const void* d, void* y, uint64_t n, const bc_drelu_params* prm,
                    const bc_seeds* seeds, uint64_t elem_base, void* stream);

/* ------------------------------------------------ multiply and truncate */

#define BC_TRUNC_NONE   0u   /* the plain product (f must be 0)                  */
#define BC_TRUNC_AFTER  1u   /* multiply, then Alg. 1 on the product by f bits   */
#define BC_TRUNC_BEFORE 2u   /* Alg. linear: Alg. 1 on x by floor(f/2) bits and
                                on y by ceil(f/2) bits, then multiply            */

/* Elementwise product of 2-of-2 shares with the SecureML truncation (Alg. 1)
 * before the product (truncate-then-multiply, Alg. linear, Sec. 4) or after
 * it (multiply-then-truncate), all three parties in one kernel.
 * In  : x0, x1, y0, y1 -- n shares of x and of y in Z_{2^ell}.
 * Out : z0, z1 -- n shares in Z_{2^ell} of trc(x, f/2) trc(y, f/2)
 *       (BEFORE), trc(x y, f) (AFTER) or x y (NONE), each truncation with
 *       the e0 and e1 of Alg. 1 for its shares.
 * The multiplication uses a Beaver triple: [a]_0, [b]_0, [c]_0 from seed02,
 * [a]_1, [b]_1 from seed12 (tag 6, the block layout of bc_relu's triple),
 * [c]_1 = (a0 + a1)(b0 + b1) - c0 formed by P2; d = x - a and e = y - b are
 * opened between P0 and P1.
 * ell in [1, 64]; f < ell (AFTER), ceil(f/2) < ell (BEFORE), f = 0 (NONE).
 * z may equal x or y (in place).  Other conventions as bc_drelu; seed01 is
 * not drawn from. */
int bc_mul_trunc(const void* x0, const void* x1, const void* y0, const void* y1, void* z0, void* z1, uint64_t n,
                 uint32_t ell, uint32_t f, uint32_t order, const bc_seeds* seeds, uint64_t elem_base, void* stream);

/* ------------------------------------------- replicated sharing (RSS) */

/* Bicoptor 2.0 DReLU over replicated shares, Alg. drelu2 (appendix), all
 * three parties in one kernel.
 * In  : x0, x1, x2 -- the shares [x]_0, [x]_1, [x]_2 of x in Z_{2^ell}
 *       (x = x0 + x1 + x2); P_j holds ([x]_j, [x]_{j+1}), indices mod 3.
 * Out : y0, y1, y2 -- the three shares of DReLU(x) in Z_{2^ell}.  The bit is
 *       the one bc_drelu gives for the 2-of-2 input ([x]_0 + [x]_1, [x]_2)
 *       with the same seed01 and nonce (P0 enters [x]_0 + [x]_1, P1 enters
 *       [x]_2); P2 replies with D'' = s xor D', and the shares are those of
 *       D'' xor s xor t, with D'' added to share 0.
 * Randomness: t, the shuffle, r_i and z_i from seed01 exactly as bc_drelu;
 *       from seed012 the alphas of [t] = (a0 - a2, a1 - a0 + t, a2 - a1),
 *       [s]_1 and the zero sharing of the product [s][t]; [s]_2 from seed12;
 *       P2's bit s from seed2 (tag 5 of the counter layout of bc_prg_blocks).
 * capture: NULL, or the round-1 messages of P0 and P1, laid out as for
 *       bc_drelu.
 * acct: NULL, or receives bc_msg_account(BC_OP_RSS_DRELU, prm, n).
 * y_j may equal x_j.  Other conventions as bc_drelu. */
int bc_rss_drelu(const void* x0, const void* x1, const void* x2, void* y0, void* y1, void* y2, uint64_t n,
                 const bc_drelu_params* prm, const bc_rss_seeds* seeds, uint64_t elem_base, void* capture,
                 bc_msg_acct* acct, void* stream);

/* ReLU over replicated shares (appendix): bc_rss_drelu, then the
 * replicated-sharing product of [x] (full precision) and [DReLU(x)]: P_j
 * forms u_j v_j + u_j v_{j+1} + u_{j+1} v_j plus a zero share from seed012.
 * Outputs are the three shares of x DReLU(x).  Arguments as bc_rss_drelu;
 * acct receives bc_msg_account(BC_OP_RSS_RELU, prm, n). */
int bc_rss_relu(const void* x0, const void* x1, const void* x2, void* y0, void* y1, void* y2, uint64_t n,
                const bc_drelu_params* prm, const bc_rss_seeds* seeds, uint64_t elem_base, void* capture,
                bc_msg_acct* acct, void* stream);

/* ------------------------------------------ precomputed randomness */

/* Everything the parties draw from their seeds is independent of the input
 * (Alg. 7: flip, shuffle, masks, reshares, P2's reply; Alg. 8's
 * preprocessing), so it can be expanded ahead of time and kept resident; the
 * online call then streams shares plus this record.  The record keeps what
 * would cost the online phase its shuffle, its seed_01 draws or a message: the
 * flip and the shuffle, r and z, and for the ReLU P2's [c]_1 of the Beaver
 * triple.  What a party draws from seed_02 or seed_12 alone (rho, and the
 * parties' own triple shares) the online call regenerates from the seeds, so
 * it takes the seeds, nonce and element offset the record was expanded with.
 * Results and messages are bit-identical to bc_drelu / bc_relu with the same
 * seeds, nonce and element indices.
 *
 * Record of n elements (structure of arrays, sections at 256-byte
 * boundaries): the shuffle as bytes sigma(slot) packed four per uint32 with
 * t in bit 7 of the first byte; r and z per slot in N-bit fields,
 * floor(64 / N) to a uint64 (one per uint64 at N = 33); for the ReLU then
 * [c]_1 (ring width). */

/* What a record was expanded for, in host memory: bc_rand_expand fills it,
 * and every call that reads the record checks it against its own op,
 * setting and n before anything is enqueued (a record read with another
 * stride or field packing would give wrong outputs without any error). */
#define BC_RAND_MAGIC 0x44524342u   /* "BCRD" */
typedef struct {
    uint32_t magic;          /* BC_RAND_MAGIC once filled                  */
    uint32_t op;             /* BC_OP_DRELU or BC_OP_RELU                  */
    bc_drelu_params prm;     /* the setting, with p resolved               */
    uint64_t n;              /* elements                                   */
    uint64_t bytes;          /* bytes of the record, bc_rand_bytes(op, prm, n) */
    uint64_t nonce;          /* seeds->nonce of the expansion              */
    uint64_t elem_base;      /* global index of element 0                  */
} bc_rand_desc;

/* Bytes of the record of `op` on n elements; 0 if the setting is invalid. */
uint64_t bc_rand_bytes(uint32_t op, const bc_drelu_params* prm, uint64_t n);

/* Offline: expand the seeds of elements elem_base .. elem_base + n - 1 into
 * `rand` (device, 16-byte aligned, rand_bytes >= bc_rand_bytes).  desc:
 * NULL, or host memory that receives the record's description. */
int bc_rand_expand(void* rand, uint64_t rand_bytes, uint64_t n, uint32_t op, const bc_drelu_params* prm,
                   const bc_seeds* seeds, uint64_t elem_base, bc_rand_desc* desc, void* stream);

/* Online DReLU (Alg. 7) / ReLU (Alg. 8) from an expanded record.  desc is
 * the record's description from bc_rand_expand (host memory, required): a
 * record of another op, setting, n, nonce (seeds->nonce) or elem_base is
 * refused with BC_ERR_ARG.  seeds must be those of the expansion (seed02
 * and seed12 regenerate rho and the parties' triple shares).  Other
 * arguments as bc_drelu. */
int bc_drelu_pre(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, const bc_drelu_params* prm,
                 const bc_seeds* seeds, uint64_t elem_base, const void* rand, const bc_rand_desc* desc, void* capture,
                 bc_msg_acct* acct, void* stream);
int bc_relu_pre(const void* x0, const void* x1, void* y0, void* y1, uint64_t n, const bc_drelu_params* prm,
                const bc_seeds* seeds, uint64_t elem_base, const void* rand, const bc_rand_desc* desc, void* capture,
                bc_msg_acct* acct, void* stream);

/* ------------------------------------------------------ ragged batching */

/* One segment of a ragged batch: a share pair of its own length, op, nonce,
 * global element offset and input truncation, and optionally a precomputed
 * randomness record.  Every element of a segment gets exactly the result of
 * bc_drelu / bc_relu (k_in = 0) or bc_trunc_drelu / bc_trunc_relu with
 * k1 = k_in on that segment, with seeds->nonce = nonce and the same
 * elem_base.  A segment with a record (rand != NULL, from bc_rand_expand for
 * the segment's op, the batch's setting, its n, its nonce and its elem_base
 * under the batch's seeds, as its rand_desc must say) takes its seed_01 draws
 * and P2's [c]_1 from the record, with the same result.  Outputs of one
 * segment must not overlap inputs or outputs of another. */
typedef struct {
    const void* x0;
    const void* x1;
    void* y0;
    void* y1;
    uint64_t n;          /* elements (0 allowed)                       */
    uint64_t elem_base;  /* global index of element 0 (n + base <= 2^48) */
    uint64_t nonce;      /* per-segment nonce                          */
    uint32_t op;         /* BC_OP_DRELU or BC_OP_RELU                   */
    uint32_t k_in;       /* low bits each party first truncates from its
                            input share (Alg. 5); the inputs are then
                            shares of Z_{2^(ell + k_in)}, of the storage
                            width of ell.  0 = none                      */
    const void* rand;    /* NULL, or a device record of bc_rand_expand
                            (16-byte aligned)                          */
    const bc_rand_desc* rand_desc; /* its description (host memory, read
                            by bc_batch_plan only); required with rand  */
} bc_segment;

/* Bytes of the plan buffer for nseg segments: a 64-byte header, the segment
 * table (80 bytes per segment) and the first tile of every segment
 * (8 bytes per segment, plus one). */
uint64_t bc_batch_plan_bytes(uint32_t nseg);

/* Host only.  Validates every segment against `prm` (one setting for the
 * whole batch) and writes the plan into host memory `plan`, of plan_bytes
 * bytes.  Each segment is cut into tiles of tile_elems elements (0 = default
 * 1024; at most 2^20, so that a tile is indexed in 32 bits; BC_ERR_ARG
 * above).  The caller then copies the plan, byte for byte, to device memory
 * it owns.  nseg in [1, 2^20]. */
int bc_batch_plan(const bc_segment* segs, uint32_t nseg, const bc_drelu_params* prm, uint32_t tile_elems,
                  void* plan, uint64_t plan_bytes);

/* One persistent launch over every tile of the plan.  dev_plan is the
 * device copy of host_plan (the host copy selects the kernel; the kernel
 * reads the device copy).  seeds->seed01/02/12 apply to all segments;
 * seeds->nonce is ignored (each segment has its own).  grid = blocks of 256
 * threads (0 = a default filling every compute unit).  Enqueues exactly one
 * kernel and nothing else, so it can be captured into a HIP graph. */
int bc_batch_run(const void* dev_plan, const void* host_plan, const bc_seeds* seeds, uint32_t grid, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): bc_batch_run
 * without a device plan.  The plan built by bc_batch_plan (host memory, read
 * during the call only) is copied, by upload kernels enqueued on `stream`
 * that carry its bytes as launch arguments, into a fixed area of
 * BC_STATIC_PLAN_BYTES in device memory that the library holds on each GPU it
 * runs on until the process ends; the batch kernel then reads it from there.
 * Outputs are those of bc_batch_run on the same plan.  Nothing is allocated:
 * no hipMalloc, hipFree or allocating library call.
 *   - Plans above BC_STATIC_PLAN_BYTES (more than BC_STATIC_MAX_SEGMENTS
 *     segments) fail with BC_ERR_WORKSPACE before anything is enqueued.
 *   - Every call on one GPU shares that GPU's area.  Calls ordered on one
 *     stream are safe; calls that overlap on one GPU (other streams, other
 *     threads without ordering) race for the area and give undefined results.
 *   - The first call on a device looks up the area's address (with that
 *     device current) and keeps it.
 * Other arguments and conventions as bc_batch_run. */
#define BC_STATIC_PLAN_BYTES 65536u
#define BC_STATIC_MAX_SEGMENTS 743u   /* largest nseg with bc_batch_plan_bytes(nseg) <= BC_STATIC_PLAN_BYTES */
int bc_batch_run_static(const void* host_plan, const bc_seeds* seeds, uint32_t grid, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* BICOP_H */
