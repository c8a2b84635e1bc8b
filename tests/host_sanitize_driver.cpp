// Drives the host side of libbicop's C ABI on the CPU: parameter validation,
// default primes and Miller-Rabin, key-bit windows, message accounting,
// record sizes, ragged-batch plans, the schedule table and every argument
// check of the compute calls (n = 0, NULL, misaligned and out-of-range
// arguments), so that a build with AddressSanitizer and
// UndefinedBehaviorSanitizer sees all of it.  No kernel is launched: every
// call either fails validation or has nothing to do.  Prints a digest of the
// results and "driver done".
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "bicop.h"

static uint64_t g_digest = 1469598103934665603ull;
static void mix(uint64_t v) {
    g_digest ^= v;
    g_digest *= 1099511628211ull;
}

static uint64_t lcg(uint64_t& s) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return s >> 11;
}

int main() {
    mix((uint64_t)strlen(bc_version()));
    for (int c = 1; c >= -9; --c) mix(strlen(bc_strerror(c)));
    mix(strlen(bc_last_error()));

    // default primes for every window width, and the ones outside the range
    uint64_t prime_sum = 0;
    for (uint32_t lx = 0; lx <= 40; ++lx) prime_sum += bc_default_prime(lx);
    printf("default_prime_sum %llu\n", (unsigned long long)prime_sum);
    mix(prime_sum);

    // parameter validation over a grid, with default and explicit primes
    uint64_t seed = 12345;
    int ok = 0, bad = 0;
    for (uint32_t ell = 0; ell <= 66; ++ell)
        for (uint32_t lx = 0; lx <= 34; lx += 1)
            for (uint32_t k_lo = 0; k_lo <= 40; k_lo += 7) {
                bc_drelu_params prm = {ell, lx, k_lo, 0, 0};
                bc_drelu_params res;
                int rc = bc_check_params(&prm, &res);
                mix((uint64_t)(rc + 16));
                (rc == BC_OK ? ok : bad)++;
                if (lx >= 1 && lx <= 32) {
                    prm.p = (1ull << lx) + 1 + lcg(seed) % (1ull << lx);   // often composite
                    mix((uint64_t)(bc_check_params(&prm, nullptr) + 16));
                }
                prm.p = 0;
                prm.reserved = 1;
                mix((uint64_t)(bc_check_params(&prm, &res) + 16));
            }
    mix((uint64_t)(bc_check_params(nullptr, nullptr) + 16));
    printf("check_params ok %d bad %d\n", ok, bad);

    // key-bit windows
    for (uint32_t ell = 1; ell <= 64; ell += 3)
        for (uint32_t f = 0; f <= 40; f += 5)
            for (uint32_t ib = 0; ib <= 34; ib += 3)
                for (uint32_t fb = 0; fb <= 20; fb += 4) {
                    bc_drelu_params out;
                    mix((uint64_t)(bc_keybit_params(ell, f, ib, fb, &out) + 16));
                }
    mix((uint64_t)(bc_keybit_params(64, 13, 17, 1, nullptr) + 16));
    for (int e = 0; e < 64; ++e)
        for (uint32_t f = 0; f <= 64; f += 8) mix(bc_keybit_int_bits(1ull << e, f));
    mix(bc_keybit_int_bits(~0ull, 0));

    // message accounting and record sizes
    for (uint32_t op = 0; op <= 5; ++op)
        for (uint32_t lx = 1; lx <= 32; ++lx) {
            bc_drelu_params prm = {64, lx, 0, 0, 0};
            bc_msg_acct a;
            for (uint64_t n : {0ull, 1ull, 1000ull, 1ull << 40}) {
                int rc = bc_msg_account(op, &prm, n, &a);
                mix((uint64_t)(rc + 16));
                if (rc == BC_OK)
                    for (int l = 0; l < BC_NLINKS; ++l) mix(a.bits[l] ^ a.stored_bytes[l]);
                mix(bc_rand_bytes(op, &prm, n));
            }
            mix((uint64_t)(bc_msg_account(op, &prm, 10, nullptr) + 16));
        }
    for (uint32_t npos = 0; npos <= 40; ++npos) mix(bc_msg_words(npos));

    // ragged-batch plans: random valid and invalid segment tables
    bc_drelu_params prm = {51, 7, 11, 0, 0};
    for (int trial = 0; trial < 200; ++trial) {
        const uint32_t nseg = 1 + (uint32_t)(lcg(seed) % 1200);
        std::vector<bc_segment> segs(nseg);
        std::vector<bc_rand_desc> descs(nseg);
        for (uint32_t i = 0; i < nseg; ++i) {
            bc_segment& s = segs[i];
            memset(&s, 0, sizeof(s));
            const uint64_t r = lcg(seed);
            s.n = r % 5000;
            uintptr_t base = 0x100000 + 0x1000 * (uintptr_t)i;
            s.x0 = (const void*)(base + ((r >> 20) % 97 == 0 ? 4 : 0));           // rarely misaligned
            s.x1 = (const void*)(base + 0x100);
            s.y0 = (void*)(base + 0x200);
            s.y1 = (r >> 30) % 211 == 0 ? nullptr : (void*)(base + 0x300);      // rarely NULL
            s.elem_base = (r >> 13) % 1000 == 0 ? (1ull << 48) - 3 : 10 * i;
            s.nonce = r;
            s.op = (r >> 40) % 301 == 0 ? 7u : (uint32_t)((r >> 8) & 1);
            s.k_in = (r >> 44) % 3 == 0 ? 13u : ((r >> 46) % 53 == 0 ? 14u : 0u);
            if ((r >> 50) % 4 == 0) {
                s.rand = (const void*)(0x40000000ull + 0x10000ull * i + ((r >> 52) % 89 == 0 ? 8 : 0));
                bc_rand_desc& d = descs[i];
                // the description of a real expansion, sometimes for another n or op, or missing
                bc_rand_expand(nullptr, 0, 0, s.op & 1, &prm, nullptr, 0, &d, nullptr);   // refused: seeds NULL
                bc_seeds sd0 = {1, 2, 3, 4};
                const uint64_t dn = s.n + ((r >> 55) % 71 == 0 ? 1 : 0);
                sd0.nonce = (r >> 58) % 67 == 0 ? s.nonce + 1 : s.nonce;            // rarely another nonce
                bc_rand_expand(nullptr, ~0ull, 0, s.op & 1, &prm, &sd0, 0, &d, nullptr);  // n = 0: fills d
                d.n = dn;
                d.elem_base = s.elem_base;
                d.bytes = bc_rand_bytes(s.op & 1, &prm, dn);
                s.rand_desc = (r >> 57) % 97 == 0 ? nullptr : &d;
            }
        }
        const uint64_t nbytes = bc_batch_plan_bytes(nseg);
        std::vector<uint8_t> plan(nbytes);
        const uint32_t tile = (uint32_t)(lcg(seed) % 3000);
        int rc = bc_batch_plan(segs.data(), nseg, &prm, tile, plan.data(), nbytes);
        mix((uint64_t)(rc + 16));
        mix((uint64_t)(bc_batch_plan(segs.data(), nseg, &prm, tile, plan.data(), nbytes - 1) + 16));
        if (rc == BC_OK) {
            uint64_t words = 0;
            for (uint64_t b = 0; b < nbytes; b += 8) {
                uint64_t w;
                memcpy(&w, plan.data() + b, 8);
                words += w;
            }
            mix(words);
            // more segments than the fixed plan area holds: refused before any HIP call
            if (nbytes > BC_STATIC_PLAN_BYTES) {
                bc_seeds sd = {1, 2, 3, 4};
                mix((uint64_t)(bc_batch_run_static(plan.data(), &sd, 0, nullptr) + 16));
            }
        }
    }
    {
        std::vector<uint8_t> junk(256, 0xAB);
        bc_seeds sd = {1, 2, 3, 4};
        mix((uint64_t)(bc_batch_run(junk.data(), junk.data(), &sd, 0, nullptr) + 16));
        mix((uint64_t)(bc_batch_run_static(junk.data(), &sd, 0, nullptr) + 16));
        mix((uint64_t)(bc_batch_run_static(nullptr, &sd, 0, nullptr) + 16));
        mix((uint64_t)(bc_batch_plan(nullptr, 1, &prm, 0, junk.data(), 256) + 16));
    }

    // the schedule table: every kind, window count, width and op, and wildcards
    for (uint32_t kind = 0; kind <= 7; ++kind)
        for (uint32_t npos = 0; npos <= 35; ++npos)
            for (uint32_t w : {0u, 4u, 8u, 16u, BC_SCHED_ALL})
                for (uint32_t op : {0u, 1u, 2u, BC_SCHED_ALL}) {
                    mix((uint64_t)(bc_set_schedule(kind, npos, w, op, (npos * 7 + kind) % 9) + 16));
                    mix(bc_get_schedule(kind, npos, w, op));
                }
    for (uint32_t kind = 0; kind <= 5; ++kind) bc_set_schedule(kind, BC_SCHED_ALL, BC_SCHED_ALL, BC_SCHED_ALL, 0);

    // argument checks of the compute calls: nothing valid with n > 0 reaches a launch here
    bc_seeds sd = {1, 2, 3, 4};
    bc_rss_seeds rsd = {1, 2, 3, 4, 5, 6};
    bc_msg_acct acct;
    const void* P = (const void*)0x10000;
    void* Q = (void*)0x20000;
    void* M = (void*)0x20004;                          // 4-byte aligned only
    for (uint32_t ell = 0; ell <= 65; ell += 13)
        for (uint32_t lx : {0u, 1u, 7u, 18u, 32u, 33u}) {
            bc_drelu_params p2 = {ell, lx, 3, 0, 0};
            for (uint64_t n : {0ull, 5ull, 1ull << 49}) {
                mix((uint64_t)(bc_drelu(P, P, Q, Q, n, &p2, &sd, 0, nullptr, &acct, nullptr) + 16));
                mix((uint64_t)(bc_relu(nullptr, P, Q, Q, n, &p2, &sd, 0, nullptr, nullptr, nullptr) + 16));
                mix((uint64_t)(bc_drelu(P, P, M, Q, n, &p2, &sd, 0, nullptr, nullptr, nullptr) + 16));
                mix((uint64_t)(bc_relu(P, P, Q, Q, n, &p2, nullptr, 0, nullptr, nullptr, nullptr) + 16));
                mix((uint64_t)(bc_trunc_drelu(P, P, Q, Q, n, ell + 13, 13, &p2, &sd, 0, nullptr, nullptr, nullptr) + 16));
                mix((uint64_t)(bc_trunc_relu(P, P, Q, Q, n, ell + 1, 0, &p2, &sd, 0, nullptr, nullptr, nullptr) + 16));
                mix((uint64_t)(bc_rss_drelu(P, P, P, Q, Q, Q, n, &p2, &rsd, 0, nullptr, &acct, nullptr) + 16));
                mix((uint64_t)(bc_rss_relu(P, nullptr, P, Q, Q, Q, n, &p2, &rsd, 0, nullptr, nullptr, nullptr) + 16));
                bc_rand_desc d;
                memset(&d, 0, sizeof(d));
                mix((uint64_t)(bc_rand_expand(M, 0, n, 0, &p2, &sd, 0, &d, nullptr) + 16));
                mix((uint64_t)(bc_drelu_pre(P, P, Q, Q, n, &p2, &sd, 0, nullptr, &d, nullptr, nullptr, nullptr) + 16));
                mix((uint64_t)(bc_relu_pre(P, P, Q, Q, n, &p2, &sd, 0, M, &d, nullptr, nullptr, nullptr) + 16));
                mix((uint64_t)(bc_relu_pre(P, P, Q, Q, n, &p2, &sd, 0, M, nullptr, nullptr, nullptr, nullptr) + 16));
                mix((uint64_t)(bc_drelu_pre(P, P, Q, Q, n, &p2, nullptr, 0, M, &d, nullptr, nullptr, nullptr) + 16));
                mix((uint64_t)(bc_drelu_pre(P, P, Q, Q, n, &p2, &sd, 9, M, &d, nullptr, nullptr, nullptr) + 16));
                mix((uint64_t)(bc_drelu_send(2, P, (uint32_t*)Q, n, &p2, &sd, 0, nullptr) + 16));
                mix((uint64_t)(bc_drelu_reply(nullptr, (const uint32_t*)P, Q, Q, n, &p2, &sd, 0, nullptr) + 16));
                mix((uint64_t)(bc_drelu_finish(0, P, M, n, &p2, &sd, 0, nullptr) + 16));
                mix((uint64_t)(bc_trunc_det(P, P, Q, Q, n, ell, 13, 60, nullptr) + 16));
                mix((uint64_t)(bc_trunc_prob(P, nullptr, Q, Q, n, ell, ell, nullptr) + 16));
                mix((uint64_t)(bc_mod_switch(P, P, Q, Q, n, ell, 1ull << ell % 64, nullptr) + 16));
                mix((uint64_t)(bc_mul_trunc(P, P, P, P, Q, Q, n, ell, 26, 3, &sd, 0, nullptr) + 16));
                mix((uint64_t)(bc_zp_mul_add((const uint64_t*)P, nullptr, (const uint64_t*)P, (uint64_t*)Q, n, lx,
                                             0, nullptr) + 16));
                mix((uint64_t)(bc_prg_blocks((uint32_t*)Q, n, 0, 1, 2, 300, 0, nullptr) + 16));
            }
        }
    printf("digest %016llx\n", (unsigned long long)g_digest);
    printf("driver done\n");
    return 0;
}
