// Philox4x32-10 words from rocRAND's header-only engine, an implementation
// independent of the oracle's, for the oracle's Philox pin (test
// infrastructure; host code only, no GPU).  For each input line
// "seed subsequence offset count" it prints `count` 32-bit words, one per
// line: the engine keyed by the 64-bit seed, its 128-bit counter started at
// subsequence * 2^64 + offset / 4, words taken in order.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
    unsigned long long seed, sub, off, count;
    while (std::scanf("%llu %llu %llu %llu", &seed, &sub, &off, &count) == 4) {
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        for (unsigned long long i = 0; i < count; ++i) std::printf("%u\n", e());
    }
    return 0;
}
