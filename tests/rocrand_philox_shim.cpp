// Host-side shim over rocRAND's Philox4x32-10 engine (the library's own
// header implementation), used only by the tests to cross-check the
// oracle's generator.  rocRAND's engine keys on (seed lo, seed hi); a
// subsequence advances counter words 2-3 and skipping 4 m numbers advances
// words 0-1 by m, so the first four outputs after subsequence c2 + 2^32 c3,
// an offset of 4 c0 and four skips of 2^32 c1 numbers (c1 2^30 blocks each,
// which keeps every skip below 2^64) are the block of counter
// (c0, c1, c2, c3).
#include <rocrand/rocrand_philox4x32_10.h>

extern "C" void rr_philox_blocks(unsigned long long n, const unsigned *ctr, const unsigned *key, unsigned *out) {
    for (unsigned long long i = 0; i < n; ++i) {
        const unsigned *c = ctr + 4 * i;
        const unsigned long long seed = key[2 * i] | ((unsigned long long)key[2 * i + 1] << 32);
        const unsigned long long sub = c[2] | ((unsigned long long)c[3] << 32);
        rocrand_device::philox4x32_10_engine e(seed, sub, 4ull * c[0]);
        for (int q = 0; q < 4; ++q) e.discard((unsigned long long)c[1] << 32);
        for (int j = 0; j < 4; ++j) out[4 * i + j] = e.next();
    }
}
