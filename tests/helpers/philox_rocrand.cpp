// Prints Philox4x32-10 outputs computed by rocRAND's host-callable engine, for
// (key, counter) pairs read from stdin, one "k0 k1 c0 c1 c2 c3" per line.
// The engine is addressed through its public seed/subsequence/offset API:
// seed = k0 | k1 << 32 and subsequence = c2 | c3 << 32 set the key and the upper
// counter words; offset 4 * c0 and then four discards of c1 << 32 numbers each
// (c1 << 30 blocks) set the lower words, so the counter is (c0, c1, c2, c3);
// four next() calls then return the four words of that block.  Used only to pin
// the oracle's generator.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        rocrand_device::philox4x32_10_engine eng;
        eng.seed(k0 | (k1 << 32), c2 | (c3 << 32), 4ull * c0);
        for (int q = 0; q < 4; ++q) eng.discard(c1 << 32);
        unsigned int w[4];
        for (int i = 0; i < 4; ++i) w[i] = eng.next();
        std::printf("%u %u %u %u\n", w[0], w[1], w[2], w[3]);
    }
    return 0;
}
