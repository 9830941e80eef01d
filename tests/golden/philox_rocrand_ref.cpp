// Independent Philox4x32-10 reference for the oracle tests: rocRAND's
// host-callable philox4x32_10_engine.  Reads lines "c0 c1 c2 c3 k0 k1"
// (decimal uint32) from stdin and prints the four output words of the block
// function for that counter and key.
//
// rocRAND's engine keeps the key as the 64-bit seed (low word first) and a
// 128-bit counter: `subsequence` is added to counter words 2..3 and
// `offset / 4` to words 0..1, so engine(seed, c2 | c3 << 32, 4 * (c0 | c1 << 32))
// returns the block for counter (c0, c1, c2, c3) first.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const unsigned long long seed = k0 | (k1 << 32);
        const unsigned long long sub = c2 | (c3 << 32);
        const unsigned long long lo = c0 | (c1 << 32);
        // offset is a count of 32-bit outputs, so 4 * lo can overflow 64 bits:
        // advance the counter in four quarter steps plus the remainder.
        rocrand_device::philox4x32_10_engine e(seed, sub, 0);
        const unsigned long long quarter = lo >> 2;
        for (int j = 0; j < 4; ++j) e.discard(4ull * quarter);
        e.discard(4ull * (lo & 3ull));
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
