// Independent pin for the oracle's Philox4x32-10: rocRAND's header-only
// engine, compiled for the host.  Reads "seed c0 c1 c2 c3" lines on stdin and
// prints the four output words of that (key, counter) block.
//
// rocRAND's engine(seed, subsequence, offset) starts from counter
// (0, 0, sub_lo, sub_hi) and skips offset/4 blocks, so counter
// (c0, c1, c2, c3) is reached with subsequence = c3:c2 and
// offset = 4 * (c1:c0) (which needs c1 < 2^30).
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned long long seed;
    unsigned int c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        unsigned long long off = 4ull * (((unsigned long long)c1 << 32) | c0);
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
