// Prints Philox4x32-10 blocks computed by rocRAND's host-callable engine, for
// the counters and keys read from stdin (one "c0 c1 c2 c3 k0 k1" per line).
// rocRAND's engine sets counter = (offset/4 low, offset/4 high, subsequence
// low, subsequence high) and key = (seed low, seed high); the first block
// returned by next4() is the Philox block of that counter.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long offset = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
