// Independent Philox4x32-10 for pinning the oracle: rocRAND's host-callable
// engine.  Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin and prints the four
// output words.  engine(seed, subsequence, offset) keys with seed = k1:k0 and
// starts at counter (offset/4 split over c0,c1) + (subsequence over c2,c3).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        unsigned long long off = 4ULL * (((unsigned long long)c1 << 32) | c0);
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned r0 = e.next(), r1 = e.next(), r2 = e.next(), r3 = e.next();
        std::printf("%08x %08x %08x %08x\n", r0, r1, r2, r3);
    }
    return 0;
}
