// Known-answer source for the oracle's Philox4x32-10: rocRAND's header-only
// philox4x32_10 engine (an independent implementation), run on the host.
// Reads lines "x y z w k0 k1" (counter words, key words) and prints the four
// output words of that block.  The engine's key is its seed; its counter
// words z, w are the subsequence and x, y are offset / 4.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned x, y, z, w, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &x, &y, &z, &w, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)z | ((unsigned long long)w << 32);
        unsigned long long off = 4ULL * ((unsigned long long)x | ((unsigned long long)y << 32));
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned a = e.next(), b = e.next(), c = e.next(), d = e.next();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
