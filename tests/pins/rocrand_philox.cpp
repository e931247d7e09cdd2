// Host-side Philox4x32-10 words from rocRAND, used only to pin the oracle's generator.
// Reads "key0 key1 c0 c1 c2 c3" lines (decimal) and prints the four output words.
// rocRAND keys the engine with the 64-bit seed, puts the subsequence in counter words 2-3 and
// advances counter words 0-1 by offset/4.
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

int main()
{
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        rocrand_state_philox4x32_10 st;
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long subsequence = c2 | (c3 << 32);
        unsigned long long offset = 4ULL * (c0 | (c1 << 32));
        rocrand_init(seed, subsequence, offset, &st);
        uint4 v = rocrand4(&st);
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
