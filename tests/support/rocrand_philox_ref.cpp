// Host-side reference stream from rocRAND's philox4x32_10 engine, used to pin
// the oracle's Philox4x32-10.  Reads lines "c0 c1 c2 c3 seed_lo seed_hi" on
// stdin and prints the four output words for that counter and key.
// rocRAND maps key = (seed lo, seed hi); subsequence s advances counter words
// (2,3) by s; offset k advances the 128-bit counter by k/4.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subsequence = ((unsigned long long)c3 << 32) | c2;
        unsigned long long offset = 4ull * (((unsigned long long)c1 << 32) | c0);
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
