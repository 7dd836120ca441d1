// Reference Philox4x32-10 blocks from the rocRAND library implementation (host side), used only
// by the test-suite to pin the oracle's own Philox.  Reads lines "c0 c1 c2 c3 k0 k1" (uint32,
// decimal) from stdin and prints the four output words of the block at that counter and key.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned int c[4], k[2];
    while (std::scanf("%u %u %u %u %u %u", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        unsigned long long seed = (unsigned long long)k[0] | ((unsigned long long)k[1] << 32);
        unsigned long long subsequence = (unsigned long long)c[2] | ((unsigned long long)c[3] << 32);
        unsigned long long offset = 4ull * ((unsigned long long)c[0] | ((unsigned long long)c[1] << 32));
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
