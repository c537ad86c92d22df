// Prints rocRAND's Philox4x32-10 block for counters and keys read from stdin
// (one "c0 c1 c2 c3 k0 k1" line each, decimal).  Used only by the oracle's
// pin tests as an independent library implementation of the generator.
#include <cstdio>
#include <rocrand/rocrand_kernel.h>

int main()
{
    unsigned int c[4], k[2];
    while (std::scanf("%u %u %u %u %u %u", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        unsigned long long seed = (unsigned long long)k[0] | ((unsigned long long)k[1] << 32);
        unsigned long long subseq = (unsigned long long)c[2] | ((unsigned long long)c[3] << 32);
        unsigned long long offset = 4ull * ((unsigned long long)c[0] | ((unsigned long long)c[1] << 32));
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subseq, offset, &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
