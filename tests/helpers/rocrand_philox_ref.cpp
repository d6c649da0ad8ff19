// Independent Philox4x32-10 reference for the oracle's own implementation:
// rocRAND's host-callable engine.  Reads lines "seed subsequence quad_offset"
// on stdin and prints the four 32-bit words the engine returns for that
// position.  rocRAND places the seed in the key, the subsequence in counter
// words (z, w) and the quad offset in counter words (x, y).
#include <cstdio>
#include <rocrand/rocrand_kernel.h>

int main()
{
    unsigned long long seed, subseq, quad;
    while (std::scanf("%llu %llu %llu", &seed, &subseq, &quad) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subseq, 4ull * quad, &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
