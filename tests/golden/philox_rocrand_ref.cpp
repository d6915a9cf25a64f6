// Prints Philox4x32-10 outputs from rocRAND's host-callable engine, used by the test-suite as a
// library reference for the oracle's independently written generator.  For key (seed lo, seed hi)
// and counter (c0, c1, c2, c3): rocRAND's seed(seed, subsequence, offset) places offset/4 in
// (c0, c1) and subsequence in (c2, c3), and the first next4() returns the block for that counter.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv)
{
    // args: seed c0 c1 c2 c3 (decimal); offset = 4 * (c0 | c1 << 32) must not overflow.
    if (argc != 6) return 2;
    unsigned long long seed = strtoull(argv[1], 0, 10);
    unsigned long long c0 = strtoull(argv[2], 0, 10), c1 = strtoull(argv[3], 0, 10);
    unsigned long long c2 = strtoull(argv[4], 0, 10), c3 = strtoull(argv[5], 0, 10);
    unsigned long long offset = 4ull * (c0 | (c1 << 32));
    unsigned long long subseq = c2 | (c3 << 32);
    rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
    uint4 v = eng.next4();
    printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    return 0;
}
