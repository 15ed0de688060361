// Prints Philox4x32-10 blocks from rocRAND's host-callable engine, used as a
// black-box cross-check of the oracle's generator.  Engine(seed, subsequence,
// offset) keys Philox with the 64-bit seed and starts at counter
// (offset/4 as a 64-bit value, subsequence as a 64-bit value).
// Usage: rocrand_philox_dump seed subsequence block  -> four hex words
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char **argv)
{
    if (argc != 4) return 2;
    unsigned long long seed = std::strtoull(argv[1], nullptr, 0);
    unsigned long long sub = std::strtoull(argv[2], nullptr, 0);
    unsigned long long block = std::strtoull(argv[3], nullptr, 0);
    rocrand_device::philox4x32_10_engine e(seed, sub, block * 4ull);
    for (int i = 0; i < 4; ++i) std::printf("%08x ", e());
    std::printf("\n");
    return 0;
}
