// Prints the four 32-bit words that rocRAND's Philox4x32-10 engine returns for each
// "seed subsequence offset" line read from stdin.  rocRAND is an independent, separately
// maintained implementation; the tests run this probe (host side only, no GPU) to check
// the oracle's Philox block and its counter layout (subsequence = trajectory, offset =
// 4 * step).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long seed, sub, off;
    while (std::scanf("%llx %llx %llx", &seed, &sub, &off) == 3) {
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        uint4 v = e.next4();
        std::printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
