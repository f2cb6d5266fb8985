// Host-side reference Philox4x32-10 blocks from rocRAND's engine (an independent,
// published implementation), used only to pin the oracle's own Philox.
// Reads "c0 c1 c2 c3 k0 k1" lines from stdin, prints "x0 x1 x2 x3".
// rocRAND's engine state is (counter, key) with key = seed, counter words 2..3 =
// subsequence and counter words 0..1 = offset / 4, so seeding the engine with
// those values and drawing four numbers yields the block of that counter.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        const unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        const unsigned long long offset = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        unsigned x0 = eng(), x1 = eng(), x2 = eng(), x3 = eng();
        std::printf("%u %u %u %u\n", x0, x1, x2, x3);
    }
    return 0;
}
