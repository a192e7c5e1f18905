// Host-only probe: prints rocRAND's Philox-4x32-10 output words for given
// (key, counter) so that the oracle's generator can be checked against an
// independent, published implementation.  rocRAND's engine with seed S,
// subsequence Q and offset 4c evaluates the generator at key (lo32 S, hi32 S)
// and counter (lo32 c, hi32 c, lo32 Q, hi32 Q).
// Input lines: "seed subsequence block"; output lines: four hex words.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long seed, subseq, block;
    while (std::scanf("%llu %llu %llu", &seed, &subseq, &block) == 3) {
        rocrand_device::philox4x32_10_engine eng(seed, subseq, 4ull * block);
        unsigned int w[4];
        for (int i = 0; i < 4; ++i) w[i] = eng.next();
        std::printf("%08x %08x %08x %08x\n", w[0], w[1], w[2], w[3]);
    }
    return 0;
}
