// Prints Philox4x32-10 blocks computed by rocRAND's engine (an independent
// implementation shipped with ROCm) for counters read from stdin, so that a
// test can compare them with the oracle's generator.  Host-only build.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned long long seed;
    unsigned c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        // rocRAND: key = seed; subsequence adds to counter words (2, 3);
        // offset / 4 adds to counter words (0, 1).
        rocrand_device::philox4x32_10_engine e(
            seed, ((unsigned long long)c3 << 32) | c2,
            4ull * (((unsigned long long)c1 << 32) | c0));
        unsigned w0 = e(), w1 = e(), w2 = e(), w3 = e();
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
