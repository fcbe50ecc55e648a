// Host-only probe used by tests/test_oracle_pins.py: prints rocRAND's
// Philox4x32-10 words for (seed, subsequence, offset) triples read from stdin.
// rocRAND's engine keeps the counter as (offset/4 low, high, subsequence low,
// high) and the key as the seed, so four draws after rocrand_init(seed,
// subsequence, 4 t) are the block for counter (t, subsequence) under key seed.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, off, &st);
        unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
