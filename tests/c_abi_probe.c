/* A plain C11 program against include/rewl.h and librewl.so: the host-only
 * entry points, called without a GPU.  Prints one line per check; exits 0 when
 * every check holds. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "rewl.h"

static int fails = 0;
#define CHECK(c)                                                 \
    do {                                                         \
        if (!(c)) {                                              \
            printf("FAIL %s (line %d): %s\n", #c, __LINE__,      \
                   rewl_last_error());                           \
            ++fails;                                             \
        }                                                        \
    } while (0)

int main(void)
{
    /* footprint of the 32x32 Ising workload and a refused parameter set */
    rewl_params p;
    memset(&p, 0, sizeof p);
    p.model = REWL_ISING;
    p.L = 32;
    p.q = 2;
    p.e_min = -2048;
    p.e_max = 2048;
    p.n_windows = 16;
    p.overlap = 0.75;
    p.walkers_per_window = 4;
    p.flatness = 0.8;
    p.lnf_init = 1.0;
    p.lnf_final = 1e-8;
    p.attempts_per_round = 10000;
    p.seed = 1;
    p.schedule = REWL_HALVING;
    size_t dev = 0, lds = 0;
    CHECK(rewl_footprint(&p, &dev, &lds) == REWL_OK);
    CHECK(dev > 0 && lds > 0 && lds <= 160 * 1024);
    printf("footprint: %zu device bytes, %zu LDS bytes\n", dev, lds);
    p.overlap = 1.0;
    CHECK(rewl_footprint(&p, &dev, &lds) == REWL_EINVAL);
    p.overlap = 0.75;

    /* balanced partition of a uniform density = the equal partition */
    int64_t pre_lo[4] = {0, 9, 18, 27}, pre_hi[4] = {37, 46, 55, 64};
    int64_t first[4] = {38, 38, 38, 38};
    int64_t lo[4], hi[4];
    CHECK(rewl_partition_balanced(65, 4, 0.75, 4, pre_lo, pre_hi, first, lo, hi) == REWL_OK);
    for (int k = 0; k < 4; ++k) CHECK(lo[k] == pre_lo[k] && hi[k] == pre_hi[k]);

    /* jackknife of two runs: mean, and |a - b| / 2 */
    double lng[2 * 3] = {1.0, 2.0, -INFINITY, 3.0, 2.0, 5.0};
    double mean[3], err[3];
    CHECK(rewl_jackknife(lng, 2, 3, mean, err) == REWL_OK);
    CHECK(mean[0] == 2.0 && fabs(err[0] - 1.0) < 1e-15);
    CHECK(mean[1] == 2.0 && err[1] == 0.0);
    CHECK(isinf(mean[2]) && isnan(err[2]));
    printf("%s\n", fails ? "c-abi probe: FAILED" : "c-abi probe: ok");
    return fails ? 1 : 0;
}
