/*
 * rewl_oracle.h -- plain CPU oracle for replica-exchange Wang-Landau sampling
 * (Vogel, Li, Wuest & Landau, "A generic, hierarchical framework for massively
 * parallel Wang-Landau sampling", arXiv:1305.5615).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the GPU library; the two meet only
 * in the definitions written out in rewl_oracle.c.
 *
 * Conventions: every function returns 0 on success and a negative code on
 * failure (same numbering as the product library so tests can compare codes):
 *   -1 invalid argument, -2 out of memory, -4 initial descent failed,
 *   -7 stitching impossible (a window overlap holds no commonly visited bin).
 */
#ifndef REWL_ORACLE_H
#define REWL_ORACLE_H
#include <stdint.h>

#define ORC_ISING 0
#define ORC_POTTS 1
#define ORC_EA 2
#define ORC_EA3 3   /* +-J glass on the L x L x L torus */

typedef struct orc_run orc_run;

/* Create a run.  couplings: EA only, 2*L*L int8 values +-1, interleaved per
 * site i as [2i] = J(i, right neighbour), [2i+1] = J(i, lower neighbour);
 * EA3: 3*L^3 values, [3i + a] = J(i, next site along axis a = x, y, z), sites
 * i = (z L + y) L + x, 2 <= L <= 32 (L >= 3 for the 2D models); copied.  e_min/e_max are inclusive; for EA they are aligned inwards onto the
 * energy class of the couplings.  lnf_init is the first ln f; S the number of
 * attempts per walker per round; n_threads the OpenMP threads used by the
 * sweep (0 = runtime default); schedule 0 halves ln f at every merge, 1 halves
 * it until it would drop below W/t and then follows W/t (the 1/t rule).
 * win_lo/win_hi (both or neither): explicit windows in bins, replacing the
 * equal partition; they must run from bin 0 to the last bin with increasing
 * starts and ends, >= 2 bins each and >= 2 shared by neighbours. */
int orc_create(orc_run **out, int model, int L, int q, const int8_t *couplings,
               int64_t e_min, int64_t e_max, int n_windows, double overlap,
               int walkers_per_window, double flatness, double lnf_init,
               double lnf_final, int64_t S, uint64_t seed, int n_threads, int schedule,
               const int64_t *win_lo, const int64_t *win_hi);
void orc_destroy(orc_run *run);

/* Advance exactly `rounds` rounds (rounds of a finished run change nothing). */
int orc_step(orc_run *run, int64_t rounds);
/* Rounds until every window is done or max_rounds (<0: unbounded) elapsed.
 * Returns 0 when converged, 1 when max_rounds ran out first. */
int orc_run_to(orc_run *run, int64_t max_rounds);

/* Sizes and geometry. */
void orc_info(const orc_run *run, int64_t *n_bins, int64_t *e_min, int64_t *e_step,
              int *n_windows, int *walkers_per_window, int *n_sites, int64_t *round,
              int *all_done);
void orc_window(const orc_run *run, int k, int64_t *lo, int64_t *hi, double *lnf,
                int *done, int64_t *finish_round);
/* Walker state: spins (n_sites, int8; Potts states 0..q-1), energy, attempt
 * counter, flat flag, and window-local ln g / H / visited (hi-lo+1 entries). */
int orc_walker(const orc_run *run, int w, int8_t *spins, int64_t *E, uint64_t *t,
               int *flat, double *lng, uint32_t *H, uint8_t *visited);
/* Overwrite a walker's window-local ln g (visited set where value > 0). */
int orc_set_lng(orc_run *run, int w, const double *lng);
/* Stitched, normalised ln g over all bins; unvisited bins = -inf. */
int orc_get_lng(orc_run *run, double *out, int64_t cap);
/* Round of each window's first merge (-1 where none happened yet). */
void orc_first_merge(const orc_run *run, int64_t *out);
/* Counters: accepted sweep moves, exchange proposals and acceptances. */
void orc_stats(const orc_run *run, uint64_t *attempts, uint64_t *accepts,
               uint64_t *ex_prop, uint64_t *ex_acc);

/* Building blocks exported for the pin tests. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_ln_u(double u);
double orc_uniform(uint32_t hi, uint32_t lo);
int64_t orc_energy(int model, int L, int q, const int8_t *spins, const int8_t *couplings);
int orc_sites(int model, int L);
int orc_partition(int64_t n_bins, int n_windows, double overlap, int64_t *lo, int64_t *hi);
/* Run-time balanced partition from a pre-run's windows and first-iteration
 * rounds T (see rewl_oracle.c). */
int orc_partition_balanced(int64_t B, int h, double o, int pre_h, const int64_t *pre_lo,
                           const int64_t *pre_hi, const int64_t *T, int64_t *lo, int64_t *hi);
int orc_stitch(int n_windows, const int64_t *lo, const int64_t *hi, const double *pieces,
               int64_t stride, const uint8_t *visited, int64_t n_bins, double *out,
               int64_t *joins);

#endif
