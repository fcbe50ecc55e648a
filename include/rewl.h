/*
 * rewl.h -- C ABI of the MI355X (gfx950) replica-exchange Wang-Landau library.
 *
 * Method: Vogel, Li, Wuest & Landau, "A generic, hierarchical framework for
 * massively parallel Wang-Landau sampling", arXiv:1305.5615.  The energy range
 * is split into n_windows overlapping windows (overlap o), each sampled by
 * walkers_per_window independent Wang-Landau walkers with their own ln g(E) and
 * H(E) (the parallel-scheme paragraph after Fig. 1); moves are accepted with
 * min[1, g(E_old)/g(E_new)] and ln g(E) += ln f, H(E) += 1 at the current
 * energy after every move (the standard-WL paragraph); walkers of adjacent
 * windows exchange configurations with the probability of Eq. (1); when all
 * walkers of a window are flat their ln g are averaged and ln f is halved;
 * the run ends when every window's ln f is below lnf_final, and the window
 * pieces are joined where d ln g / dE agree best.
 *
 * Models on an L x L torus: REWL_ISING E = -sum s_i s_j (step 4),
 * REWL_POTTS E = -sum delta(s_i, s_j) (q states, step 1), REWL_EA
 * E = -sum J_ij s_i s_j with J = +-1 (step 4).
 *
 * Conventions for every function:
 *  - return value: REWL_OK (0), REWL_NOT_CONVERGED (1, informational) or a
 *    negative error code; rewl_last_error() then describes it (thread-local,
 *    valid until the next call on the same thread);
 *  - host pointers are read or written only during the call and stay owned by
 *    the caller; the library copies what it keeps;
 *  - a handle is used by one host thread at a time: a call that would advance
 *    or read a run, batch or server while another thread is inside such a call
 *    on it returns REWL_EBUSY (step, run, done, get_lng, save, server tick);
 *  - all device work runs on the stream given at creation (NULL: the null
 *    stream); functions that return host data synchronise that stream.
 * Every step of the method runs in this library's HIP kernels (sweep, flatness
 * and merge, exchange, start-up) except the final stitching, which is a host
 * loop over at most a few thousand bins.
 */
#ifndef REWL_H
#define REWL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    REWL_OK = 0,
    REWL_NOT_CONVERGED = 1,
    REWL_EINVAL = -1,   /* argument out of range or inconsistent */
    REWL_ENOMEM = -2,   /* host or device allocation failed / buffer too small */
    REWL_EDEVICE = -3,  /* a HIP call failed */
    REWL_EINIT = -4,    /* a walker could not be brought into its window */
    REWL_ECORRUPT = -5, /* state failed a consistency check */
    REWL_EBUSY = -6,    /* handle in use by another host thread, or no capacity */
    REWL_ESTITCH = -7   /* a window overlap holds no commonly visited bin */
};

/* Models (the paper's tests: 2D Ising, 2D q-state Potts, +-J spin glasses).
 * REWL_ISING, REWL_POTTS, REWL_EA live on the L x L torus (N = L^2 sites,
 * 2N bonds); REWL_EA3 is the +-J glass on the L x L x L torus (N = L^3
 * sites, 3N bonds, the paper's 12^3 ground-state test). */
enum { REWL_ISING = 0, REWL_POTTS = 1, REWL_EA = 2, REWL_EA3 = 3 };

/* ln f schedules.  REWL_HALVING: ln f halves at every merge (f -> sqrt f).
 * REWL_ONE_OVER_T: halving until a halving would take ln f below W/t (W bins
 * of the window, t attempts per walker so far); from then on ln f = W/t renewed
 * after every attempt, the window's walkers are averaged every round without a
 * flatness test, and the window is done once W/t < lnf_final (the 1/t rule of
 * Belardinelli & Pereyra, one of the update rules the paper names as usable). */
enum { REWL_HALVING = 0, REWL_ONE_OVER_T = 1 };

/* Parameters of one run.
 *  couplings: REWL_EA: 2*L*L values +-1, [2i] = J(i, right neighbour),
 *             [2i+1] = J(i, lower neighbour), site i = row*L + column;
 *             REWL_EA3: 3*L^3 values, [3i + a] = J(i, next site along axis a),
 *             a = x, y, z, site i = (z L + y) L + x; else NULL.
 *  e_min, e_max: inclusive energy range; clipped to the model's range
 *             ([-2N, 2N], Potts [-2N, 0], 3D [-3N, 3N]) and, for the glasses,
 *             aligned inwards onto the energy class -B + 2 n_neg (mod 4) of the
 *             couplings (B bonds, n_neg of them -1).
 *  n_windows >= 1, 0 < overlap < 1, walkers_per_window in [1, 64],
 *  0 < flatness <= 1, lnf_init > 0, lnf_final > 0,
 *  attempts_per_round >= 1 (attempts per walker between exchange steps),
 *  seed: Philox4x32-10 key, schedule: REWL_HALVING or REWL_ONE_OVER_T.
 *  Windows narrower than 2 bins, overlaps below 2 bins, 3 > L or L > 256
 *  (REWL_EA3: 2 > L or L > 32), q outside [2, 127] (Potts) are REWL_EINVAL. */
typedef struct rewl_params {
    int model;
    int L;
    int q;
    const int8_t *couplings;
    int64_t e_min;
    int64_t e_max;
    int n_windows;
    double overlap;
    int walkers_per_window;
    double flatness;
    double lnf_init;
    double lnf_final;
    int64_t attempts_per_round;
    uint64_t seed;
    int schedule;  /* REWL_HALVING or REWL_ONE_OVER_T */
    /* Explicit windows (both or neither; NULL: the equal partition): n_windows
     * first and last bins each, bin b = (E - e_min) / step after the range is
     * aligned; they must start at bin 0, end at the last bin, have increasing
     * starts and ends, >= 2 bins each and >= 2 bins shared by neighbours.
     * Copied by the calls that take a rewl_params. */
    const int64_t *window_lo;
    const int64_t *window_hi;
} rewl_params;

typedef struct rewl_ctx rewl_ctx; /* opaque, owned by the library */

/* Device bytes a run needs (device_bytes) and the LDS bytes one walker's
 * sweep work-group uses (lds_bytes).  REWL_EINVAL if the parameters are
 * invalid or one walker's window does not fit the 160 KiB LDS of a CU. */
int rewl_footprint(const rewl_params *p, size_t *device_bytes, size_t *lds_bytes);

/* Create a run: validate, partition the energy range, allocate device state,
 * then, on the device, draw every walker's random start configuration and walk
 * it into its window (the start-up step; Ising and Potts walkers that cannot
 * get there by single-site moves restart from the ordered state).
 *  device_buffer: NULL to let the library allocate (hipMalloc) and free its
 *     own memory, or caller-owned device memory of at least rewl_footprint()
 *     bytes, 256-byte aligned, which the library never frees;
 *  hip_stream: the hipStream_t all work of this run is queued on (NULL: null
 *     stream).
 * On error *out is NULL.  REWL_EINIT if the start-up step fails. */
int rewl_create_ex(rewl_ctx **out, const rewl_params *p, void *device_buffer,
                   size_t buffer_bytes, void *hip_stream);

/* Positional form with lnf_init = 1, 10^4 attempts per round, library-owned
 * memory and the null stream. */
int rewl_create(rewl_ctx **out, int model, int L, int q, const int8_t *couplings,
                int64_t e_min, int64_t e_max, int n_windows, double overlap,
                int walkers_per_window, double flatness, double lnf_final, uint64_t seed);

/* Run rounds until every window is done or max_rounds rounds (< 0: no limit)
 * have been issued.  A round is: attempts_per_round sweep attempts by every
 * walker of every unfinished window, the flatness check, the merges, then one
 * exchange step between windows (k, k+1), k = round mod 2.  Returns REWL_OK
 * when converged, REWL_NOT_CONVERGED when max_rounds ran out first.
 * *rounds_done (may be NULL) receives the number of the round in which the
 * last window finished plus one, or the rounds issued so far. */
int rewl_run(rewl_ctx *h, int64_t max_rounds, int64_t *rounds_done);

/* Queue exactly `rounds` rounds (no convergence polling, asynchronous). */
int rewl_step(rewl_ctx *h, int64_t rounds);

/* Stitched, normalised ln g over all n_bins = (e_max - e_min)/e_step + 1
 * energy bins; bins no walker visited hold -INFINITY.  Normalisation: Ising
 * ln g(-2N) = ln 2, Potts ln g(-2N) = ln q when the requested range started at
 * -2N; EA and EA3: ln sum g = N ln 2 when it was the whole [-2N, 2N]
 * (resp. [-3N, 3N]); otherwise the lowest visited bin is 0.  cap: entries available in out.  Returns
 * REWL_NOT_CONVERGED (with the data) when some window is not done yet. */
int rewl_get_lng(rewl_ctx *h, double *out, int64_t cap, int64_t *n_bins, int64_t *e_min,
                 int64_t *e_step);

/* Raw state of walker w = window * walkers_per_window + slot: spins (n_sites
 * int8, L*L, or L^3 for EA3; Potts states 0..q-1), energy, attempts made, flat flag, and the window-local
 * ln g / H / visited arrays (hi - lo + 1 entries of the walker's window).  Any
 * output pointer may be NULL. */
int rewl_get_walker(rewl_ctx *h, int w, int8_t *spins, int64_t *E, uint64_t *t, int *flat,
                    double *lng, uint32_t *H, uint8_t *visited);

/* Window k: bin range [lo, hi], current ln f, done flag, round it finished in
 * (-1 before). */
int rewl_get_window(rewl_ctx *h, int k, int64_t *lo, int64_t *hi, double *lnf, int *done,
                    int64_t *finish_round);

/* Geometry and counters: bins, energy origin and step, windows, walkers per
 * window, sites, rounds issued, total sweep attempts made, accepted moves,
 * exchange proposals and acceptances. */
int rewl_get_info(rewl_ctx *h, int64_t *n_bins, int64_t *e_min, int64_t *e_step,
                  int *n_windows, int *walkers_per_window, int *n_sites, int64_t *rounds,
                  uint64_t *attempts, uint64_t *accepts, uint64_t *ex_prop, uint64_t *ex_acc);

/* Round in which each window first merged (halved ln f), -1 where it has not
 * yet: out[k] for k < min(cap, n_windows).  With a run on the equal partition
 * stepped until every entry is >= 0, these are the first-iteration times that
 * rewl_partition_balanced takes (as first + 1 rounds). */
int rewl_get_first_merge(rewl_ctx *h, int64_t *out, int cap);

/* Run-time balanced windows (the paper's Fig. 1b and its scaling discussion:
 * windows chosen so that all of them complete the first WL iteration after
 * the same number of sweeps, estimated from a pre-run on the equal
 * partition).  Host-only; all arrays are caller-owned host memory.
 *   n_bins, n_windows, overlap: the new partition (n_windows >= 1, 0 < o < 1);
 *   pre_lo/pre_hi (pre_windows entries): the pre-run's windows, a valid
 *   partition of the same bins; first_rounds: rounds each pre-run window took
 *   for its first iteration (>= 1).
 * Each bin gets the first-iteration time density t(b) = mean of
 * first_rounds[k] / (pre_hi[k] - pre_lo[k] + 1) over the pre-run windows that
 * contain it; bins are points on the axis F(0) = 0,
 * F(b+1) = F(b) + (t(b) + t(b+1)) / 2, and the result is the equal partition
 * of that axis: x_k = k (1-o) w, w = F(last) / (1 + (n_windows-1)(1-o)), lo_k =
 * last bin with F <= x_k, hi_k = first bin with F >= x_k + w (the last bin for
 * k = n_windows - 1).  A uniform density gives the equal partition exactly.
 * Returns REWL_EINVAL for bad arguments or when the result is not a valid
 * partition (windows narrower than 2 bins or overlapping by fewer). */
int rewl_partition_balanced(int64_t n_bins, int n_windows, double overlap, int pre_windows,
                            const int64_t *pre_lo, const int64_t *pre_hi,
                            const int64_t *first_rounds, int64_t *lo, int64_t *hi);

/* Jackknife (leave-one-out) mean and error of ln g per bin over independent
 * runs, the paper's resampling estimate of statistical errors.  Host-only.
 * lng: runs x n_bins doubles, row r = run r's stitched, normalised ln g
 * (caller-owned); mean, err: n_bins each (caller-owned).  For bin b with
 * values x_r: mean = sum_r x_r / R; theta_i = (sum_r x_r - x_i) / (R-1);
 * err = sqrt((R-1)/R * sum_i (theta_i - mean_i theta_i)^2).  A bin that any
 * run left unvisited (-inf) gets mean -inf and err NaN.  runs >= 2. */
int rewl_jackknife(const double *lng, int runs, int64_t n_bins, double *mean, double *err);

/* Checkpoint and resume.  rewl_save waits for the run's pending work, then
 * writes its parameters, couplings, windows and complete device state to
 * `path` (through path.tmp, renamed when complete; the caller owns the path).
 * rewl_load recreates the run from such a file -- device memory as in
 * rewl_create_ex -- so that stepping it continues exactly as the saved run
 * would have (same rounds, same results, bit for bit).  REWL_ECORRUPT: not a
 * checkpoint, truncated, checksum (FNV-1a 64 over the file) mismatch, or a
 * saved state that does not fit the saved parameters (windows, every walker's
 * energy inside its window, spins that are states of the model, +-1
 * couplings), checked on the host before anything reaches the GPU;
 * REWL_EINVAL: the file cannot be opened or written, or the parameters it
 * holds are ones rewl_create_ex refuses.  Works for a run of a
 * batch too (it is saved alone and loads as a run of its own). */
int rewl_save(rewl_ctx *h, const char *path);
int rewl_load(rewl_ctx **out, const char *path, void *device_buffer, size_t buffer_bytes,
              void *hip_stream);

/* Timing of the sweep kernel: with on != 0, every later round records a HIP
 * event right before and right after its sweep launch on the run's stream;
 * rewl_get_timing synchronises the stream and returns the summed elapsed time
 * of those launches (milliseconds) and their number since the last
 * rewl_set_timing.  Costs two event records per round; off by default. */
int rewl_set_timing(rewl_ctx *h, int on);
int rewl_get_timing(rewl_ctx *h, double *sweep_ms, int64_t *sweep_launches);

/* Release a run made by rewl_create_ex / rewl_create (and its device memory if
 * the library allocated it).  Runs obtained from a batch are released with the
 * batch; rewl_destroy ignores them. */
void rewl_destroy(rewl_ctx *h);

/* ---------------------------------------------------------------- batches
 * Many independent runs advanced together: every round is one launch of each
 * kernel over all runs (sweep groups of walkers_per_wave walkers of one run per
 * wave, windows, window pairs) plus a round-counter update, on one stream.
 * Each run keeps its own round counter, seed and state, so its results are
 * bit-identical to the same run made alone with rewl_create_ex.  Run i's state
 * is read with the rewl_get_* functions on the handle rewl_batch_get_run
 * returns (owned by the batch).
 *  walkers_per_wave: 1, 2, 4 or 8 (0: 1); more walkers per wave share each
 *    wave's instructions, fewer give each walker a whole wave (lower latency).
 *    (The sweep's instantiation also depends on whether a launch has more
 *    waves than the device has compute units; results never do.)
 *  REWL_EINVAL if the walkers of one wave do not fit the LDS of a CU. */
typedef struct rewl_batch rewl_batch;
int rewl_batch_create(rewl_batch **out, const rewl_params *runs, int n_runs,
                      int walkers_per_wave, void *hip_stream);
int rewl_batch_get_run(rewl_batch *b, int i, rewl_ctx **run);
int rewl_batch_set_walkers_per_wave(rewl_batch *b, int walkers_per_wave);
/* How rounds are launched (results never depend on it):
 *  REWL_FORM_ROUNDS (default): every round is one launch of each kernel over
 *    all runs (sweep, flatness/merge, exchange, round counters); the walkers'
 *    state goes through device memory between them;
 *  REWL_FORM_PERSISTENT: one launch per call of rewl_batch_step (cut into
 *    launches of at most 1024 rounds) in which one work-group holds one run,
 *    loads its walkers' state into LDS once and loops the rounds -- sweep,
 *    flatness, merges and the exchange step (Eq. (1)) as work-group steps
 *    between barriers -- then writes it back; the h x m hierarchy of the
 *    parallel-scheme paragraph held by one CU.  A work-group finishes early
 *    once every window of its run is done.  Requires every run to fit one
 *    work-group: at most 64 walkers, at most 8 waves of walkers_per_wave
 *    walkers, and their LDS within one CU (160 KiB); REWL_EINVAL otherwise,
 *    and the form is left unchanged.  Graphs are not used in this form. */
enum { REWL_FORM_ROUNDS = 0, REWL_FORM_PERSISTENT = 1 };
int rewl_batch_set_form(rewl_batch *b, int form);
/* rounds_per_graph > 0: rounds are issued as replays of a captured HIP graph of
 * that many rounds (remaining rounds as direct launches); 0: direct launches.
 * Graphs are not used while timing is on. */
int rewl_batch_set_graph(rewl_batch *b, int rounds_per_graph);
int rewl_batch_step(rewl_batch *b, int64_t rounds);
/* Rounds until every run is done or max_rounds (< 0: no limit) issued;
 * *rounds_issued: rounds issued by the batch so far.  REWL_NOT_CONVERGED if
 * some run is still running. */
int rewl_batch_run(rewl_batch *b, int64_t max_rounds, int64_t *rounds_issued);
/* flags[i] = 1 when run i is done (cap >= number of runs). */
int rewl_batch_done(rewl_batch *b, int *flags, int cap);
int rewl_batch_set_timing(rewl_batch *b, int on);
int rewl_batch_get_timing(rewl_batch *b, double *sweep_ms, int64_t *sweep_launches);
void rewl_batch_destroy(rewl_batch *b);

/* ------------------------------------------------------------------ server
 * Continuous batching of arriving runs.  Submitted runs wait in arrival order
 * and are admitted at round boundaries while their device state fits the
 * budget (and, lowering walkers_per_wave if needed, their LDS footprint fits a
 * CU); admitted runs start their own round count at 0 and are advanced together
 * with the runs already on the device; a finished run is stitched on the host,
 * its device state freed, and its result kept until released.  A run's result
 * is bit-identical to the same run made alone.
 *  rewl_server_tick: retire finished runs, admit waiting ones, then advance all
 *    running runs by rounds_per_tick rounds (synchronous in its retire step).
 *  rewl_server_next_done: id of the next finished run (REWL_NOT_CONVERGED when
 *    none) and the rounds it ran.
 *  rewl_server_result: its stitched, normalised ln g (as rewl_get_lng).  A
 *    request whose start-up fails (REWL_EINIT: a walker cannot reach its
 *    window) is taken off the queue at admission and finishes at once with 0
 *    rounds; its result returns that code and the other runs go on.
 *  REWL_EBUSY from submit: the run alone exceeds the device budget. */
typedef struct rewl_server rewl_server;
int rewl_server_create(rewl_server **out, size_t device_budget_bytes, int walkers_per_wave,
                       int rounds_per_tick, void *hip_stream);
int rewl_server_submit(rewl_server *s, const rewl_params *p, int64_t *id);
int rewl_server_tick(rewl_server *s, int *n_running, int *n_queued);
int rewl_server_next_done(rewl_server *s, int64_t *id, int64_t *rounds);
int rewl_server_result(rewl_server *s, int64_t id, double *out, int64_t cap, int64_t *n_bins,
                       int64_t *e_min, int64_t *e_step);
int rewl_server_release(rewl_server *s, int64_t id);
void rewl_server_destroy(rewl_server *s);

/* ------------------------------------------------- allocation-free variant
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the run that
 * rewl_create_ex followed by rewl_step(rounds) would make, in one call that
 * allocates nothing -- no hipMalloc, hipFree or other allocating routine, and
 * no host heap either.  The caller passes the outputs, device arrays it owns:
 *   E      walkers int32: energy of walker w = window * walkers_per_window + slot;
 *   spins  walkers x spins_stride int8: walker w's configuration at
 *          spins[w * spins_stride + site] (sites as in rewl_get_walker),
 *          spins_stride >= n_sites and a multiple of 4;
 *   lng, H walkers x bins_stride (double, uint32): walker w's window-local
 *          ln g and histogram at [w * bins_stride + b], b = 0 .. window bins - 1,
 *          bins_stride >= the widest window's bins (zeroed by the call
 *          first, so unvisited bins hold 0).
 * After the call's work on hip_stream has completed they hold exactly what
 * rewl_get_walker reports for the same run made by rewl_create_ex and stepped
 * `rounds` rounds.  Everything else the run needs (walker and window
 * bookkeeping, couplings in kernel layout, launch tables) lives in one static
 * device array of the library, 128 KiB on each device it runs on, held until
 * the process ends (about 36 bytes per walker, 80 per window, 6 per site of a
 * 2D glass and 11 of a 3D one); runs needing more (some 3000 walkers or more)
 * and runs of more than 64 windows are REWL_EINVAL.
 * The call waits for the start-up (REWL_EINIT as in rewl_create_ex), then
 * queues the rounds and returns; the caller synchronises the stream before
 * reading the outputs.  Every call on a device shares that device's array and
 * overwrites it: calls that overlap on one device (other threads, or other
 * streams not ordered after this one) race and give undefined results. */
int rewl_run_noalloc(const rewl_params *p, int64_t rounds, int32_t *E, int8_t *spins,
                     int64_t spins_stride, double *lng, uint32_t *H, int64_t bins_stride,
                     void *hip_stream);

const char *rewl_last_error(void);

/* Diagnostics: evaluate the device's Philox4x32-10 block for n counters
 * (ctr: 4n words, key: 2 words, out: 4n words) and the device's ln u for n
 * word pairs (words: 2n, [2i] = high, [2i+1] = low word; out: n doubles).
 * Host pointers; synchronous on the null stream. */
int rewl_selftest_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int n);
int rewl_selftest_ln_u(const uint32_t *words, double *out, int n);

#ifdef __cplusplus
}
#endif
#endif
