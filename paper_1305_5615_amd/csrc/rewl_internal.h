// rewl_internal.h -- host/device shared layout of the runs' device state.
//
// Every run lives in one device slab carved by rewl_api.cpp:
//   spins   nw x Npad int8   (Ising/EA +-1, Potts 0..q-1)
//   E       nw int32         (current energy)
//   t       nw uint64        (sweep attempts made = stream-0 Philox counter)
//   flat    nw int32         (latched flatness flag of the current iteration)
//   lng     nw x Wmax f64    (window-local ln g; visited <=> lng > 0)
//   H       nw x Wmax uint32 (window-local histogram of the current iteration)
//   n_acc   nw uint64        (accepted sweep moves)
//   lnf     h f64, done h int32, phase h int32 (1/t rule active), finish h
//           int64, first h int64 (round of the first merge), lo/hi h int32
//           (bins)
//   ex_prop, ex_acc  h uint64 (exchange proposals / acceptances of pair (k,k+1))
//   J4      N uint32 (EA: couplings to right, left, down, up neighbour, one
//           int8 each, packed little-endian) or 2N uint32 (EA3: the same, then
//           +z, -z)
//   round   1 int64          (rounds completed; read by the merge and exchange
//                             kernels, advanced by advance_kernel)
//   status  1 int32          (start-up failure flag)
// Kernels see a run through its RunDesc.  A launch covers a batch of runs
// through three work lists: sweep groups (P walkers of one run per wave),
// windows (flatness/merge) and window pairs (exchange).
#pragma once
#include <stddef.h>
#include <stdint.h>

struct RunDesc {
    int model, L, N, q, h, m, nw;
    int Npad, Wmax;
    int e_min, step;
    uint32_t l_magic;  // ceil(2^32 / L): row = mulhi(site, l_magic) for site < L*L
    uint32_t l2_magic; // ceil(2^32 / L^2) (3D: layer = mulhi(site, l2_magic))
    uint32_t key0, key1;
    long long S;
    int schedule;      // 0 halving, 1 halving then 1/t
    double flat_p, lnf_final;
    int8_t *spins;
    int *E;
    unsigned long long *t;
    int *flat;
    double *lng;
    uint32_t *H;
    unsigned long long *n_acc;
    double *lnf;
    int *done;
    int *phase;        // per window: 1 once it follows the 1/t rule
    long long *finish;
    long long *first;  // per window: round of its first merge, -1 before
    int *lo, *hi;
    unsigned long long *ex_prop, *ex_acc;
    uint32_t *J4;      // couplings per site: EA one word (+x, -x, +y, -y), EA3
                       // two words (+x, -x, +y, -y | +z, -z), one int8 each
    long long *round;
    int *status;
};

// One wave of the sweep: walkers w0 .. w0 + count - 1 of run `run`.
struct SweepItem {
    int run, w0, count, pad;
};
// One window of one run (flatness and merge) / one pair slot of one run
// (exchange: windows k, k+1 with k = 2 * slot + round mod 2).
struct WinItem {
    int run, k;
};

struct BatchDev {
    const RunDesc *runs;
    const SweepItem *sweep;
    const WinItem *win;
    const WinItem *pair;
    int n_runs, n_sweep, n_win, n_pair;
    int P;          // walkers per wave in the sweep (1, 2, 4, 8)
    int max_N, max_W;
    int j_words;    // coupling words per site of the batch's runs (0, 1 EA, 2 EA3)
    int region;     // LDS stride of the walkers' regions: sweep_region(max_W, max_N, 64/P)
    int pwaves;     // persistent form: waves per work-group (one run each)
};

// Persistent form: one work-group holds one run for several rounds.  At most
// kPersistMaxWaves waves of P walkers and kPersistMaxWalkers walkers per run;
// the run's small state lives in PersistShared (static LDS) next to the
// walkers' regions.
constexpr int kPersistMaxWalkers = 64;
constexpr int kPersistMaxWaves = 8;

struct PersistShared {
    int E[kPersistMaxWalkers];
    int flat[kPersistMaxWalkers];
    unsigned long long t[kPersistMaxWalkers];
    double lnf[kPersistMaxWalkers];
    int done[kPersistMaxWalkers];
    int phase[kPersistMaxWalkers];
    int merge[kPersistMaxWalkers];
    long long first[kPersistMaxWalkers];   // per window: round of the first merge
    long long finish[kPersistMaxWalkers];  // per window: round it finished in
    unsigned long long ex_prop[kPersistMaxWalkers], ex_acc[kPersistMaxWalkers];
    // exchange: partner permutations (pairs x m <= walkers / 2) and the
    // accepted swaps of one step
    int perm[kPersistMaxWalkers / 2];
    int sw_i[kPersistMaxWalkers / 2], sw_j[kPersistMaxWalkers / 2];
    int n_swap, all_done;
};

// Proposals staged per block of the sweep (one per lane), decoded so that
// the in-order pass over them needs no unpacking.
constexpr int kWave = 64;
struct alignas(16) Prop {
    double thr;        // ln u of the attempt
    double lnf;        // ln f added after the attempt
    int32_t d_addr;    // energy change against the block-start configuration,
                       // in bytes of the LDS ln g array
    uint32_t sp_off;   // LDS byte offset of the site's spin
    uint32_t flags;    // new state (8 bits) | Potts r1 << 16
    uint32_t old;      // old state (8 bits)
};

// LDS bytes one walker needs in the sweep with G = 64 / P attempts per block:
// ln g (8 (W + 8), with 4 guard bins on either side), H (4 W), G + 2 staged
// proposals, G per-step bin records, per-site G-bit proposal masks (G/8 N),
// spins (N), each rounded up to 16 bytes.
inline size_t lds_up16(size_t x) { return (x + 15) & ~(size_t)15; }
inline size_t sweep_walker_lds(int W, int N, int G)
{
    size_t b = 0;
    b += lds_up16((size_t)(W + 8) * 8);
    b += lds_up16((size_t)W * 4);
    b += (size_t)(G + 2) * sizeof(Prop);
    b += lds_up16((size_t)G * 4);
    b += lds_up16((size_t)N * (size_t)(G / 8));
    b += lds_up16((size_t)N);
    return b;
}

// Stride of the walkers' regions in a work-group: a multiple of 256 bytes plus
// 32, so the records the groups read at the same offset fall in different
// LDS banks.
inline size_t sweep_region(int W, int N, int G)
{
    return ((sweep_walker_lds(W, N, G) + 255) & ~(size_t)255) + 32;
}

// LDS bytes of one sweep work-group (P walkers, couplings shared by the
// group's run: 4 j_words N).
inline size_t sweep_lds_bytes(int P, int W, int N, int j_words)
{
    return (size_t)P * sweep_region(W, N, kWave / P) + (size_t)j_words * 4 * (size_t)N;
}

// coupling words per site of a model (0 for Ising and Potts, 1 EA, 2 EA3)
inline int model_j_words(int model) { return model == 2 ? 1 : (model == 3 ? 2 : 0); }

constexpr size_t kMaxLds = 160 * 1024;

// most dynamic LDS a persistent work-group may take: the CU's LDS less 8 KiB,
// which holds PersistShared (4.7 KB) with room for the allocation granule
constexpr size_t kPersistMaxDynLds = kMaxLds - 8 * 1024;

// dynamic LDS bytes of a persistent work-group: `waves` waves of P walkers'
// regions, then the run's couplings (the static PersistShared comes on top)
inline size_t persist_lds_bytes(int P, int waves, int W, int N, int j_words)
{
    return (size_t)waves * P * sweep_region(W, N, kWave / P) + (size_t)j_words * 4 * (size_t)N;
}

// The allocation-free entry point (rewl_run_noalloc) keeps everything a run
// needs besides the caller's output arrays in one static device array of
// kNoAllocScratch bytes per device; its windows are passed to the set-up
// kernel by value, so at most kNoAllocMaxWindows of them.
constexpr size_t kNoAllocScratch = 128 * 1024;
constexpr int kNoAllocMaxWindows = 64;

struct NoAllocSetup {
    RunDesc d;             // the run: outputs in the caller's arrays, the rest in the scratch
    RunDesc *desc;         // launch tables in the scratch
    SweepItem *sweep;
    WinItem *win;
    WinItem *pair;
    const int8_t *J_raw;   // the couplings as given (bonds per site x N), in the scratch
    double lnf_init;
    int lo[kNoAllocMaxWindows], hi[kNoAllocMaxWindows];
};

// device address of the static scratch on the current device (looked up once
// per device), or an error code
int rewl_noalloc_scratch(void **ptr);
// fills the run's state and the launch tables (no memset, no host copies of
// tables): ln g and H zero, counters zero, ln f = lnf_init, unfinished
// windows, couplings packed per site, one sweep item per walker
int rewl_launch_noalloc_setup(const NoAllocSetup &s, void *stream);

// launchers (rewl_kernels.hip); a launcher that returns -3 leaves the failed
// HIP call and its error in rewl_launch_error() (per thread)
const char *rewl_launch_error(void);
int rewl_launch_init(const RunDesc &a, void *stream);
// One round of every run in the batch: sweep, flatness/merge, exchange,
// round counters.  ev0/ev1 (hipEvent_t or NULL) bracket the sweep launch.
int rewl_launch_round(const BatchDev &b, void *stream, void *ev0, void *ev1);
// `rounds` rounds of every run of the batch in one launch of the persistent
// kernel (one work-group per run, b.pwaves waves each); ev0/ev1 bracket it
int rewl_launch_persist(const BatchDev &b, long long rounds, void *stream, void *ev0, void *ev1);
// per run of the batch: out_d[i] = 1 when every window of run i is done
int rewl_launch_status(const BatchDev &b, int *out_d, void *stream);
int rewl_launch_selftest_philox(const uint32_t *ctr_d, uint32_t k0, uint32_t k1, uint32_t *out_d,
                                int n);
int rewl_launch_selftest_ln_u(const uint32_t *words_d, double *out_d, int n);
