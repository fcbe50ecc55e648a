// rewl_internal.h -- host/device shared layout of one run's device state.
//
// Everything a kernel touches is described by RunDev, passed by value.  All
// arrays live in one device allocation carved by rewl_api.cpp:
//   spins   nw x Npad int8   (Ising/EA +-1, Potts 0..q-1)
//   E       nw int32         (current energy)
//   t       nw uint64        (sweep attempts made = stream-0 Philox counter)
//   flat    nw int32         (latched flatness flag of the current iteration)
//   lng     nw x Wmax f64    (window-local ln g; visited <=> lng > 0)
//   H       nw x Wmax uint32 (window-local histogram of the current iteration)
//   n_acc   nw uint64        (accepted sweep moves)
//   lnf     h f64, done h int32, finish h int64, lo/hi h int32 (bins)
//   ex_prop, ex_acc  h uint64 (exchange proposals / acceptances of pair (k,k+1))
//   J4      N uint32         (EA: couplings to right, left, down, up neighbour,
//                             one int8 each, packed little-endian)
//   status  1 int32          (start-up failure flag)
#pragma once
#include <stddef.h>
#include <stdint.h>

struct RunDev {
    int model, L, N, q, h, m, nw;
    int Npad, Wmax;
    int e_min, step;
    uint32_t l_magic;  // ceil(2^32 / L): row = mulhi(site, l_magic) for site < L*L
    long long S;
    uint32_t key0, key1;
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
    long long *finish;
    int *lo, *hi;
    unsigned long long *ex_prop, *ex_acc;
    uint32_t *J4;
    int *status;
};

// Proposals staged per block of the sweep (one per lane), decoded so that
// the in-order pass over them needs no unpacking.
constexpr int kBlock = 64;
struct alignas(16) Prop {
    double thr;        // ln u of the attempt
    int32_t d_off;     // energy change against the block-start configuration
    int32_t d_addr;    // the same change in bytes of the per-bin LDS records
    uint32_t sp_off;   // LDS byte offset of the site's spin
    uint32_t flags;    // new state (8 bits) | old state << 8 | Potts r1 << 16
                       // | 1 << 31 if an earlier proposal of the block touches
                       //   the site or one of its neighbours
    uint32_t site;
    uint32_t pad;
};

// Per-bin LDS record of the sweep: ln g and H side by side.
struct alignas(16) BinRec {
    double lng;
    uint32_t H;
    uint32_t pad;
};

// LDS bytes of one walker's sweep work-group: bins (16 W), staged proposals,
// per-site proposal masks (8 N), EA couplings (4 N), spins (N).
inline size_t sweep_lds_bytes(int model, int W, int N)
{
    size_t b = 0;
    b += (size_t)W * sizeof(BinRec);
    b += (size_t)(kBlock + 1) * sizeof(Prop);
    b += (size_t)N * 8;
    if (model == 2) b += (size_t)N * 4;
    b += ((size_t)N + 15) & ~(size_t)15;
    return b;
}

constexpr size_t kMaxLds = 160 * 1024;

// launchers (rewl_kernels.hip)
int rewl_launch_init(const RunDev &a, void *stream);
// ev0/ev1 (hipEvent_t or NULL) are recorded right before and after the sweep
int rewl_launch_round(const RunDev &a, long long round, void *stream, void *ev0, void *ev1);
int rewl_launch_selftest_philox(const uint32_t *ctr_d, uint32_t k0, uint32_t k1, uint32_t *out_d,
                                int n);
int rewl_launch_selftest_ln_u(const uint32_t *words_d, double *out_d, int n);
