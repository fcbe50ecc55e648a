/*
 * rewl_oracle.c -- plain CPU oracle for replica-exchange Wang-Landau (REWL)
 * sampling, after Vogel, Li, Wuest & Landau, arXiv:1305.5615.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It is slow and
 * written to be checked by eye against the paper; it shares no code with the
 * GPU library.  Built with -ffp-contract=off so that every floating-point
 * operation below is one IEEE binary64 operation, rounded to nearest.
 *
 * What the paper fixes (cited by passage; the letter has no numbered sections):
 *  - standard WL (the paragraph introducing g(E), before Fig. 1): a move from
 *    E_old to E_new is accepted with probability min[1, g(E_old)/g(E_new)];
 *    after every move g(E) -> f g(E) at the current energy and H(E) += 1; when
 *    H is flat, H is reset and f is reduced; the run ends at f_final.
 *  - parallel scheme (the paragraph after Fig. 1 and Eq. (1)): the energy range
 *    is split into h windows with large overlap o, m walkers per window, each
 *    with its own g and H; an exchange of configurations X, Y between walker i
 *    and a walker j of the neighbouring window is accepted with the
 *    probability of Eq. (1); when all m walkers of a window are flat their
 *    estimates are averaged and handed back, and all proceed together; the
 *    run ends when every window has reached f_final; the pieces are joined
 *    where the slopes d ln g / dE agree best.
 *
 * What the paper leaves open is fixed here (the readings are listed with their
 * reasons in the design notes of the repository):
 *  - ln f starts at lnf_init and halves at each merge (f -> sqrt f); a window is
 *    done when the halved ln f drops below lnf_final.
 *  - optional 1/t schedule (Belardinelli & Pereyra, Phys. Rev. E 75, 046701
 *    (2007), one of the update rules the paper names): once a halving would take
 *    ln f below W/t (W bins of the window, t attempts per walker), the window
 *    switches to ln f = W/t, renewed after every attempt; from then on its
 *    walkers are averaged every round without a flatness test, and the window is
 *    done when W/t drops below lnf_final.
 *  - flat: min H * n >= p * sum H over the walker's visited bins (visited is
 *    sticky over iterations and OR-ed at the merge).
 *  - windows: span = B-1, w = span/(1+(h-1)(1-o)), lo_k = floor(k(1-o)w),
 *    hi_k = min(B-1, ceil(k(1-o)w + w)), hi_{h-1} = B-1.
 *  - a round: S attempts per walker of every unfinished window, then flatness,
 *    then merges (windows in increasing order), then one exchange step over the
 *    window pairs (k, k+1) with k = round mod 2.
 *  - the "average" of the estimates is the arithmetic mean of ln g.
 *  - moves that leave the window are rejected; the current bin is updated.
 *  - randomness: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11), key = seed,
 *    counters (t, walker, stream); the acceptance test u < P is taken as
 *    ln u < ln P with ln u from the series ln x = 2 atanh((x-1)/(x+1)).
 *
 * Pins: every function here is checked by the CPU tests against something other
 * than itself (exact densities of states, enumeration, invariants, rocRAND's
 * Philox, a high-precision logarithm, sampled distributions).  Parity
 * unpinned: the accuracy of the large workloads (q = 10 Potts 64x64, +-J 24x24,
 * the 12^3 glass) has no exact density of states to compare with; there only
 * the invariants of the small cases and bit-exactness of the GPU path apply.
 */
#include "rewl_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- Philox ---
 * Philox4x32-10 as published by Salmon et al. (SC'11): ten rounds; each round
 * multiplies counter words 0 and 2 by the two round multipliers (full 64-bit
 * products), the new word 0 is hi(product of word 2) ^ word 1 ^ key 0, the new
 * word 1 is lo(product of word 2), the new word 2 is hi(product of word 0) ^
 * word 3 ^ key 1, the new word 3 is lo(product of word 0); the key is bumped by
 * the two Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* draw(ctr) for counter (a, b, walker, stream) with key = seed */
static void draw(uint64_t seed, uint64_t counter, uint32_t walker, uint32_t stream,
                 uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)counter, (uint32_t)(counter >> 32), walker, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* uniform integer in [0, n): the high word of the 64-bit product word * n */
static uint32_t mulhi32(uint32_t word, uint32_t n)
{
    return (uint32_t)(((uint64_t)word * (uint64_t)n) >> 32);
}

/* u in (0,1) from two words: k = (hi << 20) | (lo >> 12), 52 bits;
 * u = (2k + 1) * 2^-53, exact in binary64 and never 0. */
double orc_uniform(uint32_t hi, uint32_t lo)
{
    uint64_t k = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return (double)(2 * k + 1) * 0x1p-53;
}

/* ------------------------------------------------------------------ ln u ---
 * ln u for u in (0,1), from u = f 2^e and ln f = 2 atanh(s), s = (f-1)/(f+1):
 *   ln f = 2 (s + s z Q(z)),  z = s^2,  Q(z) = 1/3 + z/5 + ... + z^10/23
 * with f moved into [sqrt(2)/2, sqrt(2)] so |s| <= 0.1716 and the truncated
 * series is below 2^-60 relative.  ln 2 enters as LN2_HI + LN2_LO, LN2_HI being
 * ln 2 rounded to 32 fractional bits so that e * LN2_HI is exact. */
static const double LN2_HI = 0x1.62e42ffp-1;        /* round(ln2 * 2^32) / 2^32 */
static const double LN2_LO = -0x1.718432a1b0e26p-35; /* RN(ln2 - LN2_HI) */
static const double SQRT2 = 0x1.6a09e667f3bcdp+0;  /* RN(sqrt 2) */

/* One Horner step of ln u's series, Q z + c rounded once (a fused multiply-add,
 * C99 fma).  Where the host has the FMA instructions the step is compiled to
 * one of them; elsewhere libm's fma gives the same, correctly rounded, value. */
#if defined(__x86_64__) && defined(__GNUC__)
__attribute__((target("fma"))) static double horner_hw(double Q, double z, double c)
{
    return __builtin_fma(Q, z, c);
}
static double horner_sw(double Q, double z, double c) { return fma(Q, z, c); }
/* set once when the library is loaded, before any thread reads it */
static int have_fma = 0;
__attribute__((constructor)) static void detect_fma(void)
{
    __builtin_cpu_init();
    have_fma = __builtin_cpu_supports("fma") ? 1 : 0;
}
static double horner(double Q, double z, double c)
{
    return have_fma ? horner_hw(Q, z, c) : horner_sw(Q, z, c);
}
#else
static double horner(double Q, double z, double c) { return fma(Q, z, c); }
#endif

double orc_ln_u(double u)
{
    int e;
    double f = frexp(u, &e);       /* u = f 2^e, f in [0.5, 1) */
    f = f * 2.0;                   /* f in [1, 2), exact */
    e = e - 1;
    if (f > SQRT2) {               /* fold into [sqrt2/2, sqrt2] */
        f = f * 0.5;
        e = e + 1;
    }
    double s = (f - 1.0) / (f + 1.0);
    double z = s * s;
    /* Horner over c_i = RN(1/(2i+1)), i = 11 .. 1, each step one fused
     * multiply-add; the leading term 1 is added last, as s + s z Q(z), to keep
     * the rounding error near one ulp */
    double Q = 1.0 / 23.0;
    for (int i = 10; i >= 1; --i)
        Q = horner(Q, z, 1.0 / (double)(2 * i + 1));
    double ed = (double)e;
    double lnf = (s + s * (z * Q)) * 2.0;
    return ed * LN2_HI + (ed * LN2_LO + lnf);
}

/* ---------------------------------------------------------------- models ---
 * Sites i = r L + c on an L x L torus.  Ising: E = -sum_<ij> s_i s_j;
 * Potts: E = -sum_<ij> delta(s_i, s_j); +-J (Edwards-Anderson):
 * E = -sum_<ij> J_ij s_i s_j.  Each bond is counted once through the right and
 * lower neighbour of every site.  The 3D +-J model (the paper's 12^3 spin-glass
 * test) lives on an L x L x L torus, sites i = (z L + y) L + x, with couplings
 * J[3i] to +x, J[3i+1] to +y and J[3i+2] to +z. */
static int right_of(int i, int L) { int r = i / L, c = i % L; return r * L + (c + 1) % L; }
static int left_of(int i, int L)  { int r = i / L, c = i % L; return r * L + (c + L - 1) % L; }
static int down_of(int i, int L)  { int r = i / L, c = i % L; return ((r + 1) % L) * L + c; }
static int up_of(int i, int L)    { int r = i / L, c = i % L; return ((r + L - 1) % L) * L + c; }

/* neighbour of site i one step along axis a (0: x, 1: y, 2: z) in direction
 * d (+1 or -1) on the L^3 torus */
static int nb3(int i, int L, int a, int d)
{
    int x = i % L, y = (i / L) % L, z = i / (L * L);
    if (a == 0) x = (x + d + L) % L;
    else if (a == 1) y = (y + d + L) % L;
    else z = (z + d + L) % L;
    return (z * L + y) * L + x;
}

int orc_sites(int model, int L) { return model == ORC_EA3 ? L * L * L : L * L; }

int64_t orc_energy(int model, int L, int q, const int8_t *s, const int8_t *J)
{
    (void)q;
    int N = orc_sites(model, L);
    int64_t E = 0;
    for (int i = 0; i < N; ++i) {
        if (model == ORC_EA3) {
            for (int a = 0; a < 3; ++a)
                E -= (int64_t)J[3 * i + a] * s[i] * s[nb3(i, L, a, +1)];
            continue;
        }
        int rt = right_of(i, L), dn = down_of(i, L);
        if (model == ORC_ISING) {
            E -= (int64_t)s[i] * s[rt] + (int64_t)s[i] * s[dn];
        } else if (model == ORC_POTTS) {
            E -= (s[i] == s[rt]) + (s[i] == s[dn]);
        } else {
            E -= (int64_t)J[2 * i] * s[i] * s[rt] + (int64_t)J[2 * i + 1] * s[i] * s[dn];
        }
    }
    return E;
}

/* energy change when site i goes from s[i] to `nw` */
static int64_t delta_e(int model, int L, const int8_t *s, const int8_t *J, int i, int nw)
{
    if (model == ORC_EA3) {
        int64_t h = 0;
        for (int a = 0; a < 3; ++a) {
            int up = nb3(i, L, a, +1), dn = nb3(i, L, a, -1);
            h += (int64_t)J[3 * i + a] * s[up] + (int64_t)J[3 * dn + a] * s[dn];
        }
        return 2 * (int64_t)s[i] * h;
    }
    int rt = right_of(i, L), lf = left_of(i, L), dn = down_of(i, L), up = up_of(i, L);
    if (model == ORC_ISING)
        return 2 * (int64_t)s[i] * (s[rt] + s[lf] + s[dn] + s[up]);
    if (model == ORC_EA)
        return 2 * (int64_t)s[i] *
               (J[2 * i] * s[rt] + J[2 * lf] * s[lf] + J[2 * i + 1] * s[dn] + J[2 * up + 1] * s[up]);
    int old = s[i];
    int same_old = (s[rt] == old) + (s[lf] == old) + (s[dn] == old) + (s[up] == old);
    int same_new = (s[rt] == nw) + (s[lf] == nw) + (s[dn] == nw) + (s[up] == nw);
    return (int64_t)same_old - same_new;
}

/* ------------------------------------------------------------- partition --- */
int orc_partition(int64_t B, int h, double o, int64_t *lo, int64_t *hi)
{
    if (B < 2 || h < 1 || !(o > 0.0 && o < 1.0)) return -1;
    double span = (double)(B - 1);
    double w = span / (1.0 + (double)(h - 1) * (1.0 - o));
    for (int k = 0; k < h; ++k) {
        double x = ((double)k * (1.0 - o)) * w;
        lo[k] = (int64_t)floor(x);
        int64_t top = (int64_t)ceil(x + w);
        hi[k] = top < B - 1 ? top : B - 1;
    }
    hi[h - 1] = B - 1;
    for (int k = 0; k < h; ++k) {
        if (hi[k] - lo[k] + 1 < 2) return -1;
        if (k + 1 < h) {
            if (lo[k + 1] <= lo[k] || hi[k + 1] < hi[k]) return -1;
            if (hi[k] - lo[k + 1] + 1 < 2) return -1;
        }
    }
    return 0;
}

/* Check a partition: h windows of >= 2 bins from bin 0 to bin B-1, starts and
 * ends increasing, adjacent windows sharing >= 2 bins. */
static int partition_ok(int64_t B, int h, const int64_t *lo, const int64_t *hi)
{
    if (h < 1 || lo[0] != 0 || hi[h - 1] != B - 1) return 0;
    for (int k = 0; k < h; ++k) {
        if (lo[k] < 0 || hi[k] > B - 1 || hi[k] - lo[k] + 1 < 2) return 0;
        if (k + 1 < h) {
            if (lo[k + 1] <= lo[k] || hi[k + 1] <= hi[k]) return 0;
            if (hi[k] - lo[k + 1] + 1 < 2) return 0;
        }
    }
    return 1;
}

/* Run-time balanced partition (the paper's Fig. 1b and its scaling
 * discussion: windows chosen so that all finish the first WL iteration after
 * the same number of sweeps, estimated from a pre-run on the equal
 * partition).  The pre-run's window k (bins pre_lo[k]..pre_hi[k]) needed T_k
 * rounds for its first iteration; a bin's first-iteration time density t(b)
 * is the mean of T_k / W_k over the pre-run windows that contain it.  Bins are
 * points on a time axis F with F(0) = 0 and F(b+1) = F(b) + (t(b) + t(b+1))/2,
 * and the new windows are the equal partition of that axis: window k covers
 * F in [x_k, x_k + w], x_k = k (1-o) w, w = F(B-1) / (1 + (h-1)(1-o)); lo_k is
 * the last bin with F <= x_k, hi_k the first bin with F >= x_k + w (B-1 for
 * the last window).  With t = 1 everywhere this is orc_partition exactly. */
int orc_partition_balanced(int64_t B, int h, double o, int pre_h, const int64_t *pre_lo,
                           const int64_t *pre_hi, const int64_t *T, int64_t *lo, int64_t *hi)
{
    if (B < 2 || h < 1 || pre_h < 1 || !(o > 0.0 && o < 1.0)) return -1;
    if (!partition_ok(B, pre_h, pre_lo, pre_hi)) return -1;
    for (int k = 0; k < pre_h; ++k) if (T[k] < 1) return -1;
    double *t = malloc((size_t)B * sizeof(double));
    double *F = malloc((size_t)B * sizeof(double));
    if (!t || !F) { free(t); free(F); return -2; }
    for (int64_t b = 0; b < B; ++b) {
        double sum = 0.0;
        int n = 0;
        for (int k = 0; k < pre_h; ++k) {
            if (b < pre_lo[k] || b > pre_hi[k]) continue;
            sum = sum + (double)T[k] / (double)(pre_hi[k] - pre_lo[k] + 1);
            n += 1;
        }
        t[b] = sum / (double)n;
    }
    F[0] = 0.0;
    for (int64_t b = 0; b + 1 < B; ++b) F[b + 1] = F[b] + (t[b] + t[b + 1]) * 0.5;
    double w = F[B - 1] / (1.0 + (double)(h - 1) * (1.0 - o));
    for (int k = 0; k < h; ++k) {
        double x = ((double)k * (1.0 - o)) * w;
        double y = x + w;
        int64_t a = 0;
        while (a + 1 < B && F[a + 1] <= x) ++a;
        int64_t e = 0;
        while (e < B - 1 && F[e] < y) ++e;
        lo[k] = a;
        hi[k] = e;
    }
    hi[h - 1] = B - 1;
    free(t);
    free(F);
    return partition_ok(B, h, lo, hi) ? 0 : -1;
}

/* ------------------------------------------------------------------- run --- */
struct orc_run {
    int model, L, q, N, h, m, nw, n_threads;
    int64_t e_min, e_max, step, B, S, round;
    int full_lo, full_hi;   /* requested range reached the ground / top state */
    double p, lnf_final;
    int schedule;       /* 0: halving, 1: halving then 1/t */
    uint64_t seed;
    int8_t *J;          /* 2N, EA only */
    int64_t *lo, *hi;   /* h windows, bins */
    int64_t Wmax;
    double *lnf;        /* h */
    int *done;          /* h */
    int *phase;         /* h: 1 once the window runs the 1/t rule */
    int64_t *finish;    /* h: round in which the window finished, -1 before */
    int64_t *first;     /* h: round of the window's first merge, -1 before */
    int8_t *spins;      /* nw * N */
    int64_t *E;         /* nw */
    uint64_t *t;        /* nw */
    int *flat;          /* nw */
    double *lng;        /* nw * Wmax, window-local */
    uint32_t *H;        /* nw * Wmax */
    uint8_t *vis;       /* nw * Wmax */
    uint64_t *n_acc;    /* nw */
    uint64_t ex_prop, ex_acc;
    int *perm;          /* m: exchange partner permutation (scratch) */
    int8_t *swap;       /* N: configuration swap buffer (scratch) */
};

static int window_of(const orc_run *run, int w) { return w / run->m; }
static int64_t wsize(const orc_run *run, int k) { return run->hi[k] - run->lo[k] + 1; }
static int64_t bin_of(const orc_run *run, int64_t E) { return (E - run->e_min) / run->step; }
static int in_window(const orc_run *run, int k, int64_t E)
{
    if (E < run->e_min || E > run->e_max) return 0;
    int64_t b = bin_of(run, E);
    return b >= run->lo[k] && b <= run->hi[k];
}

void orc_destroy(orc_run *run)
{
    if (!run) return;
    free(run->J); free(run->lo); free(run->hi); free(run->lnf); free(run->done); free(run->phase);
    free(run->finish); free(run->first); free(run->spins); free(run->E); free(run->t); free(run->flat);
    free(run->lng); free(run->H); free(run->vis); free(run->n_acc);
    free(run->perm); free(run->swap);
    free(run);
}

/* start-up of walker w: random spins (stream 1), then single-site moves
 * (stream 2, proposed as in a sweep) accepted whenever they do not take the
 * energy further from the window; Ising and Potts walkers that are still
 * outside after 200 N moves restart from the ordered state. */
static int64_t dist_to_window(const orc_run *run, int k, int64_t E)
{
    int64_t lo_e = run->e_min + run->lo[k] * run->step;
    int64_t hi_e = run->e_min + run->hi[k] * run->step;
    if (E < lo_e) return lo_e - E;
    if (E > hi_e) return E - hi_e;
    return 0;
}

static int init_walker(orc_run *run, int w)
{
    int N = run->N, k = window_of(run, w);
    int8_t *s = run->spins + (size_t)w * N;
    uint32_t r[4];
    for (int i = 0; i < N; ++i) {
        draw(run->seed, (uint64_t)i, (uint32_t)w, 1u, r);
        if (run->model == ORC_POTTS)
            s[i] = (int8_t)mulhi32(r[0], (uint32_t)run->q);
        else
            s[i] = (r[0] >> 31) ? 1 : -1;
    }
    int64_t E = orc_energy(run->model, run->L, run->q, s, run->J);
    int64_t cap = 200 * (int64_t)N;
    uint64_t d = 0;
    while (dist_to_window(run, k, E) > 0) {
        if (d == (uint64_t)cap) {
            if (run->model == ORC_EA || run->model == ORC_EA3) return -4;
            for (int i = 0; i < N; ++i) s[i] = (run->model == ORC_POTTS) ? 0 : 1;
            E = orc_energy(run->model, run->L, run->q, s, run->J);
        }
        if (d == (uint64_t)(2 * cap)) return -4;
        draw(run->seed, d, (uint32_t)w, 2u, r);
        d += 1;
        int site = (int)mulhi32(r[0], (uint32_t)N);
        int nw = (run->model == ORC_POTTS)
                     ? (s[site] + 1 + (int)mulhi32(r[1], (uint32_t)(run->q - 1))) % run->q
                     : -s[site];
        int64_t En = E + delta_e(run->model, run->L, s, run->J, site, nw);
        if (dist_to_window(run, k, En) <= dist_to_window(run, k, E)) {
            s[site] = (int8_t)nw;
            E = En;
        }
    }
    run->E[w] = E;
    return 0;
}

int orc_create(orc_run **out, int model, int L, int q, const int8_t *couplings,
               int64_t e_min, int64_t e_max, int h, double o, int m, double p,
               double lnf_init, double lnf_final, int64_t S, uint64_t seed, int n_threads,
               int schedule, const int64_t *win_lo, const int64_t *win_hi)
{
    *out = NULL;
    if (model < 0 || model > 3 || L > 256 || h < 1 || m < 1 || S < 1) return -1;
    if (model == ORC_EA3 ? (L < 2 || L > 32) : L < 3) return -1;
    if (model == ORC_POTTS && (q < 2 || q > 127)) return -1;
    if ((model == ORC_EA || model == ORC_EA3) && !couplings) return -1;
    if (!(p > 0.0 && p <= 1.0) || !(lnf_final > 0.0) || !(lnf_init > 0.0)) return -1;
    if (schedule != 0 && schedule != 1) return -1;
    int N = orc_sites(model, L);
    int bonds = (model == ORC_EA3) ? 3 : 2;   /* bonds per site */
    int64_t step = (model == ORC_POTTS) ? 1 : 4;
    int64_t lo_full = -(int64_t)bonds * N, hi_full = (model == ORC_POTTS) ? 0 : (int64_t)bonds * N;
    int64_t cls = 0; /* energies lie on cls + step Z */
    if (model == ORC_EA || model == ORC_EA3) {
        int64_t n_neg = 0;
        for (int i = 0; i < bonds * N; ++i) {
            if (couplings[i] != 1 && couplings[i] != -1) return -1;
            n_neg += couplings[i] < 0;
        }
        cls = -(int64_t)bonds * N + 2 * n_neg;
    } else if (model == ORC_ISING) {
        cls = -2 * (int64_t)N;
    }
    int full_lo = e_min <= lo_full, full_hi = e_max >= hi_full;
    if (e_min < lo_full) e_min = lo_full;
    if (e_max > hi_full) e_max = hi_full;
    /* align onto the class: e_min up, e_max down */
    int64_t rm = ((e_min - cls) % step + step) % step;
    if (rm) e_min += step - rm;
    rm = ((e_max - cls) % step + step) % step;
    e_max -= rm;
    if (e_max <= e_min) return -1;

    orc_run *run = calloc(1, sizeof(*run));
    if (!run) return -2;
    run->model = model; run->L = L; run->q = (model == ORC_POTTS) ? q : 2; run->N = N;
    run->h = h; run->m = m; run->nw = h * m; run->n_threads = n_threads;
    run->e_min = e_min; run->e_max = e_max; run->step = step;
    run->full_lo = full_lo; run->full_hi = full_hi;
    run->B = (e_max - e_min) / step + 1; run->S = S; run->p = p;
    run->lnf_final = lnf_final; run->seed = seed; run->schedule = schedule;
    run->lo = calloc(h, sizeof(int64_t)); run->hi = calloc(h, sizeof(int64_t));
    if (!run->lo || !run->hi) { orc_destroy(run); return -2; }
    if (win_lo && win_hi) {
        for (int k = 0; k < h; ++k) { run->lo[k] = win_lo[k]; run->hi[k] = win_hi[k]; }
        if (!partition_ok(run->B, h, run->lo, run->hi)) { orc_destroy(run); return -1; }
    } else if (orc_partition(run->B, h, o, run->lo, run->hi)) {
        orc_destroy(run);
        return -1;
    }
    run->Wmax = 0;
    for (int k = 0; k < h; ++k) if (wsize(run, k) > run->Wmax) run->Wmax = wsize(run, k);
    size_t nw = (size_t)run->nw;
    run->J = calloc((size_t)bonds * N, 1);
    run->lnf = calloc(h, sizeof(double)); run->done = calloc(h, sizeof(int));
    run->phase = calloc(h, sizeof(int));
    run->finish = calloc(h, sizeof(int64_t));
    run->first = calloc(h, sizeof(int64_t));
    run->spins = calloc(nw * N, 1); run->E = calloc(nw, sizeof(int64_t));
    run->t = calloc(nw, sizeof(uint64_t)); run->flat = calloc(nw, sizeof(int));
    run->lng = calloc(nw * run->Wmax, sizeof(double));
    run->H = calloc(nw * run->Wmax, sizeof(uint32_t));
    run->vis = calloc(nw * run->Wmax, 1);
    run->n_acc = calloc(nw, sizeof(uint64_t));
    run->perm = calloc((size_t)m, sizeof(int));
    run->swap = calloc((size_t)N, 1);
    if (!run->J || !run->lnf || !run->done || !run->phase || !run->finish || !run->first ||
        !run->spins || !run->E || !run->t || !run->flat || !run->lng || !run->H ||
        !run->vis || !run->n_acc || !run->perm || !run->swap) {
        orc_destroy(run);
        return -2;
    }
    if (model == ORC_EA || model == ORC_EA3) memcpy(run->J, couplings, (size_t)bonds * N);
    for (int k = 0; k < h; ++k) { run->lnf[k] = lnf_init; run->finish[k] = -1; run->first[k] = -1; }
    for (int w = 0; w < run->nw; ++w) {
        int rc = init_walker(run, w);
        if (rc) { orc_destroy(run); return rc; }
    }
    *out = run;
    return 0;
}

/* S Wang-Landau attempts of walker w (one Philox draw per attempt, stream 0):
 * word 0 picks the site, word 1 the new Potts state, words 2 and 3 give u.
 * A move out of the window is rejected; otherwise it is accepted iff
 * ln u < ln g(E_old) - ln g(E_new).  Then ln g and H of the current bin grow. */
static void sweep_walker(orc_run *run, int w)
{
    int N = run->N, k = window_of(run, w);
    int8_t *s = run->spins + (size_t)w * N;
    double *lng = run->lng + (size_t)w * run->Wmax;
    uint32_t *H = run->H + (size_t)w * run->Wmax;
    uint8_t *vis = run->vis + (size_t)w * run->Wmax;
    double lnf = run->lnf[k];
    int one_over_t = run->phase[k];
    double Wd = (double)wsize(run, k);
    int64_t lo = run->lo[k];
    int64_t E = run->E[w];
    uint64_t acc = 0;
    for (int64_t a = 0; a < run->S; ++a) {
        uint32_t r[4];
        draw(run->seed, run->t[w], (uint32_t)w, 0u, r);
        run->t[w] += 1;
        int site = (int)mulhi32(r[0], (uint32_t)N);
        int nw = (run->model == ORC_POTTS)
                     ? (s[site] + 1 + (int)mulhi32(r[1], (uint32_t)(run->q - 1))) % run->q
                     : -s[site];
        double u = orc_uniform(r[2], r[3]);
        int64_t En = E + delta_e(run->model, run->L, s, run->J, site, nw);
        if (in_window(run, k, En)) {
            double d = lng[bin_of(run, E) - lo] - lng[bin_of(run, En) - lo];
            if (orc_ln_u(u) < d) {
                s[site] = (int8_t)nw;
                E = En;
                acc += 1;
            }
        }
        int64_t b = bin_of(run, E) - lo;
        if (one_over_t) lnf = Wd / (double)run->t[w]; /* W / attempts made so far */
        lng[b] = lng[b] + lnf;
        H[b] += 1;
        vis[b] = 1;
    }
    run->E[w] = E;
    run->n_acc[w] += acc;
}

static int is_flat(const orc_run *run, int w)
{
    int k = window_of(run, w);
    const uint32_t *H = run->H + (size_t)w * run->Wmax;
    const uint8_t *vis = run->vis + (size_t)w * run->Wmax;
    uint64_t n = 0, sum = 0;
    uint32_t hmin = 0xFFFFFFFFu;
    for (int64_t b = 0; b < wsize(run, k); ++b) {
        if (!vis[b]) continue;
        n += 1;
        sum += H[b];
        if (H[b] < hmin) hmin = H[b];
    }
    if (n == 0) return 0;
    return (double)hmin * (double)n >= run->p * (double)sum;
}

static void merge_window(orc_run *run, int k, int64_t round)
{
    int m = run->m;
    int64_t W = wsize(run, k);
    double inv = 1.0 / (double)m;
    int pow2 = (m & (m - 1)) == 0;
    for (int64_t b = 0; b < W; ++b) {
        double sum = 0.0;
        uint8_t any = 0;
        for (int s = 0; s < m; ++s) {
            int w = k * m + s;
            sum = sum + run->lng[(size_t)w * run->Wmax + b];
            any |= run->vis[(size_t)w * run->Wmax + b];
        }
        double mean = pow2 ? sum * inv : sum / (double)m;
        for (int s = 0; s < m; ++s) {
            int w = k * m + s;
            run->lng[(size_t)w * run->Wmax + b] = mean;
            run->vis[(size_t)w * run->Wmax + b] = any;
            run->H[(size_t)w * run->Wmax + b] = 0;
        }
    }
    for (int s = 0; s < m; ++s) run->flat[k * m + s] = 0;
    if (run->first[k] < 0) run->first[k] = round;
    double Wt = (double)W / (double)run->t[k * m]; /* the window's walkers share t */
    if (run->phase[k]) {
        run->lnf[k] = Wt;
    } else {
        run->lnf[k] = run->lnf[k] * 0.5;
        if (run->schedule == 1 && run->lnf[k] < Wt) {
            run->phase[k] = 1;
            run->lnf[k] = Wt;
        }
    }
    if (run->lnf[k] < run->lnf_final) {
        run->done[k] = 1;
        run->finish[k] = round;
    }
}

/* one exchange step: window pairs (k, k+1) with k = round mod 2, both unfinished.
 * Stream 3 words for the pair, counter (round, k, 3 | call << 8): first a
 * Fisher-Yates shuffle pi of the m slots of window k+1, then one u per pair.
 * Walker a of window k (configuration X) and walker pi[a] of window k+1
 * (configuration Y) swap when both energies lie in both windows and
 * ln u < [ln g_i(E_X) - ln g_i(E_Y)] + [ln g_j(E_Y) - ln g_j(E_X)]  (Eq. (1)). */
typedef struct {
    uint64_t seed, round;
    uint32_t k, call, idx, buf[4];
} word_src;

static uint32_t next_word(word_src *ws)
{
    if (ws->idx == 4) {
        uint32_t ctr[4] = {(uint32_t)ws->round, (uint32_t)(ws->round >> 32), ws->k,
                           3u | (ws->call << 8)};
        uint32_t key[2] = {(uint32_t)ws->seed, (uint32_t)(ws->seed >> 32)};
        orc_philox4x32_10(ctr, key, ws->buf);
        ws->call += 1;
        ws->idx = 0;
    }
    return ws->buf[ws->idx++];
}

static void exchange(orc_run *run, int64_t round)
{
    int m = run->m, N = run->N;
    int *perm = run->perm;
    int8_t *tmp = run->swap;
    for (int k = (int)(round % 2); k + 1 < run->h; k += 2) {
        if (run->done[k] || run->done[k + 1]) continue;
        word_src ws = {run->seed, (uint64_t)round, (uint32_t)k, 0, 4, {0, 0, 0, 0}};
        for (int a = 0; a < m; ++a) perm[a] = a;
        for (int a = m - 1; a >= 1; --a) {
            int j = (int)mulhi32(next_word(&ws), (uint32_t)(a + 1));
            int x = perm[a]; perm[a] = perm[j]; perm[j] = x;
        }
        for (int a = 0; a < m; ++a) {
            uint32_t hi = next_word(&ws);
            uint32_t lo = next_word(&ws);
            double u = orc_uniform(hi, lo);
            int wi = k * m + a, wj = (k + 1) * m + perm[a];
            int64_t EX = run->E[wi], EY = run->E[wj];
            run->ex_prop += 1;
            if (!in_window(run, k + 1, EX) || !in_window(run, k, EY)) continue;
            const double *gi = run->lng + (size_t)wi * run->Wmax;
            const double *gj = run->lng + (size_t)wj * run->Wmax;
            int64_t li = run->lo[k], lj = run->lo[k + 1];
            double lnP = (gi[bin_of(run, EX) - li] - gi[bin_of(run, EY) - li]) +
                         (gj[bin_of(run, EY) - lj] - gj[bin_of(run, EX) - lj]);
            if (orc_ln_u(u) < lnP) {
                memcpy(tmp, run->spins + (size_t)wi * N, (size_t)N);
                memcpy(run->spins + (size_t)wi * N, run->spins + (size_t)wj * N, (size_t)N);
                memcpy(run->spins + (size_t)wj * N, tmp, (size_t)N);
                run->E[wi] = EY;
                run->E[wj] = EX;
                run->ex_acc += 1;
            }
        }
    }
}

static int all_done(const orc_run *run)
{
    for (int k = 0; k < run->h; ++k) if (!run->done[k]) return 0;
    return 1;
}

static void one_round(orc_run *run)
{
    int64_t r = run->round;
    if (all_done(run)) { run->round += 1; return; }
#ifdef _OPENMP
    int nt = run->n_threads > 0 ? run->n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
#endif
    for (int w = 0; w < run->nw; ++w)
        if (!run->done[window_of(run, w)]) sweep_walker(run, w);
    for (int w = 0; w < run->nw; ++w)
        if (!run->done[window_of(run, w)] && !run->phase[window_of(run, w)] && !run->flat[w])
            run->flat[w] = is_flat(run, w);
    for (int k = 0; k < run->h; ++k) {
        if (run->done[k]) continue;
        int all = 1;
        for (int s = 0; s < run->m; ++s) all &= run->flat[k * run->m + s];
        if (all || run->phase[k]) merge_window(run, k, r);
    }
    exchange(run, r);
    run->round += 1;
}

int orc_step(orc_run *run, int64_t rounds)
{
    for (int64_t i = 0; i < rounds; ++i) one_round(run);
    return 0;
}

int orc_run_to(orc_run *run, int64_t max_rounds)
{
    for (int64_t i = 0; max_rounds < 0 || i < max_rounds; ++i) {
        if (all_done(run)) return 0;
        one_round(run);
    }
    return all_done(run) ? 0 : 1;
}

void orc_info(const orc_run *run, int64_t *n_bins, int64_t *e_min, int64_t *e_step,
              int *n_windows, int *m, int *n_sites, int64_t *round, int *done)
{
    *n_bins = run->B; *e_min = run->e_min; *e_step = run->step;
    *n_windows = run->h; *m = run->m; *n_sites = run->N; *round = run->round;
    *done = all_done(run);
}

void orc_window(const orc_run *run, int k, int64_t *lo, int64_t *hi, double *lnf,
                int *done, int64_t *finish)
{
    *lo = run->lo[k]; *hi = run->hi[k]; *lnf = run->lnf[k]; *done = run->done[k];
    *finish = run->finish[k];
}

int orc_walker(const orc_run *run, int w, int8_t *spins, int64_t *E, uint64_t *t, int *flat,
               double *lng, uint32_t *H, uint8_t *visited)
{
    if (w < 0 || w >= run->nw) return -1;
    int64_t W = wsize(run, window_of(run, w));
    if (spins) memcpy(spins, run->spins + (size_t)w * run->N, (size_t)run->N);
    if (E) *E = run->E[w];
    if (t) *t = run->t[w];
    if (flat) *flat = run->flat[w];
    if (lng) memcpy(lng, run->lng + (size_t)w * run->Wmax, sizeof(double) * (size_t)W);
    if (H) memcpy(H, run->H + (size_t)w * run->Wmax, sizeof(uint32_t) * (size_t)W);
    if (visited) memcpy(visited, run->vis + (size_t)w * run->Wmax, (size_t)W);
    return 0;
}

int orc_set_lng(orc_run *run, int w, const double *lng)
{
    if (w < 0 || w >= run->nw) return -1;
    int64_t W = wsize(run, window_of(run, w));
    for (int64_t b = 0; b < W; ++b) {
        run->lng[(size_t)w * run->Wmax + b] = lng[b];
        run->vis[(size_t)w * run->Wmax + b] = lng[b] > 0.0;
    }
    return 0;
}

void orc_first_merge(const orc_run *run, int64_t *out)
{
    for (int k = 0; k < run->h; ++k) out[k] = run->first[k];
}

void orc_stats(const orc_run *run, uint64_t *attempts, uint64_t *accepts, uint64_t *ex_prop,
               uint64_t *ex_acc)
{
    uint64_t a = 0, c = 0;
    for (int w = 0; w < run->nw; ++w) { a += run->t[w]; c += run->n_acc[w]; }
    *attempts = a; *accepts = c; *ex_prop = run->ex_prop; *ex_acc = run->ex_acc;
}

/* ---------------------------------------------------------------- stitch ---
 * Pieces P_k (window-local ln g of window k, `stride` apart) are joined in
 * order.  For windows k and k+1, the candidate joining bins are the bins of
 * their overlap visited in both pieces, at or above the previous joining bin;
 * with b' the next such bin, the slopes (P(b') - P(b)) / (b' - b) of the two
 * pieces are compared and the bin where they agree best (lowest bin on ties)
 * is the joining bin b*.  Piece k+1 is shifted to match piece k at b*; bins
 * below b* come from piece k, from b* on from piece k+1.  Unvisited: -inf. */
int orc_stitch(int h, const int64_t *lo, const int64_t *hi, const double *P, int64_t stride,
               const uint8_t *vis, int64_t B, double *out, int64_t *joins)
{
    for (int64_t b = 0; b < B; ++b) out[b] = -INFINITY;
    double shift = 0.0;
    int64_t start = lo[0];
    for (int k = 0; k < h; ++k) {
        const double *pk = P + (size_t)k * stride;
        const uint8_t *vk = vis + (size_t)k * stride;
        int64_t end = hi[k]; /* last bin taken from piece k (inclusive) */
        double next_shift = 0.0;
        if (k + 1 < h) {
            const double *pn = P + (size_t)(k + 1) * stride;
            const uint8_t *vn = vis + (size_t)(k + 1) * stride;
            int64_t a = lo[k + 1] > start ? lo[k + 1] : start;
            int64_t best = -1;
            double best_diff = INFINITY;
            int64_t prev = -1;
            for (int64_t b = a; b <= hi[k]; ++b) {
                if (!vk[b - lo[k]] || !vn[b - lo[k + 1]]) continue;
                if (prev >= 0) {
                    double sk = (pk[b - lo[k]] - pk[prev - lo[k]]) / (double)(b - prev);
                    double sn = (pn[b - lo[k + 1]] - pn[prev - lo[k + 1]]) / (double)(b - prev);
                    double diff = fabs(sk - sn);
                    if (diff < best_diff) { best_diff = diff; best = prev; }
                }
                prev = b;
            }
            if (best < 0) return -7;
            if (joins) joins[k] = best;
            end = best - 1;
            next_shift = shift + (pk[best - lo[k]] - pn[best - lo[k + 1]]);
        }
        for (int64_t b = start; b <= end; ++b)
            if (vk[b - lo[k]]) out[b] = pk[b - lo[k]] + shift;
        if (k + 1 < h) {
            start = end + 1;
            shift = next_shift;
        }
    }
    return 0;
}

/* normalisation: Ising ln g(-2N) = ln 2 and Potts ln g(-2N) = ln q when the
 * requested range starts at the ground state; +-J: ln sum g = N ln 2 when the
 * requested range is the whole [-2N, 2N]; otherwise the lowest visited bin is
 * set to 0. */
int orc_get_lng(orc_run *run, double *out, int64_t cap)
{
    if (cap < run->B) return -1;
    int h = run->h;
    double *P = malloc(sizeof(double) * (size_t)h * run->Wmax);
    uint8_t *V = malloc((size_t)h * run->Wmax);
    if (!P || !V) { free(P); free(V); return -2; }
    for (int k = 0; k < h; ++k) {
        int w = k * run->m; /* all walkers of a window agree after the last merge */
        memcpy(P + (size_t)k * run->Wmax, run->lng + (size_t)w * run->Wmax,
               sizeof(double) * (size_t)run->Wmax);
        memcpy(V + (size_t)k * run->Wmax, run->vis + (size_t)w * run->Wmax, (size_t)run->Wmax);
    }
    int rc = orc_stitch(h, run->lo, run->hi, P, run->Wmax, V, run->B, out, NULL);
    free(P);
    free(V);
    if (rc) return rc;
    int64_t N = run->N;
    double ref = 0.0, target = 0.0;
    int glass = run->model == ORC_EA || run->model == ORC_EA3;
    if (!glass && run->full_lo && isfinite(out[0])) {
        ref = out[0];
        target = log(run->model == ORC_POTTS ? (double)run->q : 2.0);
    } else if (glass && run->full_lo && run->full_hi) {
        double mx = -INFINITY;
        for (int64_t b = 0; b < run->B; ++b) if (out[b] > mx) mx = out[b];
        double sum = 0.0;
        for (int64_t b = 0; b < run->B; ++b)
            if (isfinite(out[b])) sum = sum + exp(out[b] - mx);
        ref = mx + log(sum);
        target = (double)N * log(2.0);
    } else {
        for (int64_t b = 0; b < run->B; ++b)
            if (isfinite(out[b])) { ref = out[b]; break; }
    }
    for (int64_t b = 0; b < run->B; ++b)
        if (isfinite(out[b])) out[b] = (out[b] - ref) + target;
    return 0;
}
