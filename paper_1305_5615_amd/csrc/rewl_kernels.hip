// rewl_kernels.hip -- HIP kernels of replica-exchange Wang-Landau for gfx950.
//
// One round of every run of a batch is four launches on the batch's stream:
//   sweep_kernel<P,RP> one wave per group of P walkers of one run; each
//                      walker's spins, ln g and H live in LDS for the round;
//                      the walker's 64/P lanes draw 64/P attempts at a time
//                      (Philox, site, neighbours, ln u, energy change) in
//                      parallel, then all of them apply the attempts in order,
//                      identically, which keeps the sequential single-site
//                      dynamics of the standard WL walk (standard-WL
//                      paragraph); RP: where the per-step bin records live;
//   flat_merge_kernel  one work-group per window: flatness of each walker,
//                      and when all m are flat the mean of their ln g, H reset,
//                      ln f halved (parallel-scheme paragraph); under the 1/t
//                      rule ln f = W/t and the merge runs every round;
//   exchange_kernel    one work-group per window pair (k, k+1), k = round mod
//                      2: partner permutation, Eq. (1) test, configuration swap;
//   advance_kernel     each run's round counter + 1.
// The round number lives on the device, so a captured graph of rounds replays
// correctly.  The start-up step (random configuration, energy, walk into the
// window) is init_kernel.  Compiled with -ffp-contract=off (see rewl_device.h).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>

#include "rewl_device.h"
#include "rewl_internal.h"

using namespace rewl;

namespace {

// the last failed HIP call of a launcher on this thread, for error messages
thread_local char g_launch_err[256];

int launch_fail(hipError_t e, const char *what)
{
    std::snprintf(g_launch_err, sizeof g_launch_err, "%s: %s", what, hipGetErrorString(e));
    return -3;
}

int launch_status(const char *what)
{
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : launch_fail(e, what);
}

constexpr int kIsing = 0, kPotts = 1, kEA = 2, kEA3 = 3;

// neighbours of a site for the model's lattice
template <int MODEL>
__device__ __forceinline__ Nbrs nbrs_of(int i, const RunDesc &a)
{
    if (MODEL == kEA3) return neighbours3(i, a.L, a.N, a.l_magic, a.l2_magic);
    return neighbours(i, a.L, a.N, a.l_magic);
}

template <int MODEL>
struct Step {
    static constexpr int value = (MODEL == kPotts) ? 1 : 4;
};

// energy change of site `site` going from `old` to `nw`, spins in LDS
template <int MODEL>
__device__ __forceinline__ int delta_e(const int8_t *sp, const uint32_t *J4, int site,
                                       const Nbrs &nb, int old, int nw)
{
    const int rt = nb.rt, lf = nb.lf, dn = nb.dn, up = nb.up;
    if (MODEL == kIsing) {
        return 2 * old * ((int)sp[rt] + (int)sp[lf] + (int)sp[dn] + (int)sp[up]);
    } else if (MODEL == kEA3) {
        const uint2 j = reinterpret_cast<const uint2 *>(J4)[site];
        const int h = (int8_t)(j.x & 0xFF) * sp[rt] + (int8_t)((j.x >> 8) & 0xFF) * sp[lf] +
                      (int8_t)((j.x >> 16) & 0xFF) * sp[dn] + (int8_t)(j.x >> 24) * sp[up] +
                      (int8_t)(j.y & 0xFF) * sp[nb.fw] + (int8_t)((j.y >> 8) & 0xFF) * sp[nb.bk];
        return 2 * old * h;
    } else if (MODEL == kEA) {
        const uint32_t j = J4[site];
        const int jr = (int8_t)(j & 0xFF), jl = (int8_t)((j >> 8) & 0xFF);
        const int jd = (int8_t)((j >> 16) & 0xFF), ju = (int8_t)(j >> 24);
        return 2 * old * (jr * sp[rt] + jl * sp[lf] + jd * sp[dn] + ju * sp[up]);
    } else {
        const int so = (sp[rt] == old) + (sp[lf] == old) + (sp[dn] == old) + (sp[up] == old);
        const int sn = (sp[rt] == nw) + (sp[lf] == nw) + (sp[dn] == nw) + (sp[up] == nw);
        return so - sn;
    }
}

// energy of the bonds to the right and below site i (and behind it, 3D)
template <int MODEL>
__device__ __forceinline__ int bond_energy(const int8_t *sp, const uint32_t *J4, int i,
                                           const RunDesc &a)
{
    const Nbrs nb = nbrs_of<MODEL>(i, a);
    if (MODEL == kIsing) return -(sp[i] * sp[nb.rt] + sp[i] * sp[nb.dn]);
    if (MODEL == kEA3) {
        const uint2 j = reinterpret_cast<const uint2 *>(J4)[i];
        return -((int8_t)(j.x & 0xFF) * sp[i] * sp[nb.rt] +
                 (int8_t)((j.x >> 16) & 0xFF) * sp[i] * sp[nb.dn] +
                 (int8_t)(j.y & 0xFF) * sp[i] * sp[nb.fw]);
    }
    if (MODEL == kPotts) return -((sp[i] == sp[nb.rt]) + (sp[i] == sp[nb.dn]));
    const uint32_t j = J4[i];
    const int jr = (int8_t)(j & 0xFF), jd = (int8_t)((j >> 16) & 0xFF);
    return -(jr * sp[i] * sp[nb.rt] + jd * sp[i] * sp[nb.dn]);
}

// a start-up move: site, Potts offset and the neighbours (16 bits each)
struct Move {
    uint32_t site_r1, nb_rl, nb_du, nb_fb;
};

__device__ __forceinline__ int dist_to(int E, int elo, int ehi)
{
    return E < elo ? elo - E : (E > ehi ? E - ehi : 0);
}

// block-wide integer sum (256 threads)
__device__ int block_sum_256(int v, int *scratch)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) scratch[wave] = v;
    __syncthreads();
    int s = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += scratch[i];
    __syncthreads();
    return s; // valid in thread 0
}

// ------------------------------------------------------------------ start-up
// Random configuration from stream 1 (one Philox block per site, word 0),
// its energy, then single-site moves from stream 2 accepted whenever they do
// not increase the distance to the window; Ising and Potts walkers still
// outside after 200 N moves restart from the ordered state, and a walker still
// outside after 400 N moves (EA: 200 N) fails the start-up.
template <int MODEL>
__global__ __launch_bounds__(256) void init_kernel(RunDesc a)
{
    const int w = blockIdx.x, k = w / a.m, N = a.N;
    extern __shared__ __align__(16) unsigned char smem[];
    Move *stage = reinterpret_cast<Move *>(smem);
    int *scratch = reinterpret_cast<int *>(stage + kWave);   // 8 ints
    constexpr int JW = (MODEL == kEA) ? 1 : (MODEL == kEA3 ? 2 : 0);  // coupling words per site
    uint32_t *J_s = reinterpret_cast<uint32_t *>(scratch + 8);
    int8_t *sp = reinterpret_cast<int8_t *>(J_s + JW * N);
    __shared__ int sh_E, sh_stop, sh_used;

    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const U4 r = philox((uint32_t)i, 0u, (uint32_t)w, 1u, a.key0, a.key1);
        sp[i] = (MODEL == kPotts) ? (int8_t)mulhi32(r.x, (uint32_t)a.q) : ((r.x >> 31) ? 1 : -1);
    }
    for (int i = threadIdx.x; i < JW * N; i += blockDim.x) J_s[i] = a.J4[i];
    __syncthreads();
    int e = 0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) e += bond_energy<MODEL>(sp, J_s, i, a);
    e = block_sum_256(e, scratch);
    const int elo = a.e_min + a.lo[k] * a.step, ehi = a.e_min + a.hi[k] * a.step;
    if (threadIdx.x == 0) {
        sh_E = e;
        sh_stop = dist_to(e, elo, ehi) == 0;
    }
    __syncthreads();
    const unsigned long long cap = 200ull * (unsigned long long)N;
    unsigned long long d = 0;
    while (!sh_stop) {
        if (threadIdx.x < kWave) {
            const unsigned long long c = d + threadIdx.x;
            const U4 r = philox((uint32_t)c, (uint32_t)(c >> 32), (uint32_t)w, 2u, a.key0, a.key1);
            const int site = (int)mulhi32(r.x, (uint32_t)N);
            const uint32_t r1 = (MODEL == kPotts) ? 1u + mulhi32(r.y, (uint32_t)(a.q - 1)) : 0u;
            const Nbrs nb = nbrs_of<MODEL>(site, a);
            Move p;
            p.site_r1 = (uint32_t)site | (r1 << 16);
            p.nb_rl = (uint32_t)nb.rt | ((uint32_t)nb.lf << 16);
            p.nb_du = (uint32_t)nb.dn | ((uint32_t)nb.up << 16);
            p.nb_fb = (uint32_t)nb.fw | ((uint32_t)nb.bk << 16);
            stage[threadIdx.x] = p;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int E = sh_E, stop = 0, j = 0;
            for (; j < kWave; ++j) {
                if (dist_to(E, elo, ehi) == 0) { stop = 1; break; }
                const unsigned long long dd = d + j;
                if (dd == cap) {
                    if (MODEL == kEA || MODEL == kEA3) { a.status[0] = 1; stop = 1; break; }
                    const int8_t v = (MODEL == kPotts) ? 0 : 1;
                    for (int i = 0; i < N; ++i) sp[i] = v;
                    E = -2 * N;
                }
                if (dd == 2 * cap) { a.status[0] = 1; stop = 1; break; }
                const Move p = stage[j];
                const int site = (int)(p.site_r1 & 0xFFFFu);
                const int old = sp[site];
                int nw;
                if (MODEL == kPotts) {
                    nw = old + (int)(p.site_r1 >> 16);
                    if (nw >= a.q) nw -= a.q;
                } else {
                    nw = -old;
                }
                const Nbrs nb{(int)(p.nb_rl & 0xFFFFu), (int)(p.nb_rl >> 16),
                              (int)(p.nb_du & 0xFFFFu), (int)(p.nb_du >> 16),
                              (int)(p.nb_fb & 0xFFFFu), (int)(p.nb_fb >> 16)};
                const int En = E + delta_e<MODEL>(sp, J_s, site, nb, old, nw);
                if (dist_to(En, elo, ehi) <= dist_to(E, elo, ehi)) {
                    sp[site] = (int8_t)nw;
                    E = En;
                }
            }
            if (!stop && dist_to(E, elo, ehi) == 0) stop = 1;
            sh_E = E;
            sh_stop = stop;
            sh_used = j;
        }
        __syncthreads();
        d += (unsigned long long)sh_used;
    }
    int8_t *sg = a.spins + (size_t)w * a.Npad;
    for (int i = threadIdx.x; i < N; i += blockDim.x) sg[i] = sp[i];
    if (threadIdx.x == 0) a.E[w] = sh_E;
}

// ------------------------------------------------------------------- sweep
// Attempts are taken G = 64/P at a time per walker.  Lane g of a walker's
// group draws attempt t+g (Philox stream 0: site, Potts offset, u -> ln u),
// computes its energy change against the configuration at the start of the
// block, and flags it when an earlier proposal of the block hits its site or a
// neighbour (per-site masks in LDS, set with an atomic OR).  Every lane of the
// group then applies the G attempts in order, identically; an attempt whose
// site or neighbour was changed by an earlier accepted move of the block
// recomputes its energy change from the current spins, every other one uses
// the precomputed value, so the result is that of the plain sequential walk.
template <int MODEL>
__device__ __forceinline__ int new_state(int old, uint32_t r1, int q)
{
    if (MODEL == kPotts) {
        int nw = old + (int)r1;
        return nw >= q ? nw - q : nw;
    }
    return -old;
}

// G-bit masks of a block's proposals, one per site
template <int G> struct TagOf;
template <> struct TagOf<64> { using T = unsigned long long; };
template <> struct TagOf<32> { using T = uint32_t; };
template <> struct TagOf<16> { using T = uint16_t; };
template <> struct TagOf<8> { using T = uint8_t; };

__device__ __forceinline__ size_t up16(size_t x) { return (x + 15) & ~(size_t)15; }

template <int G>
__device__ __forceinline__ void tag_set(typename TagOf<G>::T *tag, int site, uint64_t bit)
{
    if constexpr (G == 64) {
        atomicOr(reinterpret_cast<unsigned long long *>(tag) + site, (unsigned long long)bit);
    } else {
        // OR into the aligned 32-bit word that holds the site's mask
        constexpr int per = 32 / G;
        uint32_t *w32 = reinterpret_cast<uint32_t *>(tag);
        atomicOr(w32 + site / per, (uint32_t)bit << (G * (site % per)));
    }
}

// bit 0 of every group of G lanes in a 64-bit lane mask
template <int G> struct kFirstLanes {
    static constexpr uint64_t value = (G == 64) ? 1ull : (kFirstLanes<2 * G>::value * ((1ull << G) + 1ull));
};
template <> struct kFirstLanes<64> { static constexpr uint64_t value = 1ull; };

__device__ __forceinline__ double pick(bool c, double a, double b) { return c ? a : b; }

// bins one move can reach (largest |dE| / energy step): Ising and the 2D glass
// 2, the 3D glass 3, Potts 4
template <int MODEL> struct kReach {
    static constexpr int value = (MODEL == kPotts) ? 4 : (MODEL == kEA3 ? 3 : 2);
};
// whether a recomputed move picks its target among preloaded bins (cheaper
// than a second LDS round trip up to 7 candidates)
template <int MODEL> struct kCandidates {
    static constexpr bool value = MODEL != kPotts;
};

// sum over the G aligned lanes of a walker group
template <int G>
__device__ __forceinline__ unsigned int group_sum(unsigned int v)
{
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// guard bins on either side of a window's ln g: the largest single-site
// energy change is 8 (Ising, +-J: 2 bins of 4) or 4 (Potts: 4 bins of 1)
constexpr int kGuard = 4;

// LDS region of one walker in a sweep work-group (the sizes of
// sweep_walker_lds): ln g with kGuard guard bins on either side, H, the staged
// proposals (G + 2), the per-step bin records, the per-site G-bit proposal
// masks, the spins.
template <int G>
struct WalkerLds {
    double *lng;                  // lng[0] is the window's first bin
    uint32_t *H;
    Prop *stage;
    uint32_t *post;
    typename TagOf<G>::T *tag;
    int8_t *sp;
};

template <int G>
__device__ __forceinline__ WalkerLds<G> walker_lds(unsigned char *mine, int max_W, int max_N)
{
    using TagT = typename TagOf<G>::T;
    WalkerLds<G> r;
    r.lng = reinterpret_cast<double *>(mine) + kGuard;
    r.H = reinterpret_cast<uint32_t *>(mine + up16((size_t)(max_W + 2 * kGuard) * 8));
    r.stage = reinterpret_cast<Prop *>(reinterpret_cast<unsigned char *>(r.H) +
                                       up16((size_t)max_W * 4));
    r.post = reinterpret_cast<uint32_t *>(r.stage + G + 2);
    r.tag = reinterpret_cast<TagT *>(reinterpret_cast<unsigned char *>(r.post) +
                                     up16((size_t)G * 4));
    r.sp = reinterpret_cast<int8_t *>(reinterpret_cast<unsigned char *>(r.tag) +
                                      up16((size_t)max_N * sizeof(TagT)));
    return r;
}

// Orders the LDS writes of a wave's lanes before the reads of other lanes of
// the same wave.  A wave's LDS instructions execute in order, so this only has
// to keep the compiler from moving accesses across it: a wave barrier, which
// the compiler treats as touching memory and which emits no instruction.  No
// memory fence, which would make the wave wait for all of its outstanding LDS
// operations; other waves of the work-group are not waited for.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_wave_barrier();
}

// HBM -> LDS: a walker's ln g (guard bins of +inf on either side: a move that
// leaves the window meets +inf and is rejected by the ordinary test), H and
// spins, and its proposal masks cleared.  The G lanes of its group share the
// copy.
template <int G>
__device__ __forceinline__ void walker_load(const RunDesc &a, const WalkerLds<G> &L, int w,
                                            int W, int gl)
{
    using TagT = typename TagOf<G>::T;
    const double *lng_g = a.lng + (size_t)w * a.Wmax;
    const uint32_t *H_g = a.H + (size_t)w * a.Wmax;
    for (int i = gl; i < W; i += G) {
        L.lng[i] = lng_g[i];
        L.H[i] = H_g[i];
    }
    if (gl < kGuard) {
        L.lng[-1 - gl] = __builtin_inf();
        L.lng[W + gl] = __builtin_inf();
    }
    const uint32_t *src = reinterpret_cast<const uint32_t *>(a.spins + (size_t)w * a.Npad);
    uint32_t *dst = reinterpret_cast<uint32_t *>(L.sp);
    for (int i = gl; i < (a.N + 3) / 4; i += G) dst[i] = src[i];
    for (int i = gl; i < a.N; i += G) L.tag[i] = (TagT)0;
}

// LDS -> HBM: the walker's ln g, H and spins
template <int G>
__device__ __forceinline__ void walker_store(const RunDesc &a, const WalkerLds<G> &L, int w,
                                             int W, int gl)
{
    double *lng_g = a.lng + (size_t)w * a.Wmax;
    uint32_t *H_g = a.H + (size_t)w * a.Wmax;
    for (int i = gl; i < W; i += G) {
        lng_g[i] = L.lng[i];
        H_g[i] = L.H[i];
    }
    const uint32_t *src = reinterpret_cast<const uint32_t *>(L.sp);
    uint32_t *dst = reinterpret_cast<uint32_t *>(a.spins + (size_t)w * a.Npad);
    for (int i = gl; i < (a.N + 3) / 4; i += G) dst[i] = src[i];
}

// LDS byte address of a pointer into the work-group's shared memory, and
// loads / stores at such an address: the in-order pass carries addresses, so
// its loads need no base added
using lds_u8 = __attribute__((address_space(3))) unsigned char;
__device__ __forceinline__ uint32_t lds_addr(const void *p)
{
    return (uint32_t)(uintptr_t)(const lds_u8 *)p;
}
__device__ __forceinline__ double lds_ld_f64(uint32_t addr)
{
    return *(const __attribute__((address_space(3))) double *)(uintptr_t)addr;
}
__device__ __forceinline__ void lds_st_f64(uint32_t addr, double v)
{
    *(__attribute__((address_space(3))) double *)(uintptr_t)addr = v;
}
__device__ __forceinline__ void lds_st_u8(uint32_t addr, unsigned char v)
{
    *(lds_u8 *)(uintptr_t)addr = v;
}

// the two proposals past the last of a block, read ahead by the in-order
// pass: zero moves
template <int G>
__device__ __forceinline__ void stage_guards(const WalkerLds<G> &L, int gl)
{
    const uint32_t sp_base = lds_addr(L.sp);
    for (int i = gl; i < 2; i += G) L.stage[G + i] = Prop{0.0, 0.0, 0, sp_base, 0u, 0u};
}

// RP: the per-step bin records (bin | accepted, for the H update at the end
// of a block) are kept in a register of the lane that drew the attempt rather
// than stored to LDS.  That costs VALU work per step and saves an LDS store;
// it measured faster when several waves share a CU's LDS and slower with one
// wave per CU, so the launcher picks it by the number of waves.
//
// S attempts of the walker of this lane's group (standard-WL paragraph), its
// state in LDS at L.  live: the walker exists and its
// window is running (a group that is not live only keeps the wave's lanes in
// step).  Returns the walker's bin after the attempts (window-local) and adds
// its accepted moves to acc.
template <int MODEL, int P, bool RP>
__device__ __forceinline__ int sweep_attempts(const RunDesc &a, const WalkerLds<kWave / P> &L,
                                              const uint32_t *J_s,
                                              int w, bool live, int W, int b0, double lnf,
                                              bool one_over_t, unsigned long long t0,
                                              unsigned int &acc)
{
    constexpr int G = kWave / P;
    using TagT = typename TagOf<G>::T;
    constexpr int STEP = Step<MODEL>::value;
    constexpr int ADDR_PER_E = 8 / STEP;   // bytes of ln g per energy unit
    const int lane = threadIdx.x & (kWave - 1), gl = lane % G;
    const int N = a.N, q = a.q;
    // a wave none of whose walkers is live has nothing to do
    if (__builtin_amdgcn_ballot_w64(live) == 0) return b0;
    double *lng_s = L.lng;
    uint32_t *H_s = L.H;
    Prop *stage = L.stage;
    uint32_t *post_s = L.post;
    TagT *tag = L.tag;
    int8_t *sp = L.sp;
    const uint32_t sp_base = lds_addr(sp);
    const uint32_t lng_base = lds_addr(lng_s);

    // the 1/t rule: ln f = W / t after each attempt, t = attempts made so far
    const double Wd = (double)W;
    const long long S = a.S;
    // chain state, identical in every lane of the group: LDS byte offset of
    // the current bin's ln g, and its value
    uint32_t baddr = lng_base + (uint32_t)b0 * 8u;
    double gcur = live ? lng_s[b0] : 0.0;
    const uint64_t bit = 1ull << gl;

    // state-independent part of an attempt: Philox draw, site, neighbours,
    // Potts offset, ln u
    struct Draw {
        int site;
        Nbrs nb;
        uint32_t r1;
        double thr;
    };
    // a draw taken in 8 pieces (five of two Philox rounds each, then site and
    // neighbours, then the two halves of ln u), so that the draws of the next
    // block can be spread over the in-order pass of this one, where they fill
    // the wait for each LDS round trip
    struct DrawSt {
        U4 c;
        uint32_t k0, k1;
        LnU lu;
        Draw out;
    };
    auto draw_start = [&](long long base) {
        DrawSt st;
        const unsigned long long c = t0 + (unsigned long long)base + gl;
        st.c = U4{(uint32_t)c, (uint32_t)(c >> 32), (uint32_t)w, 0u};
        st.k0 = a.key0;
        st.k1 = a.key1;
        return st;
    };
    auto draw_piece = [&](DrawSt &st, int piece) {
        if (piece < 5) {
            philox_rounds(st.c, st.k0, st.k1, 2 * piece, 2 * piece + 2);
        } else if (piece == 5) {
            st.out.site = (int)mulhi32(st.c.x, (uint32_t)N);
            st.out.r1 = (MODEL == kPotts) ? 1u + mulhi32(st.c.y, (uint32_t)(q - 1)) : 0u;
            st.out.nb = nbrs_of<MODEL>(st.out.site, a);
        } else if (piece == 6) {
            st.lu = ln_u_reduce(st.c.z, st.c.w);
        } else {
            st.out.thr = ln_u_sum(st.lu);
        }
    };
    auto draw = [&](long long base) {
        DrawSt st = draw_start(base);
#pragma unroll
        for (int piece = 0; piece < 8; ++piece) draw_piece(st, piece);
        return st.out;
    };
    Draw cur = draw(0);

    for (long long base = 0; base < S; base += G) {
        const int n = (S - base < G) ? (int)(S - base) : G;
        const bool active = live && gl < n;
        // earlier attempts of the block that touched this attempt's site or a
        // neighbour (one bit per lane of the group)
        uint64_t earlier = 0;
        uint32_t post = 0;
        // state-dependent part, against the configuration at the block start
        if (active) {
            const int old = sp[cur.site];
            const int nw = new_state<MODEL>(old, cur.r1, q);
            const int dE = delta_e<MODEL>(sp, J_s, cur.site, cur.nb, old, nw);
            tag_set<G>(tag, cur.site, bit);
            uint64_t seen = (uint64_t)tag[cur.site] | tag[cur.nb.rt] | tag[cur.nb.lf] |
                            tag[cur.nb.dn] | tag[cur.nb.up];
            if (MODEL == kEA3) seen |= (uint64_t)tag[cur.nb.fw] | tag[cur.nb.bk];
            Prop p;
            p.thr = cur.thr;
            p.lnf = one_over_t ? Wd / (double)(t0 + (unsigned long long)base + gl + 1) : lnf;
            p.d_addr = dE * ADDR_PER_E;
            p.sp_off = sp_base + (uint32_t)cur.site;
            p.flags = ((uint32_t)nw & 0xFFu) | (cur.r1 << 16);
            p.old = (uint32_t)old & 0xFFu;
            stage[gl] = p;
            earlier = seen & (bit - 1ull);
        } else {
            // records past the last attempt: a zero move, read ahead only
            stage[gl] = Prop{0.0, 0.0, 0, sp_base, 0u, 0u};
        }
        wave_sync();
        if (active) tag[cur.site] = (TagT)0;
        // draws of the next block: with several walkers per wave, in pieces
        // between the steps of the in-order pass below; with one, whole here.
        // Either way they do not depend on the pass, and the compiler is free
        // to place them (it gathers them after the pass; pinning the pieces
        // between the steps measured no faster)
        constexpr bool kSpread = G < 64;
        DrawSt nxt = draw_start(base + G);
        if (!kSpread) {
#pragma unroll
            for (int piece = 0; piece < 8; ++piece) draw_piece(nxt, piece);
        }
        // Attempts whose energy change must be recomputed, one bit per lane
        // (wave-uniform): those for which an earlier attempt of the block that
        // touched their site or a neighbour has been accepted.  Filled in as
        // the pass accepts moves; only those moves change spins.
        uint64_t pending = 0;
        if (live) {
            // In-order pass, executed identically by every lane of the group.
            // The only branch is taken when some group of the wave has a
            // pending attempt at this position; it is wave-uniform (a scalar
            // test of `pending`), so other positions cost no exec-mask
            // changes.  As soon as an attempt is decided the current bin's
            // ln g is written back and the ln g at the next attempt's target is
            // loaded (after the write, which a wave's in-order LDS accesses
            // make visible to it, so a target equal to the current bin needs no
            // forwarding); the spin store and the bookkeeping follow.
            struct Rec {
                double thr, lnf;
                int d;
                uint32_t sp_off, flags, old;
            };
            auto fetch = [&](int j) {
                const uint4 v = *reinterpret_cast<const uint4 *>(&stage[j]);
                const uint4 u = *reinterpret_cast<const uint4 *>(&stage[j].d_addr);
                Rec f;
                f.thr = __hiloint2double((int)v.y, (int)v.x);
                f.lnf = __hiloint2double((int)v.w, (int)v.z);
                f.d = (int)u.x;
                f.sp_off = u.y;
                f.flags = u.z;
                f.old = u.w;
                return f;
            };
            auto ld = [&](uint32_t addr) { return lds_ld_f64(addr); };
            Rec r0 = fetch(0), r1 = fetch(1);
            // ln g at the first attempt's target
            double gnx = ld(baddr + (uint32_t)r0.d);
            auto step = [&](int j) {
                const Rec r2 = fetch(j + 2);
                int d = r0.d;
                // the spin store takes the low byte of these words
                uint32_t nw = r0.flags, old = r0.old;
                double gn = gnx;
                if (__builtin_expect((pending & (kFirstLanes<G>::value << j)) != 0, 0)) {
                    // some group's attempt j is pending: every group recomputes
                    // from its current spins, the pending ones keep the result.
                    // The ln g of every bin one move can reach is loaded
                    // together with the spins (one LDS round trip, not two);
                    // with one walker per wave the neighbours come from the
                    // lane that drew the attempt.
                    const int s = (int)(r0.sp_off - sp_base);
                    Nbrs nb;
                    if (G == kWave) {
                        nb.rt = __builtin_amdgcn_readlane(cur.nb.rt, j);
                        nb.lf = __builtin_amdgcn_readlane(cur.nb.lf, j);
                        nb.dn = __builtin_amdgcn_readlane(cur.nb.dn, j);
                        nb.up = __builtin_amdgcn_readlane(cur.nb.up, j);
                        nb.fw = (MODEL == kEA3) ? __builtin_amdgcn_readlane(cur.nb.fw, j) : s;
                        nb.bk = (MODEL == kEA3) ? __builtin_amdgcn_readlane(cur.nb.bk, j) : s;
                    } else {
                        nb = nbrs_of<MODEL>(s, a);
                    }
                    constexpr int R = kReach<MODEL>::value;
                    double cand[2 * R + 1];
                    if (kCandidates<MODEL>::value) {
#pragma unroll
                        for (int c = 0; c <= 2 * R; ++c)
                            cand[c] = ld(baddr + (uint32_t)((c - R) * 8));
                    }
                    const int o2 = sp[s];
                    const int n2 = new_state<MODEL>(o2, (r0.flags >> 16) & 0x7Fu, q);
                    const uint32_t o2w = (uint32_t)o2 & 0xFFu, n2w = (uint32_t)n2 & 0xFFu;
                    const int d2 = delta_e<MODEL>(sp, J_s, s, nb, o2, n2) * ADDR_PER_E;
                    double g2;
                    if (kCandidates<MODEL>::value) {
                        g2 = cand[0];
#pragma unroll
                        for (int c = 1; c <= 2 * R; ++c) g2 = pick(d2 == (c - R) * 8, cand[c], g2);
                    } else {
                        g2 = ld(baddr + (uint32_t)d2);
                    }
                    const bool f = ((pending >> ((lane & ~(G - 1)) + j)) & 1ull) != 0;
                    old = f ? o2w : old;
                    nw = f ? n2w : nw;
                    d = f ? d2 : d;
                    gn = pick(f, g2, gn);
                }
                // outside the window the target holds +inf: gcur - gn = -inf
                // never exceeds ln u, so the move is rejected
                const bool accept = gcur - gn > r0.thr;
                // an accepted move makes the later attempts that touch its site
                // or a neighbour pending (their lanes' `earlier` has bit j)
                pending |= __builtin_amdgcn_ballot_w64(((earlier >> j) & 1ull) != 0) &
                           __builtin_amdgcn_ballot_w64(accept);
                baddr = accept ? baddr + (uint32_t)d : baddr;
                const double gsel = pick(accept, gn, gcur);
                gcur = gsel + r0.lnf;
                lds_st_f64(baddr, gcur);
                gnx = ld(baddr + (uint32_t)r1.d);
                lds_st_u8(r0.sp_off, (unsigned char)(accept ? nw : old));
                // bin after attempt j and its acceptance, for lane j's H update
                if constexpr (RP)
                    post = (gl == j) ? (baddr | (accept ? 1u : 0u)) : post;
                else
                    post_s[j] = baddr | (accept ? 1u : 0u);
                r0 = r1;
                r1 = r2;
            };
            if (n == G) {
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    step(j);
                    // pieces ceil(8j/G) .. ceil(8(j+1)/G)-1 of the next draws
                    if (kSpread) {
#pragma unroll
                        for (int piece = (8 * j + G - 1) / G; piece < (8 * (j + 1) + G - 1) / G;
                             ++piece)
                            draw_piece(nxt, piece);
                    }
                }
            } else {
                for (int j = 0; j < n; ++j) step(j);
            }
        }
        // H of the block's attempts, one atomic per lane
        if (active) {
            const uint32_t v = RP ? post : post_s[gl];
            atomicAdd(&H_s[((v & ~7u) - lng_base) >> 3], 1u);
            acc += v & 1u;
        }
        // (a block shorter than G is the last one: its next draws are unused)
        cur = nxt.out;
        wave_sync();
    }
    return (int)((baddr - lng_base) >> 3);
}

// One round's sweep of one wave of a launch (a group of P walkers of one run):
// load the walkers' state into LDS, S attempts each, store it back.
template <int MODEL, int P, bool RP>
__device__ __forceinline__ void sweep_body(const RunDesc &a, const SweepItem &it,
                                           const BatchDev &bd, unsigned char *smem)
{
    constexpr int G = kWave / P;
    constexpr int STEP = Step<MODEL>::value;
    const int lane = threadIdx.x, grp = lane / G, gl = lane % G;
    const int N = a.N;
    const int w = it.w0 + grp;
    const int k = w / a.m;
    // a walker group is live when it exists and its window is still running
    const bool live = grp < it.count && !a.done[k];
    const WalkerLds<G> L = walker_lds<G>(smem + (size_t)grp * bd.region, bd.max_W, bd.max_N);
    uint32_t *J_s = reinterpret_cast<uint32_t *>(smem + (size_t)P * bd.region);
    const int lo = live ? a.lo[k] : 0;
    const int W = live ? a.hi[k] - lo + 1 : 1;
    if (live) walker_load<G>(a, L, w, W, gl);
    stage_guards<G>(L, gl);
    constexpr int JW = (MODEL == kEA) ? 1 : (MODEL == kEA3 ? 2 : 0);  // coupling words per site
    for (int i = lane; i < JW * N; i += kWave) J_s[i] = a.J4[i];
    __syncthreads();

    const int elo = a.e_min + lo * STEP;
    const double lnf = live ? a.lnf[k] : 0.0;
    const bool one_over_t = live && a.phase[k] != 0;
    const unsigned long long t0 = live ? a.t[w] : 0ull;
    const int b0 = live ? (a.E[w] - elo) / STEP : 0;
    unsigned int acc = 0;
    const int b = sweep_attempts<MODEL, P, RP>(a, L, J_s, w, live, W, b0, lnf, one_over_t, t0, acc);
    if (live) {
        walker_store<G>(a, L, w, W, gl);
        const unsigned int acc_w = group_sum<G>(acc);
        if (gl == 0) {
            a.E[w] = elo + b * STEP;
            a.t[w] = t0 + (unsigned long long)a.S;
            a.n_acc[w] += acc_w;
        }
    }
}

template <int P, bool RP>
__global__ __launch_bounds__(kWave) void sweep_kernel(BatchDev bd)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const SweepItem it = bd.sweep[blockIdx.x];
    const RunDesc a = bd.runs[it.run];
    switch (a.model) {
    case kIsing: sweep_body<kIsing, P, RP>(a, it, bd, smem); break;
    case kPotts: sweep_body<kPotts, P, RP>(a, it, bd, smem); break;
    case kEA: sweep_body<kEA, P, RP>(a, it, bd, smem); break;
    default: sweep_body<kEA3, P, RP>(a, it, bd, smem); break;
    }
}

// ------------------------------------------------------- flatness + merge
// flat <=> min H * n >= p * sum H over the walker's visited bins (lng > 0);
// when all m walkers of the window are flat: ln g <- (sum_s ln g_s) / m summed
// s = 0..m-1 in order, H <- 0, flags cleared, ln f halved, done below lnf_final.
__global__ __launch_bounds__(256) void flat_merge_kernel(BatchDev bd)
{
    const WinItem it = bd.win[blockIdx.x];
    const RunDesc &a = bd.runs[it.run];
    const int k = it.k;
    if (a.done[k]) return;
    const long long round = *a.round;
    const int lo = a.lo[k], W = a.hi[k] - lo + 1, m = a.m;
    __shared__ unsigned long long sh_sum[4];
    __shared__ unsigned int sh_min[4], sh_n[4];
    __shared__ int sh_all;
    const int tid = threadIdx.x, wave = tid >> 6;
    const bool one_over_t = a.phase[k] != 0;  // no flatness test: merge every round
    for (int s = 0; s < m && !one_over_t; ++s) {
        const int w = k * m + s;
        if (a.flat[w]) continue;
        const double *g = a.lng + (size_t)w * a.Wmax;
        const uint32_t *H = a.H + (size_t)w * a.Wmax;
        unsigned long long sum = 0;
        unsigned int hmin = 0xFFFFFFFFu, n = 0;
        for (int i = tid; i < W; i += blockDim.x) {
            if (g[i] > 0.0) {
                const uint32_t h = H[i];
                sum += h;
                n += 1;
                hmin = h < hmin ? h : hmin;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            sum += __shfl_xor(sum, off);
            n += __shfl_xor(n, off);
            const unsigned int o = __shfl_xor(hmin, off);
            hmin = o < hmin ? o : hmin;
        }
        if ((tid & 63) == 0) {
            sh_sum[wave] = sum;
            sh_min[wave] = hmin;
            sh_n[wave] = n;
        }
        __syncthreads();
        if (tid == 0) {
            for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
                sum += sh_sum[i];
                n += sh_n[i];
                hmin = sh_min[i] < hmin ? sh_min[i] : hmin;
            }
            const int f = (n > 0) && ((double)hmin * (double)n >= a.flat_p * (double)sum);
            a.flat[w] = f;
        }
        __syncthreads();
    }
    if (tid == 0) {
        int all = 1;
        for (int s = 0; s < m; ++s) all &= (a.flat[k * m + s] != 0);
        sh_all = all || one_over_t;
    }
    __syncthreads();
    if (!sh_all) return;
    const bool pow2 = (m & (m - 1)) == 0;
    const double inv = 1.0 / (double)m;
    for (int i = tid; i < W; i += blockDim.x) {
        double sum = 0.0;
        for (int s = 0; s < m; ++s) sum = sum + a.lng[(size_t)(k * m + s) * a.Wmax + i];
        const double mean = pow2 ? sum * inv : sum / (double)m;
        for (int s = 0; s < m; ++s) {
            a.lng[(size_t)(k * m + s) * a.Wmax + i] = mean;
            a.H[(size_t)(k * m + s) * a.Wmax + i] = 0u;
        }
    }
    if (tid == 0) {
        for (int s = 0; s < m; ++s) a.flat[k * m + s] = 0;
        if (a.first[k] < 0) a.first[k] = round;
        const double Wt = (double)W / (double)a.t[k * m];  // the window's walkers share t
        double nl;
        if (one_over_t) {
            nl = Wt;
        } else {
            nl = a.lnf[k] * 0.5;
            if (a.schedule == 1 && nl < Wt) {
                a.phase[k] = 1;
                nl = Wt;
            }
        }
        a.lnf[k] = nl;
        if (nl < a.lnf_final) {
            a.done[k] = 1;
            a.finish[k] = round;
        }
    }
}

// -------------------------------------------------------------- exchange
// Stream-3 words of pair (k, k+1) in round r come from counters
// (r_lo, r_hi, k, 3 | call << 8): first m-1 words for a Fisher-Yates shuffle
// pi of the slots of window k+1 (a = m-1 .. 1 swaps pi[a], pi[mulhi(word, a+1)]),
// then two words per slot a for u.  Walker a of window k (configuration X)
// and walker pi[a] of window k+1 (configuration Y) swap configurations iff
// both energies lie in both windows and
// ln u < [ln g_i(E_X) - ln g_i(E_Y)] + [ln g_j(E_Y) - ln g_j(E_X)]   (Eq. (1)).
// One thread decides the pair.  get_E(w) / set_E(w, E): walker w's energy;
// lng_at(w, b): walker w's ln g at window-local bin b; swapped(wi, wj): the
// configurations of the two walkers are to be exchanged.  perm: m ints.
// Returns the accepted swaps (the pair made m proposals).
template <class GetE, class SetE, class LngAt, class Swapped>
__device__ unsigned long long exchange_pair(const RunDesc &a, int k, long long round, int *perm,
                                            GetE get_E, SetE set_E, LngAt lng_at,
                                            Swapped swapped)
{
    const int m = a.m;
    uint32_t buf[4] = {0, 0, 0, 0};
    uint32_t call = 0;
    int idx = 4;
    auto next = [&]() -> uint32_t {
        if (idx == 4) {
            const U4 r = philox((uint32_t)round, (uint32_t)((unsigned long long)round >> 32),
                                (uint32_t)k, 3u | (call << 8), a.key0, a.key1);
            buf[0] = r.x; buf[1] = r.y; buf[2] = r.z; buf[3] = r.w;
            call += 1;
            idx = 0;
        }
        return buf[idx++];
    };
    for (int s = 0; s < m; ++s) perm[s] = s;
    for (int s = m - 1; s >= 1; --s) {
        const int j = (int)mulhi32(next(), (uint32_t)(s + 1));
        const int x = perm[s];
        perm[s] = perm[j];
        perm[j] = x;
    }
    const int lo_i = a.lo[k], hi_i = a.hi[k], lo_j = a.lo[k + 1], hi_j = a.hi[k + 1];
    unsigned long long acc = 0;
    for (int s = 0; s < m; ++s) {
        const uint32_t hi = next();
        const uint32_t lo = next();
        const double thr = ln_u(hi, lo);
        const int wi = k * m + s, wj = (k + 1) * m + perm[s];
        const int EX = get_E(wi), EY = get_E(wj);
        const int bX = (EX - a.e_min) / a.step, bY = (EY - a.e_min) / a.step;
        if (bX < lo_j || bX > hi_j || bY < lo_i || bY > hi_i) continue;
        const double lnP = (lng_at(wi, bX - lo_i) - lng_at(wi, bY - lo_i)) +
                           (lng_at(wj, bY - lo_j) - lng_at(wj, bX - lo_j));
        if (thr < lnP) {
            set_E(wi, EY);
            set_E(wj, EX);
            swapped(wi, wj);
            ++acc;
        }
    }
    return acc;
}

// One work-group per window-pair slot: thread 0 decides, all threads swap
// the accepted configurations in HBM.
__global__ __launch_bounds__(256) void exchange_kernel(BatchDev bd)
{
    const WinItem it = bd.pair[blockIdx.x];
    const RunDesc &a = bd.runs[it.run];
    const long long round = *a.round;
    const int k = 2 * it.k + (int)(round & 1);
    if (k + 1 >= a.h) return;
    if (a.done[k] || a.done[k + 1]) return;
    __shared__ int sh_n, sh_wi[64], sh_wj[64], perm[64];
    if (threadIdx.x == 0) {
        int n = 0;
        const unsigned long long acc = exchange_pair(
            a, k, round, perm, [&](int w) { return a.E[w]; },
            [&](int w, int E) { a.E[w] = E; },
            [&](int w, int b) { return a.lng[(size_t)w * a.Wmax + b]; },
            [&](int wi, int wj) {
                sh_wi[n] = wi;
                sh_wj[n] = wj;
                ++n;
            });
        a.ex_prop[k] += (unsigned long long)a.m;
        a.ex_acc[k] += acc;
        sh_n = n;
    }
    __syncthreads();
    const int words = a.Npad / 4;
    for (int p = 0; p < sh_n; ++p) {
        uint32_t *x = reinterpret_cast<uint32_t *>(a.spins + (size_t)sh_wi[p] * a.Npad);
        uint32_t *y = reinterpret_cast<uint32_t *>(a.spins + (size_t)sh_wj[p] * a.Npad);
        for (int i = threadIdx.x; i < words; i += blockDim.x) {
            const uint32_t v = x[i];
            x[i] = y[i];
            y[i] = v;
        }
    }
}

// --------------------------------------------------------- persistent form
// One work-group per run, for runs whose walkers all fit one work-group: the
// whole run stays in LDS for `rounds` rounds (sweep, flatness, merges,
// exchange, each a work-group step between barriers), the hierarchy of the
// parallel-scheme paragraph (h windows x m walkers) held by one CU.  Wave v
// sweeps walkers vP .. vP+P-1 exactly as sweep_kernel does; walker w's LDS
// region is the w-th of the work-group.  The results are those of the same
// rounds launched kernel by kernel.
template <int MODEL, int P, bool RP>
__device__ __forceinline__ void persist_body(const RunDesc &a, const BatchDev &bd,
                                             unsigned char *smem, long long rounds,
                                             PersistShared &ps)
{
    constexpr int G = kWave / P;
    constexpr int STEP = Step<MODEL>::value;
    const int tid = threadIdx.x, nthr = blockDim.x, wave = tid / kWave, lane = tid % kWave;
    const int grp = lane / G, gl = lane % G;
    const int N = a.N, m = a.m, h = a.h, nw = a.nw;
    const size_t region = (size_t)bd.region;
    const int w = wave * P + grp;
    const bool exists = w < nw;
    const int k = exists ? w / m : 0;
    unsigned char *wbase = smem + (size_t)wave * P * region;
    const WalkerLds<G> L = walker_lds<G>(wbase + (size_t)grp * region, bd.max_W, bd.max_N);
    uint32_t *J_s = reinterpret_cast<uint32_t *>(smem + (size_t)(nthr / kWave) * P * region);
    auto lng_of = [&](int v) { return walker_lds<G>(smem + (size_t)v * region, bd.max_W, bd.max_N); };
    const int lo = exists ? a.lo[k] : 0;
    const int W = exists ? a.hi[k] - lo + 1 : 1;
    const int elo = a.e_min + lo * STEP;

    if (exists) walker_load<G>(a, L, w, W, gl);
    stage_guards<G>(L, gl);
    constexpr int JW = (MODEL == kEA) ? 1 : (MODEL == kEA3 ? 2 : 0);
    for (int i = tid; i < JW * N; i += nthr) J_s[i] = a.J4[i];
    for (int i = tid; i < nw; i += nthr) {
        ps.E[i] = a.E[i];
        ps.flat[i] = a.flat[i];
        ps.t[i] = a.t[i];
    }
    for (int i = tid; i < h; i += nthr) {
        ps.lnf[i] = a.lnf[i];
        ps.done[i] = a.done[i];
        ps.phase[i] = a.phase[i];
        ps.first[i] = a.first[i];
        ps.finish[i] = a.finish[i];
        ps.ex_prop[i] = a.ex_prop[i];
        ps.ex_acc[i] = a.ex_acc[i];
    }
    if (tid == 0) ps.n_swap = 0;
    // from here to the write-back every access is to LDS: no device-memory
    // operation stays in flight across the rounds' waits on LDS loads
    __syncthreads();

    const long long round0 = *a.round;
    const bool pow2 = (m & (m - 1)) == 0;
    const double inv = 1.0 / (double)m;
    unsigned int acc_all = 0;
    for (long long r = 0; r < rounds; ++r) {
        // a finished run changes no more (its round counter still advances)
        if (tid == 0) {
            int all = 1;
            for (int kk = 0; kk < h; ++kk) all &= (ps.done[kk] != 0);
            ps.all_done = all;
        }
        __syncthreads();
        if (ps.all_done) break;
        const long long round = round0 + r;

        // (1) sweep: S attempts by every walker of an unfinished window
        {
            const bool live = exists && !ps.done[k];
            const unsigned long long t0 = exists ? ps.t[w] : 0ull;
            const int b0 = exists ? (ps.E[w] - elo) / STEP : 0;
            unsigned int acc = 0;
            const int b = sweep_attempts<MODEL, P, RP>(a, L, J_s, w, live, W, b0,
                                                       live ? ps.lnf[k] : 0.0,
                                                       live && ps.phase[k] != 0, t0, acc);
            acc_all += acc;
            if (live && gl == 0) {
                ps.E[w] = elo + b * STEP;
                ps.t[w] = t0 + (unsigned long long)a.S;
            }
        }
        __syncthreads();

        // (2) flatness of each walker of a running window on the halving rule
        // that is not flat yet: min H * n >= p * sum H over its visited bins
        if (exists && !ps.done[k] && !ps.phase[k] && !ps.flat[w]) {
            unsigned long long sum = 0;
            unsigned int hmin = 0xFFFFFFFFu, n = 0;
            for (int i = gl; i < W; i += G) {
                if (L.lng[i] > 0.0) {
                    const uint32_t hv = L.H[i];
                    sum += hv;
                    n += 1;
                    hmin = hv < hmin ? hv : hmin;
                }
            }
            for (int off = G / 2; off > 0; off >>= 1) {
                sum += __shfl_xor(sum, off);
                n += __shfl_xor(n, off);
                const unsigned int o = __shfl_xor(hmin, off);
                hmin = o < hmin ? o : hmin;
            }
            if (gl == 0)
                ps.flat[w] = (n > 0) && ((double)hmin * (double)n >= a.flat_p * (double)sum);
        }
        __syncthreads();

        // (3) schedule of each window whose m walkers are all flat (or that
        // follows the 1/t rule): flags cleared, ln f halved (or W/t), done
        // below ln f_final
        if (tid < h) {
            const int kk = tid;
            int mg = 0;
            if (!ps.done[kk]) {
                int all = 1;
                for (int s = 0; s < m; ++s) all &= (ps.flat[kk * m + s] != 0);
                if (all || ps.phase[kk]) {
                    mg = 1;
                    for (int s = 0; s < m; ++s) ps.flat[kk * m + s] = 0;
                    if (ps.first[kk] < 0) ps.first[kk] = round;
                    const int Wk = a.hi[kk] - a.lo[kk] + 1;
                    const double Wt = (double)Wk / (double)ps.t[kk * m];
                    double nl;
                    if (ps.phase[kk]) {
                        nl = Wt;
                    } else {
                        nl = ps.lnf[kk] * 0.5;
                        if (a.schedule == 1 && nl < Wt) {
                            ps.phase[kk] = 1;
                            nl = Wt;
                        }
                    }
                    ps.lnf[kk] = nl;
                    if (nl < a.lnf_final) {
                        ps.done[kk] = 1;
                        ps.finish[kk] = round;
                    }
                }
            }
            ps.merge[kk] = mg;
        }
        __syncthreads();

        // (4) merge: every walker of the window gets the mean of their ln g
        // (summed in slot order), H <- 0
        for (int kk = 0; kk < h; ++kk) {
            if (!ps.merge[kk]) continue;
            const int Wk = a.hi[kk] - a.lo[kk] + 1;
            for (int i = tid; i < Wk; i += nthr) {
                double sum = 0.0;
                for (int s = 0; s < m; ++s) sum = sum + lng_of(kk * m + s).lng[i];
                const double mean = pow2 ? sum * inv : sum / (double)m;
                for (int s = 0; s < m; ++s) {
                    const WalkerLds<G> v = lng_of(kk * m + s);
                    v.lng[i] = mean;
                    v.H[i] = 0u;
                }
            }
        }
        __syncthreads();

        // (5) exchange between windows (kk, kk+1), kk = round mod 2 + 2 slot
        if (tid < h / 2) {
            const int kk = 2 * tid + (int)(round & 1);
            if (kk + 1 < h && !ps.done[kk] && !ps.done[kk + 1]) {
                const unsigned long long acc = exchange_pair(
                    a, kk, round, ps.perm + tid * m, [&](int v) { return ps.E[v]; },
                    [&](int v, int E) { ps.E[v] = E; },
                    [&](int v, int b) { return lng_of(v).lng[b]; },
                    [&](int wi, int wj) {
                        const int at = atomicAdd(&ps.n_swap, 1);
                        ps.sw_i[at] = wi;
                        ps.sw_j[at] = wj;
                    });
                ps.ex_prop[kk] += (unsigned long long)m;
                ps.ex_acc[kk] += acc;
            }
        }
        __syncthreads();
        // (6) the accepted configuration swaps (disjoint pairs of walkers)
        const int nsw = ps.n_swap;
        const int words = (N + 3) / 4;
        for (int p = 0; p < nsw; ++p) {
            uint32_t *x = reinterpret_cast<uint32_t *>(lng_of(ps.sw_i[p]).sp);
            uint32_t *y = reinterpret_cast<uint32_t *>(lng_of(ps.sw_j[p]).sp);
            for (int i = tid; i < words; i += nthr) {
                const uint32_t v = x[i];
                x[i] = y[i];
                y[i] = v;
            }
        }
        __syncthreads();
        if (tid == 0) ps.n_swap = 0;
    }
    __syncthreads();

    // LDS -> HBM
    if (exists) {
        walker_store<G>(a, L, w, W, gl);
        const unsigned int acc_w = group_sum<G>(acc_all);
        if (gl == 0) a.n_acc[w] += acc_w;
    }
    for (int i = tid; i < nw; i += nthr) {
        a.E[i] = ps.E[i];
        a.flat[i] = ps.flat[i];
        a.t[i] = ps.t[i];
    }
    for (int i = tid; i < h; i += nthr) {
        a.lnf[i] = ps.lnf[i];
        a.done[i] = ps.done[i];
        a.phase[i] = ps.phase[i];
        a.first[i] = ps.first[i];
        a.finish[i] = ps.finish[i];
        a.ex_prop[i] = ps.ex_prop[i];
        a.ex_acc[i] = ps.ex_acc[i];
    }
    if (tid == 0) *a.round = round0 + rounds;
}

template <int P, bool RP>
__global__ __launch_bounds__(kWave * kPersistMaxWaves) void persist_kernel(BatchDev bd,
                                                                           long long rounds)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ PersistShared ps;
    const RunDesc a = bd.runs[blockIdx.x];
    switch (a.model) {
    case kIsing: persist_body<kIsing, P, RP>(a, bd, smem, rounds, ps); break;
    case kPotts: persist_body<kPotts, P, RP>(a, bd, smem, rounds, ps); break;
    case kEA: persist_body<kEA, P, RP>(a, bd, smem, rounds, ps); break;
    default: persist_body<kEA3, P, RP>(a, bd, smem, rounds, ps); break;
    }
}

// ----------------------------------------------- allocation-free entry point
// The static device array behind rewl_run_noalloc.  Host code never passes its
// name to a kernel (in host code the name is not a device address): it looks
// the address up with hipGetSymbolAddress once per device and uses that.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

// Set-up of an allocation-free run: grid-stride loops over the caller's ln g
// and H arrays (zero) and the run's bookkeeping in the scratch; block 0 also
// writes the launch tables and packs the couplings (EA: right, left, down, up
// per site; EA3: +x, -x, +y, -y | +z, -z, one int8 each).
__global__ __launch_bounds__(256) void noalloc_setup_kernel(NoAllocSetup s)
{
    const RunDesc &a = s.d;
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nthr = (size_t)gridDim.x * blockDim.x;
    const size_t cells = (size_t)a.nw * (size_t)a.Wmax;
    for (size_t i = tid; i < cells; i += nthr) {
        a.lng[i] = 0.0;
        a.H[i] = 0u;
    }
    for (size_t w = tid; w < (size_t)a.nw; w += nthr) {
        a.t[w] = 0ull;
        a.flat[w] = 0;
        a.n_acc[w] = 0ull;
        s.sweep[w] = SweepItem{0, (int)w, 1, 0};
    }
    for (size_t k = tid; k < (size_t)a.h; k += nthr) {
        a.lnf[k] = s.lnf_init;
        a.done[k] = 0;
        a.phase[k] = 0;
        a.finish[k] = -1;
        a.first[k] = -1;
        a.lo[k] = s.lo[k];
        a.hi[k] = s.hi[k];
        a.ex_prop[k] = 0ull;
        a.ex_acc[k] = 0ull;
        s.win[k] = WinItem{0, (int)k};
        if ((int)k < a.h / 2) s.pair[k] = WinItem{0, (int)k};
    }
    const int L = a.L, N = a.N;
    const uint8_t *J = reinterpret_cast<const uint8_t *>(s.J_raw);
    if (a.model == kEA) {
        for (size_t i = tid; i < (size_t)N; i += nthr) {
            const int ii = (int)i, r = ii / L, c = ii % L;
            const int lf = r * L + (c + L - 1) % L, up = ((r + L - 1) % L) * L + c;
            a.J4[i] = (uint32_t)J[2 * ii] | ((uint32_t)J[2 * lf] << 8) |
                      ((uint32_t)J[2 * ii + 1] << 16) | ((uint32_t)J[2 * up + 1] << 24);
        }
    } else if (a.model == kEA3) {
        const int L2 = L * L;
        for (size_t i = tid; i < (size_t)N; i += nthr) {
            const int ii = (int)i, x = ii % L, y = (ii / L) % L, z = ii / L2;
            const int xm = ii - x + (x + L - 1) % L;
            const int ym = z * L2 + ((y + L - 1) % L) * L + x;
            const int zm = ((z + L - 1) % L) * L2 + y * L + x;
            a.J4[2 * i] = (uint32_t)J[3 * ii] | ((uint32_t)J[3 * xm] << 8) |
                          ((uint32_t)J[3 * ii + 1] << 16) | ((uint32_t)J[3 * ym + 1] << 24);
            a.J4[2 * i + 1] = (uint32_t)J[3 * ii + 2] | ((uint32_t)J[3 * zm + 2] << 8);
        }
    }
    if (tid == 0) {
        s.desc[0] = a;
        *a.round = 0;
        *a.status = 0;
    }
}

// per run: 1 when every window is done
__global__ void status_kernel(BatchDev bd, int *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= bd.n_runs) return;
    const RunDesc &a = bd.runs[i];
    int all = 1;
    for (int k = 0; k < a.h; ++k) all &= (a.done[k] != 0);
    out[i] = all;
}

// every run's round counter + 1 (the oracle counts rounds of finished runs too)
__global__ void advance_kernel(BatchDev bd)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < bd.n_runs) *bd.runs[i].round += 1;
}

__global__ void selftest_philox_kernel(const uint32_t *ctr, uint32_t k0, uint32_t k1,
                                       uint32_t *out, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const U4 r = philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
    out[4 * i] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

__global__ void selftest_ln_u_kernel(const uint32_t *words, double *out, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = ln_u(words[2 * i], words[2 * i + 1]);
}

template <int MODEL>
int launch_init_t(const RunDesc &a, hipStream_t s)
{
    const size_t lds = kWave * sizeof(Move) + 8 * sizeof(int) +
                       (size_t)model_j_words(MODEL) * 4 * (size_t)a.N + (size_t)a.N + 16;
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&init_kernel<MODEL>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return launch_fail(e, "hipFuncSetAttribute(init_kernel)");
    }
    hipLaunchKernelGGL(init_kernel<MODEL>, dim3(a.nw), dim3(256), lds, s, a);
    return launch_status("init_kernel launch");
}

template <int P, bool RP>
int launch_sweep_rp(const BatchDev &b, hipStream_t s, size_t lds)
{
    // the LDS limit is raised once per device the kernel runs on
    static std::atomic<bool> attr_set[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -3;
    if (!attr_set[dev].load()) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&sweep_kernel<P, RP>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)kMaxLds);
        if (e != hipSuccess) return launch_fail(e, "hipFuncSetAttribute(sweep_kernel)");
        attr_set[dev].store(true);
    }
    hipLaunchKernelGGL((sweep_kernel<P, RP>), dim3(b.n_sweep), dim3(kWave), lds, s, b);
    return 0;
}

// compute units of the current device (cached per device)
int device_cus()
{
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cus[dev].load() == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cus[dev].store(n);
    }
    return cus[dev].load();
}

template <int P>
int launch_sweep_t(const BatchDev &b, hipStream_t s, size_t lds)
{
    // more waves than compute units: several waves share each LDS
    if (b.n_sweep > device_cus()) return launch_sweep_rp<P, true>(b, s, lds);
    return launch_sweep_rp<P, false>(b, s, lds);
}

template <int P, bool RP>
int launch_persist_rp(const BatchDev &b, hipStream_t s, size_t lds, long long rounds)
{
    static std::atomic<bool> attr_set[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -3;
    if (!attr_set[dev].load()) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&persist_kernel<P, RP>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)kPersistMaxDynLds);
        if (e != hipSuccess) return launch_fail(e, "hipFuncSetAttribute(persist_kernel)");
        attr_set[dev].store(true);
    }
    hipLaunchKernelGGL((persist_kernel<P, RP>), dim3(b.n_runs), dim3(kWave * b.pwaves), lds, s, b,
                       rounds);
    return 0;
}

template <int P>
int launch_persist_t(const BatchDev &b, hipStream_t s, size_t lds, long long rounds)
{
    // as for the sweep: several waves per CU keep the bin records in registers
    if ((long long)b.n_runs * b.pwaves > device_cus())
        return launch_persist_rp<P, true>(b, s, lds, rounds);
    return launch_persist_rp<P, false>(b, s, lds, rounds);
}

}  // namespace

int rewl_launch_persist(const BatchDev &b, long long rounds, void *stream, void *ev0, void *ev1)
{
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0 = reinterpret_cast<hipEvent_t>(ev0), e1 = reinterpret_cast<hipEvent_t>(ev1);
    if (b.n_runs <= 0 || rounds <= 0) return 0;
    if (b.pwaves < 1 || b.pwaves > kPersistMaxWaves) return -1;
    const size_t lds = persist_lds_bytes(b.P, b.pwaves, b.max_W, b.max_N, b.j_words);
    if (lds > kPersistMaxDynLds) return -1;
    if (e0 && hipEventRecord(e0, s) != hipSuccess) return -3;
    int rc;
    switch (b.P) {
    case 1: rc = launch_persist_t<1>(b, s, lds, rounds); break;
    case 2: rc = launch_persist_t<2>(b, s, lds, rounds); break;
    case 4: rc = launch_persist_t<4>(b, s, lds, rounds); break;
    case 8: rc = launch_persist_t<8>(b, s, lds, rounds); break;
    default: return -1;
    }
    if (rc) return rc;
    if (e1 && hipEventRecord(e1, s) != hipSuccess) return -3;
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

const char *rewl_launch_error(void) { return g_launch_err; }

int rewl_noalloc_scratch(void **ptr)
{
    static std::atomic<void *> addr[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -3;
    void *p = addr[dev].load();
    if (!p) {
        // with this device current: the array's address on this device
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return launch_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return -3;
        addr[dev].store(p);
    }
    *ptr = p;
    return 0;
}

int rewl_launch_noalloc_setup(const NoAllocSetup &s, void *stream)
{
    hipLaunchKernelGGL(noalloc_setup_kernel, dim3(64), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), s);
    return launch_status("noalloc_setup_kernel launch");
}

int rewl_launch_init(const RunDesc &a, void *stream)
{
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    switch (a.model) {
    case kIsing: return launch_init_t<kIsing>(a, s);
    case kPotts: return launch_init_t<kPotts>(a, s);
    case kEA: return launch_init_t<kEA>(a, s);
    default: return launch_init_t<kEA3>(a, s);
    }
}

int rewl_launch_round(const BatchDev &b, void *stream, void *ev0, void *ev1)
{
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0 = reinterpret_cast<hipEvent_t>(ev0), e1 = reinterpret_cast<hipEvent_t>(ev1);
    const size_t lds = sweep_lds_bytes(b.P, b.max_W, b.max_N, b.j_words);
    if (lds > kMaxLds) return -1;
    if (e0 && hipEventRecord(e0, s) != hipSuccess) return -3;
    if (b.n_sweep > 0) {
        int rc;
        switch (b.P) {
        case 1: rc = launch_sweep_t<1>(b, s, lds); break;
        case 2: rc = launch_sweep_t<2>(b, s, lds); break;
        case 4: rc = launch_sweep_t<4>(b, s, lds); break;
        case 8: rc = launch_sweep_t<8>(b, s, lds); break;
        default: return -1;
        }
        if (rc) return rc;
    }
    if (e1 && hipEventRecord(e1, s) != hipSuccess) return -3;
    if (b.n_win > 0) hipLaunchKernelGGL(flat_merge_kernel, dim3(b.n_win), dim3(256), 0, s, b);
    if (b.n_pair > 0) hipLaunchKernelGGL(exchange_kernel, dim3(b.n_pair), dim3(256), 0, s, b);
    if (b.n_runs > 0)
        hipLaunchKernelGGL(advance_kernel, dim3((b.n_runs + 255) / 256), dim3(256), 0, s, b);
    return launch_status("round launches");
}

int rewl_launch_status(const BatchDev &b, int *out_d, void *stream)
{
    if (b.n_runs <= 0) return 0;
    hipLaunchKernelGGL(status_kernel, dim3((b.n_runs + 255) / 256), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), b, out_d);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int rewl_launch_selftest_philox(const uint32_t *ctr_d, uint32_t k0, uint32_t k1, uint32_t *out_d,
                                int n)
{
    hipLaunchKernelGGL(selftest_philox_kernel, dim3((n + 255) / 256), dim3(256), 0, 0, ctr_d, k0,
                       k1, out_d, n);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int rewl_launch_selftest_ln_u(const uint32_t *words_d, double *out_d, int n)
{
    hipLaunchKernelGGL(selftest_ln_u_kernel, dim3((n + 255) / 256), dim3(256), 0, 0, words_d,
                       out_d, n);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
