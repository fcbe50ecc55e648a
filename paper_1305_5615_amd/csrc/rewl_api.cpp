// rewl_api.cpp -- host runtime and C ABI of the REWL library (include/rewl.h).
//
// The host validates parameters, lays the energy range out in windows,
// carves one device allocation into the run's arrays, queues the kernels of
// rewl_kernels.hip on the run's stream and, at the end, joins the window pieces
// of ln g.  It never computes a Monte Carlo step itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "rewl.h"
#include "rewl_internal.h"

namespace {

// the calling thread's last error message (a fixed buffer: setting it never
// allocates)
thread_local char g_err[512];

int fail(int code, const char *msg)
{
    std::snprintf(g_err, sizeof g_err, "%s", msg);
    return code;
}

int fail(int code, const std::string &msg) { return fail(code, msg.c_str()); }

int hip_fail(hipError_t e, const char *what)
{
    std::snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
    return REWL_EDEVICE;
}

#define HIP_TRY(call)                                  \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// most rounds one persistent launch loops (a longer request is several launches)
constexpr int64_t kPersistChunk = 1024;

// bonds per site: 2 on the square lattice, 3 on the cubic one
int bonds_per_site(int model) { return model == REWL_EA3 ? 3 : 2; }

// Geometry of a run derived from its parameters.
struct Geometry {
    int N = 0, step = 0, nw = 0, Npad = 0, Wmax = 0;
    int64_t e_min = 0, e_max = 0, B = 0;
    bool full_lo = false, full_hi = false;
    std::vector<int64_t> lo, hi;
};

// Windows: span = B-1, w = span / (1 + (h-1)(1-o)); lo_k = floor(k (1-o) w),
// hi_k = min(B-1, ceil(k (1-o) w + w)), hi_{h-1} = B-1 ("equal-size intervals
// with overlap o", Fig. 1a caption), evaluated in this order in binary64.
int make_windows(int64_t B, int h, double o, int64_t *lo, int64_t *hi)
{
    const double span = (double)(B - 1);
    const double w = span / (1.0 + (double)(h - 1) * (1.0 - o));
    for (int k = 0; k < h; ++k) {
        const double x = ((double)k * (1.0 - o)) * w;
        lo[k] = (int64_t)std::floor(x);
        hi[k] = std::min<int64_t>(B - 1, (int64_t)std::ceil(x + w));
    }
    hi[h - 1] = B - 1;
    for (int k = 0; k < h; ++k) {
        if (hi[k] - lo[k] + 1 < 2) return fail(REWL_EINVAL, "a window is narrower than 2 bins");
        if (k + 1 < h) {
            if (lo[k + 1] <= lo[k] || hi[k + 1] < hi[k])
                return fail(REWL_EINVAL, "windows are not increasing");
            if (hi[k] - lo[k + 1] + 1 < 2)
                return fail(REWL_EINVAL, "adjacent windows overlap by fewer than 2 bins");
        }
    }
    return REWL_OK;
}

// An explicit partition: n windows from bin 0 to bin B-1, starts and ends
// increasing, >= 2 bins each, >= 2 bins shared by neighbours.
int check_windows(int64_t B, int n, const int64_t *lo, const int64_t *hi)
{
    if (n < 1 || lo[0] != 0 || hi[n - 1] != B - 1)
        return fail(REWL_EINVAL, "windows must run from the first to the last bin");
    for (int k = 0; k < n; ++k) {
        if (lo[k] < 0 || hi[k] > B - 1 || hi[k] - lo[k] + 1 < 2)
            return fail(REWL_EINVAL, "a window is narrower than 2 bins");
        if (k + 1 < n) {
            if (lo[k + 1] <= lo[k] || hi[k + 1] <= hi[k])
                return fail(REWL_EINVAL, "windows are not increasing");
            if (hi[k] - lo[k + 1] + 1 < 2)
                return fail(REWL_EINVAL, "adjacent windows overlap by fewer than 2 bins");
        }
    }
    return REWL_OK;
}

// Checks the parameters and derives the geometry; the windows (n_windows
// first and last bins) go to lo / hi, which hold n_windows entries.
int validate_into(const rewl_params *p, Geometry &g, int64_t *lo, int64_t *hi)
{
    if (!p) return fail(REWL_EINVAL, "params is NULL");
    if (p->model < 0 || p->model > 3) return fail(REWL_EINVAL, "unknown model");
    if (p->model == REWL_EA3 ? (p->L < 2 || p->L > 32) : (p->L < 3 || p->L > 256))
        return fail(REWL_EINVAL, "L must be in [3, 256] (3D glass: [2, 32])");
    if (p->model == REWL_POTTS && (p->q < 2 || p->q > 127))
        return fail(REWL_EINVAL, "q must be in [2, 127]");
    if (p->n_windows < 1) return fail(REWL_EINVAL, "n_windows must be >= 1");
    if (!(p->overlap > 0.0 && p->overlap < 1.0)) return fail(REWL_EINVAL, "overlap must be in (0,1)");
    if (p->walkers_per_window < 1 || p->walkers_per_window > 64)
        return fail(REWL_EINVAL, "walkers_per_window must be in [1, 64]");
    if (!(p->flatness > 0.0 && p->flatness <= 1.0)) return fail(REWL_EINVAL, "flatness must be in (0,1]");
    if (!(p->lnf_init > 0.0) || !(p->lnf_final > 0.0))
        return fail(REWL_EINVAL, "lnf_init and lnf_final must be > 0");
    if (p->attempts_per_round < 1) return fail(REWL_EINVAL, "attempts_per_round must be >= 1");
    if (p->schedule != REWL_HALVING && p->schedule != REWL_ONE_OVER_T)
        return fail(REWL_EINVAL, "unknown ln f schedule");
    const int64_t N = (int64_t)p->L * p->L * (p->model == REWL_EA3 ? p->L : 1);
    const int64_t nb = bonds_per_site(p->model);
    g.N = (int)N;
    g.step = (p->model == REWL_POTTS) ? 1 : 4;
    const int64_t lo_full = -nb * N, hi_full = (p->model == REWL_POTTS) ? 0 : nb * N;
    int64_t cls = 0;
    if (p->model == REWL_EA || p->model == REWL_EA3) {
        if (!p->couplings) return fail(REWL_EINVAL, "the glass models need couplings");
        int64_t n_neg = 0;
        for (int64_t i = 0; i < nb * N; ++i) {
            const int8_t c = p->couplings[i];
            if (c != 1 && c != -1) return fail(REWL_EINVAL, "couplings must be +-1");
            n_neg += c < 0;
        }
        cls = -nb * N + 2 * n_neg;
    } else if (p->model == REWL_ISING) {
        cls = -2 * N;
    }
    int64_t e_min = p->e_min, e_max = p->e_max;
    g.full_lo = e_min <= lo_full;
    g.full_hi = e_max >= hi_full;
    e_min = std::max(e_min, lo_full);
    e_max = std::min(e_max, hi_full);
    const int64_t st = g.step;
    int64_t r = ((e_min - cls) % st + st) % st;
    if (r) e_min += st - r;
    r = ((e_max - cls) % st + st) % st;
    e_max -= r;
    if (e_max <= e_min) return fail(REWL_EINVAL, "empty energy range");
    g.e_min = e_min;
    g.e_max = e_max;
    g.B = (e_max - e_min) / st + 1;
    int rc;
    if (p->window_lo || p->window_hi) {
        if (!p->window_lo || !p->window_hi)
            return fail(REWL_EINVAL, "window_lo and window_hi go together");
        for (int k = 0; k < p->n_windows; ++k) {
            lo[k] = p->window_lo[k];
            hi[k] = p->window_hi[k];
        }
        rc = check_windows(g.B, p->n_windows, lo, hi);
    } else {
        rc = make_windows(g.B, p->n_windows, p->overlap, lo, hi);
    }
    if (rc) return rc;
    g.Wmax = 0;
    for (int k = 0; k < p->n_windows; ++k)
        g.Wmax = std::max<int>(g.Wmax, (int)(hi[k] - lo[k] + 1));
    g.nw = p->n_windows * p->walkers_per_window;
    g.Npad = (int)align_up((size_t)N, 16);
    if (sweep_lds_bytes(1, g.Wmax, g.N, model_j_words(p->model)) > kMaxLds)
        return fail(REWL_EINVAL, "one walker's window does not fit the LDS of a CU");
    return REWL_OK;
}

// most windows of a run (every window has >= 2 bins and the widest lattice has
// 2^17 + 1 bins, so more are never valid)
constexpr int kMaxWindows = 1 << 17;

int validate(const rewl_params *p, Geometry &g)
{
    if (!p) return fail(REWL_EINVAL, "params is NULL");
    if (p->n_windows < 1) return fail(REWL_EINVAL, "n_windows must be >= 1");
    if (p->n_windows > kMaxWindows) return fail(REWL_EINVAL, "too many windows");
    g.lo.assign(p->n_windows, 0);
    g.hi.assign(p->n_windows, 0);
    return validate_into(p, g, g.lo.data(), g.hi.data());
}

// Byte offsets of the arrays inside the device allocation.
struct Layout {
    size_t spins, E, t, flat, lng, H, n_acc, lnf, done, phase, finish, first, lo, hi, ex_prop,
        ex_acc, J4, round, status, total;
};

Layout layout(const rewl_params *p, const Geometry &g)
{
    Layout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    const size_t nw = (size_t)g.nw, h = (size_t)p->n_windows;
    l.spins = take(nw * g.Npad);
    l.E = take(nw * 4);
    l.t = take(nw * 8);
    l.flat = take(nw * 4);
    l.lng = take(nw * g.Wmax * 8);
    l.H = take(nw * g.Wmax * 4);
    l.n_acc = take(nw * 8);
    l.lnf = take(h * 8);
    l.done = take(h * 4);
    l.phase = take(h * 4);
    l.finish = take(h * 8);
    l.first = take(h * 8);
    l.lo = take(h * 4);
    l.hi = take(h * 4);
    l.ex_prop = take(h * 8);
    l.ex_acc = take(h * 8);
    l.J4 = take(std::max<size_t>(4, (size_t)model_j_words(p->model) * 4 * (size_t)g.N));
    l.round = take(8);
    l.status = take(4);
    l.total = off;
    return l;
}

}  // namespace

struct rewl_batch;

// One run: its parameters, geometry and device slab.  A run is stepped by the
// batch it belongs to; a run made by rewl_create_ex owns a private batch.
struct rewl_ctx {
    rewl_params p{};
    std::vector<int8_t> couplings;
    Geometry g;
    Layout l{};
    void *base = nullptr;
    bool owns = false;
    RunDesc desc{};
    rewl_batch *batch = nullptr;
    bool own_batch = false;
    int64_t id = -1;          // server request id
    int64_t admit_round = 0;  // server: batch round at admission
};

// A set of runs advanced together, round by round, by one stream.
struct rewl_batch {
    std::vector<rewl_ctx *> runs;  // slot i; nullptr = free slot (server)
    bool owns_runs = false;
    hipStream_t stream = nullptr;
    int P = 1;                     // walkers per wave in the sweep
    void *tab = nullptr;           // device work tables + per-run done flags
    size_t tab_cap = 0;
    BatchDev dev{};
    int *done_d = nullptr;
    bool dirty = true;
    int64_t rounds = 0;
    int *pinned = nullptr;
    size_t pinned_cap = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev_free, ev_pending;
    double sweep_ms = 0.0;
    int64_t sweep_launches = 0;
    int form = REWL_FORM_ROUNDS;   // REWL_FORM_ROUNDS or REWL_FORM_PERSISTENT
    int graph_rounds = 0;          // > 0: replay a captured graph of this many rounds
    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_src = nullptr;
    hipStream_t cap_stream = nullptr; // private stream the graph is captured on
    std::atomic<bool> busy{false};    // a host thread is inside a call on this batch
};

// Claims a batch for one host thread for the duration of a call; a second
// thread entering meanwhile gets REWL_EBUSY.
struct Claim {
    std::atomic<bool> *flag = nullptr;
    explicit Claim(rewl_batch *b)
    {
        bool expect = false;
        if (b && b->busy.compare_exchange_strong(expect, true)) flag = &b->busy;
    }
    ~Claim()
    {
        if (flag) flag->store(false);
    }
    explicit operator bool() const { return flag != nullptr; }
};

namespace {

int collect_timing(rewl_batch *b)
{
    for (size_t i = 0; i + 1 < b->ev_pending.size(); i += 2) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, b->ev_pending[i], b->ev_pending[i + 1]));
        b->sweep_ms += ms;
        b->sweep_launches += 1;
        b->ev_free.push_back(b->ev_pending[i]);
        b->ev_free.push_back(b->ev_pending[i + 1]);
    }
    b->ev_pending.clear();
    return REWL_OK;
}

int bsync(rewl_batch *b)
{
    HIP_TRY(hipStreamSynchronize(b->stream));
    return b->timing ? collect_timing(b) : REWL_OK;
}

int take_event(rewl_batch *b, hipEvent_t *e)
{
    if (b->ev_free.empty()) {
        hipEvent_t ev;
        HIP_TRY(hipEventCreate(&ev));
        b->ev_free.push_back(ev);
    }
    *e = b->ev_free.back();
    b->ev_free.pop_back();
    b->ev_pending.push_back(*e);
    return REWL_OK;
}

template <class T>
int d2h(rewl_ctx *h, T *dst, size_t off, size_t count)
{
    HIP_TRY(hipMemcpyAsync(dst, (char *)h->base + off, count * sizeof(T), hipMemcpyDeviceToHost,
                           h->batch->stream));
    return bsync(h->batch);
}

void drop_graph(rewl_batch *b)
{
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->graph_src) (void)hipGraphDestroy(b->graph_src);
    b->graph = nullptr;
    b->graph_src = nullptr;
}

// Work lists of the live runs: sweep groups of P walkers, windows, pair slots.
int rebuild(rewl_batch *b)
{
    drop_graph(b);
    std::vector<RunDesc> descs;
    std::vector<SweepItem> sweep;
    std::vector<WinItem> win, pair;
    int max_N = 1, max_W = 1, j_words = 0;
    for (size_t i = 0; i < b->runs.size(); ++i) {
        rewl_ctx *r = b->runs[i];
        if (!r) continue;
        const int idx = (int)descs.size();
        descs.push_back(r->desc);
        for (int w = 0; w < r->g.nw; w += b->P)
            sweep.push_back(SweepItem{idx, w, std::min(b->P, r->g.nw - w), 0});
        for (int k = 0; k < r->p.n_windows; ++k) win.push_back(WinItem{idx, k});
        for (int k = 0; k < r->p.n_windows / 2; ++k) pair.push_back(WinItem{idx, k});
        max_N = std::max(max_N, r->g.N);
        max_W = std::max(max_W, r->g.Wmax);
        j_words = std::max(j_words, model_j_words(r->p.model));
    }
    if (sweep_lds_bytes(b->P, max_W, max_N, j_words) > kMaxLds)
        return fail(REWL_EINVAL, "walkers_per_wave too large for these runs' LDS footprint");
    int pwaves = 0;
    if (b->form == REWL_FORM_PERSISTENT) {
        // every run in one work-group: its waves of P walkers and their LDS
        for (rewl_ctx *r : b->runs) {
            if (!r) continue;
            if (r->g.nw > kPersistMaxWalkers)
                return fail(REWL_EINVAL, "persistent form: a run has more than 64 walkers");
            pwaves = std::max(pwaves, (r->g.nw + b->P - 1) / b->P);
        }
        if (pwaves > kPersistMaxWaves)
            return fail(REWL_EINVAL, "persistent form: a run needs more than 8 waves at this "
                                     "walkers_per_wave");
        if (persist_lds_bytes(b->P, pwaves, max_W, max_N, j_words) > kPersistMaxDynLds)
            return fail(REWL_EINVAL, "persistent form: a run does not fit the LDS of one CU at "
                                     "this walkers_per_wave");
    }
    const size_t n_runs = descs.size();
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    const size_t o_runs = take(n_runs * sizeof(RunDesc)), o_sw = take(sweep.size() * sizeof(SweepItem));
    const size_t o_win = take(win.size() * sizeof(WinItem)), o_pair = take(pair.size() * sizeof(WinItem));
    const size_t o_done = take(std::max<size_t>(n_runs, 1) * sizeof(int));
    const size_t total = off;
    if (total > b->tab_cap) {
        if (b->tab) (void)hipFree(b->tab);
        b->tab = nullptr;
        b->tab_cap = 0;
        HIP_TRY(hipMalloc(&b->tab, total));
        b->tab_cap = total;
    }
    std::vector<char> host(total, 0);
    std::memcpy(host.data() + o_runs, descs.data(), n_runs * sizeof(RunDesc));
    std::memcpy(host.data() + o_sw, sweep.data(), sweep.size() * sizeof(SweepItem));
    std::memcpy(host.data() + o_win, win.data(), win.size() * sizeof(WinItem));
    std::memcpy(host.data() + o_pair, pair.data(), pair.size() * sizeof(WinItem));
    HIP_TRY(hipMemcpyAsync(b->tab, host.data(), total, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    char *t = (char *)b->tab;
    BatchDev &d = b->dev;
    d.runs = (const RunDesc *)(t + o_runs);
    d.sweep = (const SweepItem *)(t + o_sw);
    d.win = (const WinItem *)(t + o_win);
    d.pair = (const WinItem *)(t + o_pair);
    d.n_runs = (int)n_runs;
    d.n_sweep = (int)sweep.size();
    d.n_win = (int)win.size();
    d.n_pair = (int)pair.size();
    d.P = b->P;
    d.max_N = max_N;
    d.max_W = max_W;
    d.j_words = j_words;
    d.region = (int)sweep_region(max_W, max_N, kWave / b->P);
    d.pwaves = pwaves;
    b->done_d = (int *)(t + o_done);
    if (b->pinned_cap < std::max<size_t>(n_runs, 1)) {
        if (b->pinned) (void)hipHostFree(b->pinned);
        b->pinned = nullptr;
        b->pinned_cap = 0;
        HIP_TRY(hipHostMalloc((void **)&b->pinned, std::max<size_t>(n_runs, 1) * sizeof(int)));
        b->pinned_cap = std::max<size_t>(n_runs, 1);
    }
    b->dirty = false;
    return REWL_OK;
}

int launch_rounds(rewl_batch *b, int64_t rounds)
{
    for (int64_t i = 0; i < rounds; ++i) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (b->timing) {
            int rc = take_event(b, &e0);
            if (!rc) rc = take_event(b, &e1);
            if (rc) return rc;
        }
        const int rc = rewl_launch_round(b->dev, b->stream, e0, e1);
        if (rc)
            return fail(rc == -1 ? REWL_EINVAL : REWL_EDEVICE,
                        std::string("kernel launch failed: ") + rewl_launch_error());
        b->rounds += 1;
    }
    return REWL_OK;
}

int batch_step(rewl_batch *b, int64_t rounds)
{
    if (rounds < 0) return fail(REWL_EINVAL, "negative rounds");
    if (b->dirty) {
        int rc = rebuild(b);
        if (rc) return rc;
    }
    if (b->dev.n_runs == 0) return REWL_OK;
    if (b->form == REWL_FORM_PERSISTENT) {
        // one launch loops the rounds; long requests are cut into launches of
        // at most kPersistChunk rounds (the state passes through HBM between)
        while (rounds > 0) {
            const int64_t n = std::min<int64_t>(rounds, kPersistChunk);
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (b->timing) {
                int rc = take_event(b, &e0);
                if (!rc) rc = take_event(b, &e1);
                if (rc) return rc;
            }
            const int rc = rewl_launch_persist(b->dev, (long long)n, b->stream, e0, e1);
            if (rc)
                return fail(rc == -1 ? REWL_EINVAL : REWL_EDEVICE,
                            std::string("persistent launch failed: ") + rewl_launch_error());
            b->rounds += n;
            rounds -= n;
        }
        return REWL_OK;
    }
    const int R = b->graph_rounds;
    if (R > 0 && !b->timing) {
        if (!b->graph) {
            // the null stream cannot be captured: capture on a private stream,
            // replay on the batch's stream
            if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
            HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
            int rc = REWL_OK;
            for (int i = 0; i < R && !rc; ++i)
                rc = rewl_launch_round(b->dev, b->cap_stream, nullptr, nullptr) ? REWL_EDEVICE : 0;
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
            if (rc || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return rc ? fail(rc, "capture of the round graph failed")
                          : hip_fail(e, "hipStreamEndCapture");
            }
            b->graph_src = g;
            e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                drop_graph(b);
                return hip_fail(e, "hipGraphInstantiate");
            }
        }
        while (rounds >= R) {
            HIP_TRY(hipGraphLaunch(b->graph, b->stream));
            b->rounds += R;
            rounds -= R;
        }
    }
    return launch_rounds(b, rounds);
}

// per-run "all windows done" flags of the batch's live runs, in slot order
int batch_done(rewl_batch *b, std::vector<int> &flags)
{
    if (b->dirty) {
        int rc = rebuild(b);
        if (rc) return rc;
    }
    flags.assign((size_t)b->dev.n_runs, 0);
    if (b->dev.n_runs == 0) return REWL_OK;
    if (rewl_launch_status(b->dev, b->done_d, b->stream)) return fail(REWL_EDEVICE, "status launch");
    HIP_TRY(hipMemcpyAsync(b->pinned, b->done_d, (size_t)b->dev.n_runs * sizeof(int),
                           hipMemcpyDeviceToHost, b->stream));
    int rc = bsync(b);
    if (rc) return rc;
    for (int i = 0; i < b->dev.n_runs; ++i) flags[i] = b->pinned[i];
    return REWL_OK;
}

// rounds until every live run is done or max_rounds issued; polls after a
// doubling number of rounds (capped at 64)
int batch_run(rewl_batch *b, int64_t max_rounds, bool *all)
{
    std::vector<int> flags;
    int rc = batch_done(b, flags);
    if (rc) return rc;
    auto every = [&]() {
        for (int f : flags)
            if (!f) return false;
        return true;
    };
    int64_t issued = 0, chunk = 4;
    while (!every() && (max_rounds < 0 || issued < max_rounds)) {
        int64_t n = chunk;
        if (max_rounds >= 0) n = std::min(n, max_rounds - issued);
        rc = batch_step(b, n);
        if (rc) return rc;
        issued += n;
        rc = batch_done(b, flags);
        if (rc) return rc;
        chunk = std::min<int64_t>(chunk * 2, 64);
    }
    *all = every();
    return REWL_OK;
}

void free_run(rewl_ctx *h)
{
    if (!h) return;
    if (h->owns && h->base) (void)hipFree(h->base);
    delete h;
}

void free_batch(rewl_batch *b)
{
    if (!b) return;
    if (b->stream || b->tab) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->owns_runs)
        for (rewl_ctx *r : b->runs) free_run(r);
    if (b->tab) (void)hipFree(b->tab);
    if (b->pinned) (void)hipHostFree(b->pinned);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (hipEvent_t e : b->ev_free) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->ev_pending) (void)hipEventDestroy(e);
    delete b;
}

// The scalar fields of a run's descriptor (the array pointers are the caller's).
void fill_desc(RunDesc &d, const rewl_params *p, const Geometry &g)
{
    d.model = p->model;
    d.L = p->L;
    d.N = g.N;
    d.q = (p->model == REWL_POTTS) ? p->q : 2;
    d.h = p->n_windows;
    d.m = p->walkers_per_window;
    d.nw = g.nw;
    d.Npad = g.Npad;
    d.Wmax = g.Wmax;
    d.e_min = (int)g.e_min;
    d.step = g.step;
    d.l_magic = (uint32_t)(((uint64_t)1 << 32) / (uint64_t)p->L + 1);
    d.l2_magic = (uint32_t)(((uint64_t)1 << 32) / ((uint64_t)p->L * (uint64_t)p->L) + 1);
    d.key0 = (uint32_t)p->seed;
    d.key1 = (uint32_t)(p->seed >> 32);
    d.S = p->attempts_per_round;
    d.schedule = p->schedule;
    d.flat_p = p->flatness;
    d.lnf_final = p->lnf_final;
}

// Make one run: validate, lay out, allocate (or adopt) its slab, upload its
// parameters and run the start-up kernel on `stream`.
int make_run(rewl_ctx **out, const rewl_params *p, void *device_buffer, size_t buffer_bytes,
             hipStream_t stream, const void *slab = nullptr, size_t slab_bytes = 0)
{
    *out = nullptr;
    Geometry g;
    int rc = validate(p, g);
    if (rc) return rc;
    rewl_ctx *h = new (std::nothrow) rewl_ctx();
    if (!h) return fail(REWL_ENOMEM, "host allocation failed");
    h->p = *p;
    h->g = g;
    h->l = layout(p, g);
    // the windows live in the geometry from here on
    h->p.window_lo = h->g.lo.data();
    h->p.window_hi = h->g.hi.data();
    if (p->model == REWL_EA || p->model == REWL_EA3) {
        h->couplings.assign(p->couplings,
                            p->couplings + (size_t)bonds_per_site(p->model) * (size_t)g.N);
        h->p.couplings = h->couplings.data();
    } else {
        h->p.couplings = nullptr;
    }
    auto bail = [&](int code) {
        free_run(h);
        return code;
    };
    if (device_buffer) {
        if (buffer_bytes < h->l.total || ((uintptr_t)device_buffer & 255))
            return bail(fail(REWL_ENOMEM, "device buffer too small or not 256-byte aligned"));
        h->base = device_buffer;
    } else {
        hipError_t e = hipMalloc(&h->base, h->l.total);
        if (e != hipSuccess) return bail(fail(REWL_ENOMEM, "hipMalloc of the run state failed"));
        h->owns = true;
    }
    char *b = (char *)h->base;
    RunDesc &d = h->desc;
    fill_desc(d, p, g);
    d.spins = (int8_t *)(b + h->l.spins);
    d.E = (int *)(b + h->l.E);
    d.t = (unsigned long long *)(b + h->l.t);
    d.flat = (int *)(b + h->l.flat);
    d.lng = (double *)(b + h->l.lng);
    d.H = (uint32_t *)(b + h->l.H);
    d.n_acc = (unsigned long long *)(b + h->l.n_acc);
    d.lnf = (double *)(b + h->l.lnf);
    d.done = (int *)(b + h->l.done);
    d.phase = (int *)(b + h->l.phase);
    d.finish = (long long *)(b + h->l.finish);
    d.first = (long long *)(b + h->l.first);
    d.lo = (int *)(b + h->l.lo);
    d.hi = (int *)(b + h->l.hi);
    d.ex_prop = (unsigned long long *)(b + h->l.ex_prop);
    d.ex_acc = (unsigned long long *)(b + h->l.ex_acc);
    d.J4 = (uint32_t *)(b + h->l.J4);
    d.round = (long long *)(b + h->l.round);
    d.status = (int *)(b + h->l.status);

    if (slab) {
        // resume: the saved device state replaces the start-up
        if (slab_bytes != h->l.total) return bail(fail(REWL_ECORRUPT, "saved state has the wrong size"));
        hipError_t e = hipMemcpyAsync(h->base, slab, slab_bytes, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return bail(hip_fail(e, "upload of the saved state"));
        *out = h;
        return REWL_OK;
    }
    const int H = p->n_windows, N = g.N, L = p->L;
    std::vector<double> lnf(H, p->lnf_init);
    std::vector<long long> fin(H, -1);
    std::vector<int> lo(H), hi(H);
    for (int k = 0; k < H; ++k) {
        lo[k] = (int)g.lo[k];
        hi[k] = (int)g.hi[k];
    }
    std::vector<uint32_t> J4;
    if (p->model == REWL_EA) {
        J4.resize(N);
        const int8_t *J = h->p.couplings;
        for (int i = 0; i < N; ++i) {
            const int r = i / L, c = i % L;
            const int lf = r * L + (c + L - 1) % L, up = ((r + L - 1) % L) * L + c;
            J4[i] = (uint32_t)(uint8_t)J[2 * i] | ((uint32_t)(uint8_t)J[2 * lf] << 8) |
                    ((uint32_t)(uint8_t)J[2 * i + 1] << 16) | ((uint32_t)(uint8_t)J[2 * up + 1] << 24);
        }
    } else if (p->model == REWL_EA3) {
        // two words per site: +x, -x, +y, -y | +z, -z (bond a of site i is J[3i + a])
        J4.resize(2 * (size_t)N);
        const int8_t *J = h->p.couplings;
        const int L2 = L * L;
        for (int i = 0; i < N; ++i) {
            const int x = i % L, y = (i / L) % L, z = i / L2;
            const int xm = i - x + (x + L - 1) % L;
            const int ym = z * L2 + ((y + L - 1) % L) * L + x;
            const int zm = ((z + L - 1) % L) * L2 + y * L + x;
            J4[2 * (size_t)i] = (uint32_t)(uint8_t)J[3 * i] | ((uint32_t)(uint8_t)J[3 * xm] << 8) |
                                ((uint32_t)(uint8_t)J[3 * i + 1] << 16) |
                                ((uint32_t)(uint8_t)J[3 * ym + 1] << 24);
            J4[2 * (size_t)i + 1] = (uint32_t)(uint8_t)J[3 * i + 2] |
                                    ((uint32_t)(uint8_t)J[3 * zm + 2] << 8);
        }
    }
    hipError_t e = hipMemsetAsync(h->base, 0, h->l.total, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.lnf, lnf.data(), H * 8, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.finish, fin.data(), H * 8, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.first, fin.data(), H * 8, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.lo, lo.data(), H * 4, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.hi, hi.data(), H * 4, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !J4.empty())
        e = hipMemcpyAsync(d.J4, J4.data(), J4.size() * 4, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return bail(hip_fail(e, "upload of the run parameters"));
    rc = rewl_launch_init(d, stream);
    if (rc) return bail(fail(REWL_EDEVICE, "launch of the start-up kernel failed"));
    int status = 0;
    e = hipMemcpyAsync(&status, d.status, 4, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return bail(hip_fail(e, "start-up"));
    if (status) return bail(fail(REWL_EINIT, "a walker could not reach its window"));
    *out = h;
    return REWL_OK;
}

rewl_batch *new_batch(hipStream_t stream, int P)
{
    rewl_batch *b = new (std::nothrow) rewl_batch();
    if (!b) return nullptr;
    b->stream = stream;
    b->P = P;
    return b;
}

bool valid_P(int P) { return P == 1 || P == 2 || P == 4 || P == 8; }

// Join window pieces: for windows k and k+1, among the bins of their overlap
// visited by both pieces (at or above the previous joining bin), compare the
// slopes (P(b') - P(b)) / (b' - b) toward the next such bin b' and join at the
// bin where the two slopes agree best, lowest bin on ties ("the joining point
// ... where the inverse microcanonical temperatures best coincide").
int stitch(const rewl_ctx *h, const std::vector<double> &P, double *out)
{
    const Geometry &g = h->g;
    const int H = h->p.n_windows;
    const size_t W = (size_t)g.Wmax;
    for (int64_t b = 0; b < g.B; ++b) out[b] = -INFINITY;
    auto vis = [&](int k, int64_t b) { return P[(size_t)k * W + (size_t)(b - g.lo[k])] > 0.0; };
    auto val = [&](int k, int64_t b) { return P[(size_t)k * W + (size_t)(b - g.lo[k])]; };
    double shift = 0.0;
    int64_t start = g.lo[0];
    for (int k = 0; k < H; ++k) {
        int64_t end = g.hi[k];
        double next_shift = 0.0;
        if (k + 1 < H) {
            int64_t best = -1, prev = -1;
            double best_diff = INFINITY;
            for (int64_t b = std::max(g.lo[k + 1], start); b <= g.hi[k]; ++b) {
                if (!vis(k, b) || !vis(k + 1, b)) continue;
                if (prev >= 0) {
                    const double dk = (val(k, b) - val(k, prev)) / (double)(b - prev);
                    const double dn = (val(k + 1, b) - val(k + 1, prev)) / (double)(b - prev);
                    const double diff = std::fabs(dk - dn);
                    if (diff < best_diff) {
                        best_diff = diff;
                        best = prev;
                    }
                }
                prev = b;
            }
            if (best < 0) return fail(REWL_ESTITCH, "window overlap without commonly visited bins");
            end = best - 1;
            next_shift = shift + (val(k, best) - val(k + 1, best));
        }
        for (int64_t b = start; b <= end; ++b)
            if (vis(k, b)) out[b] = val(k, b) + shift;
        if (k + 1 < H) {
            start = end + 1;
            shift = next_shift;
        }
    }
    // normalisation
    const int64_t N = g.N;
    double ref = 0.0, target = 0.0;
    const bool glass = h->p.model == REWL_EA || h->p.model == REWL_EA3;
    if (!glass && g.full_lo && std::isfinite(out[0])) {
        ref = out[0];
        target = std::log(h->p.model == REWL_POTTS ? (double)h->p.q : 2.0);
    } else if (glass && g.full_lo && g.full_hi) {
        double mx = -INFINITY;
        for (int64_t b = 0; b < g.B; ++b) mx = std::max(mx, out[b]);
        double sum = 0.0;
        for (int64_t b = 0; b < g.B; ++b)
            if (std::isfinite(out[b])) sum = sum + std::exp(out[b] - mx);
        ref = mx + std::log(sum);
        target = (double)N * std::log(2.0);
    } else {
        for (int64_t b = 0; b < g.B; ++b)
            if (std::isfinite(out[b])) {
                ref = out[b];
                break;
            }
    }
    for (int64_t b = 0; b < g.B; ++b)
        if (std::isfinite(out[b])) out[b] = (out[b] - ref) + target;
    return REWL_OK;
}

}  // namespace

extern "C" {

const char *rewl_last_error(void) { return g_err; }

int rewl_footprint(const rewl_params *p, size_t *device_bytes, size_t *lds_bytes)
{
    Geometry g;
    int rc = validate(p, g);
    if (rc) return rc;
    if (device_bytes) *device_bytes = layout(p, g).total;
    if (lds_bytes) *lds_bytes = sweep_lds_bytes(1, g.Wmax, g.N, model_j_words(p->model));
    return REWL_OK;
}

void rewl_destroy(rewl_ctx *h)
{
    if (!h) return;
    if (h->own_batch) {
        free_batch(h->batch);  // owns the run
        return;
    }
    if (!h->batch) free_run(h);
    // runs of a user batch are released with the batch
}

}  // extern "C"

static int get_lng_impl(rewl_ctx *h, double *out, int64_t cap, int64_t *n_bins, int64_t *e_min,
                 int64_t *e_step)
{
    if (!h) return fail(REWL_EINVAL, "bad handle");
    if (n_bins) *n_bins = h->g.B;
    if (e_min) *e_min = h->g.e_min;
    if (e_step) *e_step = h->g.step;
    if (!out) return REWL_OK;
    if (cap < h->g.B) return fail(REWL_EINVAL, "output capacity below n_bins");
    const int H = h->p.n_windows, m = h->p.walkers_per_window;
    std::vector<double> P((size_t)H * h->g.Wmax);
    for (int k = 0; k < H; ++k) {
        int rc = d2h(h, P.data() + (size_t)k * h->g.Wmax,
                     h->l.lng + 8 * (size_t)(k * m) * h->g.Wmax, (size_t)h->g.Wmax);
        if (rc) return rc;
    }
    int rc = stitch(h, P, out);
    if (rc) return rc;
    std::vector<int> dn(H);
    rc = d2h(h, dn.data(), h->l.done, (size_t)H);
    if (rc) return rc;
    for (int k = 0; k < H; ++k)
        if (!dn[k]) return REWL_NOT_CONVERGED;
    return REWL_OK;
}

extern "C" {

int rewl_create_ex(rewl_ctx **out, const rewl_params *p, void *device_buffer, size_t buffer_bytes,
                   void *hip_stream)
{
    if (!out) return fail(REWL_EINVAL, "out is NULL");
    *out = nullptr;
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    rewl_ctx *h = nullptr;
    int rc = make_run(&h, p, device_buffer, buffer_bytes, stream);
    if (rc) return rc;
    rewl_batch *b = new_batch(stream, 1);
    if (!b) {
        free_run(h);
        return fail(REWL_ENOMEM, "host allocation failed");
    }
    b->runs.push_back(h);
    b->owns_runs = true;
    h->batch = b;
    h->own_batch = true;
    *out = h;
    return REWL_OK;
}

extern "C++" {
namespace {

// checkpoint file: "REWLSAV1", the parameters field by field, the couplings,
// the windows, the device slab, then an FNV-1a 64 checksum of everything before
uint64_t fnv1a(const char *p, size_t n)
{
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= (uint8_t)p[i];
        h *= 1099511628211ull;
    }
    return h;
}

template <class T> void put(std::string &s, const T &v) { s.append((const char *)&v, sizeof(T)); }

struct Reader {
    const std::string &s;
    size_t at = 0;
    bool ok = true;
    template <class T> T get()
    {
        T v{};
        if (at + sizeof(T) > s.size()) {
            ok = false;
            return v;
        }
        std::memcpy(&v, s.data() + at, sizeof(T));
        at += sizeof(T);
        return v;
    }
    const char *bytes(size_t n)
    {
        if (n > s.size() - at) {
            ok = false;
            return nullptr;
        }
        const char *p = s.data() + at;
        at += n;
        return p;
    }
};

const char kMagic[8] = {'R', 'E', 'W', 'L', 'S', 'A', 'V', '1'};

// The saved state goes to kernels that index LDS with the walkers' energies and
// windows and combine spins and couplings into energy changes: a file whose
// state does not fit its own parameters is refused (the checksum guards against
// accidents, not against a made-up file).
int check_saved_state(const rewl_params &p, const Geometry &g, const char *slab, size_t ns)
{
    const Layout l = layout(&p, g);
    if (ns != l.total) return fail(REWL_ECORRUPT, "saved state has the wrong size");
    for (int k = 0; k < p.n_windows; ++k) {
        int32_t lo, hi;
        std::memcpy(&lo, slab + l.lo + 4 * (size_t)k, 4);
        std::memcpy(&hi, slab + l.hi + 4 * (size_t)k, 4);
        if (lo != g.lo[k] || hi != g.hi[k])
            return fail(REWL_ECORRUPT, "saved windows disagree with the parameters");
    }
    for (int w = 0; w < g.nw; ++w) {
        int32_t e;
        std::memcpy(&e, slab + l.E + 4 * (size_t)w, 4);
        const int k = w / p.walkers_per_window;
        const int64_t elo = g.e_min + g.lo[k] * g.step, ehi = g.e_min + g.hi[k] * g.step;
        if (e < elo || e > ehi || (e - g.e_min) % g.step != 0)
            return fail(REWL_ECORRUPT, "a saved energy lies outside its walker's window");
        const int8_t *sp = reinterpret_cast<const int8_t *>(slab + l.spins + (size_t)w * g.Npad);
        for (int i = 0; i < g.N; ++i) {
            const int v = sp[i];
            if (p.model == REWL_POTTS ? (v < 0 || v >= p.q) : (v != 1 && v != -1))
                return fail(REWL_ECORRUPT, "a saved spin is not a state of the model");
        }
    }
    // coupling words: EA four +-1 bytes per site; EA3 six, then two zero bytes
    const int jw = model_j_words(p.model);
    for (size_t i = 0; i < (size_t)jw * 4 * (size_t)g.N; ++i) {
        const int8_t j = (int8_t)slab[l.J4 + i];
        const bool pad = jw == 2 && i % 8 >= 6;
        if (pad ? j != 0 : (j != 1 && j != -1))
            return fail(REWL_ECORRUPT, "a saved coupling is not +-1");
    }
    return REWL_OK;
}

}  // namespace
}  // extern "C++"

int rewl_save(rewl_ctx *h, const char *path)
{
    if (!h || !path) return fail(REWL_EINVAL, "bad handle or path");
    Claim c(h->batch);
    if (h->batch && !c) return fail(REWL_EBUSY, "the run is in use by another thread");
    hipStream_t stream = h->batch ? h->batch->stream : nullptr;
    std::vector<char> slab(h->l.total);
    hipError_t e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipMemcpy(slab.data(), h->base, slab.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "download of the run state");
    const rewl_params &p = h->p;
    std::string s(kMagic, 8);
    put<int32_t>(s, p.model);
    put<int32_t>(s, p.L);
    put<int32_t>(s, p.q);
    put<int32_t>(s, p.n_windows);
    put<int32_t>(s, p.walkers_per_window);
    put<int32_t>(s, p.schedule);
    put<int64_t>(s, p.e_min);
    put<int64_t>(s, p.e_max);
    put<double>(s, p.overlap);
    put<double>(s, p.flatness);
    put<double>(s, p.lnf_init);
    put<double>(s, p.lnf_final);
    put<int64_t>(s, p.attempts_per_round);
    put<uint64_t>(s, p.seed);
    put<uint64_t>(s, (uint64_t)h->couplings.size());
    s.append((const char *)h->couplings.data(), h->couplings.size());
    for (int k = 0; k < p.n_windows; ++k) put<int64_t>(s, h->g.lo[k]);
    for (int k = 0; k < p.n_windows; ++k) put<int64_t>(s, h->g.hi[k]);
    put<uint64_t>(s, (uint64_t)slab.size());
    s.append(slab.data(), slab.size());
    put<uint64_t>(s, fnv1a(s.data(), s.size()));
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(REWL_EINVAL, "cannot open the checkpoint file for writing");
    const bool wrote = std::fwrite(s.data(), 1, s.size(), f) == s.size();
    const bool closed = std::fclose(f) == 0;
    if (!wrote || !closed || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(REWL_EINVAL, "writing the checkpoint file failed");
    }
    return REWL_OK;
}

int rewl_load(rewl_ctx **out, const char *path, void *device_buffer, size_t buffer_bytes,
              void *hip_stream)
{
    if (!out || !path) return fail(REWL_EINVAL, "out or path is NULL");
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(REWL_EINVAL, "cannot open the checkpoint file");
    std::string s;
    char buf[1 << 16];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
    std::fclose(f);
    if (s.size() < 16 || std::memcmp(s.data(), kMagic, 8) != 0)
        return fail(REWL_ECORRUPT, "not a checkpoint file");
    uint64_t sum;
    std::memcpy(&sum, s.data() + s.size() - 8, 8);
    if (fnv1a(s.data(), s.size() - 8) != sum) return fail(REWL_ECORRUPT, "checkpoint checksum mismatch");
    Reader r{s, 8};
    rewl_params p{};
    p.model = r.get<int32_t>();
    p.L = r.get<int32_t>();
    p.q = r.get<int32_t>();
    p.n_windows = r.get<int32_t>();
    p.walkers_per_window = r.get<int32_t>();
    p.schedule = r.get<int32_t>();
    p.e_min = r.get<int64_t>();
    p.e_max = r.get<int64_t>();
    p.overlap = r.get<double>();
    p.flatness = r.get<double>();
    p.lnf_init = r.get<double>();
    p.lnf_final = r.get<double>();
    p.attempts_per_round = r.get<int64_t>();
    p.seed = r.get<uint64_t>();
    const uint64_t nc = r.get<uint64_t>();
    const char *cp = r.bytes((size_t)nc);
    if (!r.ok || p.n_windows < 1 || p.n_windows > (1 << 20)) return fail(REWL_ECORRUPT, "truncated checkpoint");
    std::vector<int8_t> couplings(cp, cp + nc);
    std::vector<int64_t> lo((size_t)p.n_windows), hi((size_t)p.n_windows);
    for (auto &v : lo) v = r.get<int64_t>();
    for (auto &v : hi) v = r.get<int64_t>();
    const uint64_t ns = r.get<uint64_t>();
    const char *slab = r.bytes((size_t)ns);
    if (!r.ok || r.at + 8 != s.size()) return fail(REWL_ECORRUPT, "truncated checkpoint");
    p.couplings = couplings.empty() ? nullptr : couplings.data();
    p.window_lo = lo.data();
    p.window_hi = hi.data();
    const bool glass = p.model == REWL_EA || p.model == REWL_EA3;
    if (glass ? (p.L < 2 || p.L > 256) : nc != 0)
        return fail(REWL_ECORRUPT, "checkpoint couplings do not fit the model");
    if (glass) {
        const uint64_t n = (uint64_t)p.L * (uint64_t)p.L * (p.model == REWL_EA3 ? (uint64_t)p.L : 1u);
        if (nc != n * (uint64_t)bonds_per_site(p.model))
            return fail(REWL_ECORRUPT, "checkpoint couplings do not fit the model");
    }
    Geometry g;
    int vrc = validate(&p, g);
    if (vrc) return vrc;
    vrc = check_saved_state(p, g, slab, (size_t)ns);
    if (vrc) return vrc;
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    rewl_ctx *h = nullptr;
    int rc = make_run(&h, &p, device_buffer, buffer_bytes, stream, slab, (size_t)ns);
    if (rc) return rc;
    rewl_batch *b = new_batch(stream, 1);
    if (!b) {
        free_run(h);
        return fail(REWL_ENOMEM, "host allocation failed");
    }
    b->runs.push_back(h);
    b->owns_runs = true;
    h->batch = b;
    h->own_batch = true;
    *out = h;
    return REWL_OK;
}

int rewl_create(rewl_ctx **out, int model, int L, int q, const int8_t *couplings, int64_t e_min,
                int64_t e_max, int n_windows, double overlap, int walkers_per_window,
                double flatness, double lnf_final, uint64_t seed)
{
    rewl_params p{};
    p.model = model;
    p.L = L;
    p.q = q;
    p.couplings = couplings;
    p.e_min = e_min;
    p.e_max = e_max;
    p.n_windows = n_windows;
    p.overlap = overlap;
    p.walkers_per_window = walkers_per_window;
    p.flatness = flatness;
    p.lnf_init = 1.0;
    p.lnf_final = lnf_final;
    p.attempts_per_round = 10000;
    p.seed = seed;
    p.schedule = REWL_HALVING;
    return rewl_create_ex(out, &p, nullptr, 0, nullptr);
}

int rewl_step(rewl_ctx *h, int64_t rounds)
{
    if (!h || !h->own_batch) return fail(REWL_EINVAL, "bad handle (runs of a batch step with it)");
    Claim c(h->batch);
    if (!c) return fail(REWL_EBUSY, "the run is in use by another thread");
    return batch_step(h->batch, rounds);
}

int rewl_set_timing(rewl_ctx *h, int on)
{
    if (!h || !h->batch) return fail(REWL_EINVAL, "bad handle");
    return rewl_batch_set_timing(h->batch, on);
}

int rewl_get_timing(rewl_ctx *h, double *sweep_ms, int64_t *sweep_launches)
{
    if (!h || !h->batch) return fail(REWL_EINVAL, "bad handle");
    return rewl_batch_get_timing(h->batch, sweep_ms, sweep_launches);
}

int rewl_run(rewl_ctx *h, int64_t max_rounds, int64_t *rounds_done)
{
    if (!h || !h->own_batch) return fail(REWL_EINVAL, "bad handle (runs of a batch run with it)");
    Claim c(h->batch);
    if (!c) return fail(REWL_EBUSY, "the run is in use by another thread");
    bool done = false;
    int rc = batch_run(h->batch, max_rounds, &done);
    if (rc) return rc;
    if (rounds_done) {
        *rounds_done = h->batch->rounds;
        if (done) {
            std::vector<long long> fin(h->p.n_windows);
            rc = d2h(h, fin.data(), h->l.finish, fin.size());
            if (rc) return rc;
            *rounds_done = *std::max_element(fin.begin(), fin.end()) + 1;
        }
    }
    return done ? REWL_OK : REWL_NOT_CONVERGED;
}

int rewl_get_window(rewl_ctx *h, int k, int64_t *lo, int64_t *hi, double *lnf, int *done,
                    int64_t *finish_round)
{
    if (!h || k < 0 || k >= h->p.n_windows) return fail(REWL_EINVAL, "bad handle or window");
    double l;
    int dn;
    long long f;
    int rc = d2h(h, &l, h->l.lnf + 8 * (size_t)k, 1);
    if (!rc) rc = d2h(h, &dn, h->l.done + 4 * (size_t)k, 1);
    if (!rc) rc = d2h(h, &f, h->l.finish + 8 * (size_t)k, 1);
    if (rc) return rc;
    if (lo) *lo = h->g.lo[k];
    if (hi) *hi = h->g.hi[k];
    if (lnf) *lnf = l;
    if (done) *done = dn;
    if (finish_round) *finish_round = f;
    return REWL_OK;
}

int rewl_get_first_merge(rewl_ctx *h, int64_t *out, int cap)
{
    if (!h || !out || cap < 0) return fail(REWL_EINVAL, "bad handle or output");
    const int n = std::min(cap, h->p.n_windows);
    std::vector<long long> f((size_t)h->p.n_windows);
    int rc = d2h(h, f.data(), h->l.first, f.size());
    if (rc) return rc;
    for (int k = 0; k < n; ++k) out[k] = f[(size_t)k];
    return REWL_OK;
}

int rewl_partition_balanced(int64_t n_bins, int n_windows, double overlap, int pre_windows,
                            const int64_t *pre_lo, const int64_t *pre_hi,
                            const int64_t *first_rounds, int64_t *lo, int64_t *hi)
{
    if (n_bins < 2 || n_windows < 1 || pre_windows < 1 || !(overlap > 0.0 && overlap < 1.0) ||
        !pre_lo || !pre_hi || !first_rounds || !lo || !hi)
        return fail(REWL_EINVAL, "bad arguments");
    const std::vector<int64_t> plo(pre_lo, pre_lo + pre_windows), phi(pre_hi, pre_hi + pre_windows);
    if (check_windows(n_bins, pre_windows, plo.data(), phi.data())) return REWL_EINVAL;
    for (int k = 0; k < pre_windows; ++k)
        if (first_rounds[k] < 1) return fail(REWL_EINVAL, "first-iteration rounds must be >= 1");
    // time density of each bin in the first iteration: the pre-run windows
    // that hold the bin, each contributing its rounds per bin
    std::vector<double> dens((size_t)n_bins);
    for (int64_t b = 0; b < n_bins; ++b) {
        double acc = 0.0;
        int cover = 0;
        for (int k = 0; k < pre_windows; ++k) {
            if (b >= plo[k] && b <= phi[k]) {
                acc = acc + (double)first_rounds[k] / (double)(phi[k] - plo[k] + 1);
                ++cover;
            }
        }
        dens[(size_t)b] = acc / (double)cover;
    }
    // bins as points of the time axis (trapezoids between neighbours)
    std::vector<double> axis((size_t)n_bins);
    axis[0] = 0.0;
    for (int64_t b = 1; b < n_bins; ++b)
        axis[(size_t)b] = axis[(size_t)b - 1] + (dens[(size_t)b - 1] + dens[(size_t)b]) * 0.5;
    // the equal partition of that axis
    const double width = axis[(size_t)n_bins - 1] / (1.0 + (double)(n_windows - 1) * (1.0 - overlap));
    std::vector<int64_t> L((size_t)n_windows), H((size_t)n_windows);
    int64_t first = 0, last = 0;
    for (int k = 0; k < n_windows; ++k) {
        const double start = ((double)k * (1.0 - overlap)) * width;
        const double end = start + width;
        while (first + 1 < n_bins && axis[(size_t)first + 1] <= start) ++first;
        while (last < n_bins - 1 && axis[(size_t)last] < end) ++last;
        L[(size_t)k] = first;
        H[(size_t)k] = last;
    }
    H[(size_t)n_windows - 1] = n_bins - 1;
    if (check_windows(n_bins, n_windows, L.data(), H.data())) return REWL_EINVAL;
    for (int k = 0; k < n_windows; ++k) {
        lo[k] = L[(size_t)k];
        hi[k] = H[(size_t)k];
    }
    return REWL_OK;
}

int rewl_jackknife(const double *lng, int runs, int64_t n_bins, double *mean, double *err)
{
    if (!lng || !mean || !err || runs < 2 || n_bins < 1) return fail(REWL_EINVAL, "bad arguments");
    const double R = (double)runs;
    std::vector<double> theta((size_t)runs);
    for (int64_t b = 0; b < n_bins; ++b) {
        bool seen = true;
        double total = 0.0;
        for (int r = 0; r < runs; ++r) {
            const double x = lng[(size_t)r * (size_t)n_bins + (size_t)b];
            seen = seen && std::isfinite(x);
            total += x;
        }
        if (!seen) {
            mean[b] = -HUGE_VAL;
            err[b] = std::nan("");
            continue;
        }
        double tbar = 0.0;
        for (int r = 0; r < runs; ++r) {
            theta[(size_t)r] = (total - lng[(size_t)r * (size_t)n_bins + (size_t)b]) / (R - 1.0);
            tbar += theta[(size_t)r];
        }
        tbar /= R;
        double ss = 0.0;
        for (int r = 0; r < runs; ++r) ss += (theta[(size_t)r] - tbar) * (theta[(size_t)r] - tbar);
        mean[b] = total / R;
        err[b] = std::sqrt((R - 1.0) / R * ss);
    }
    return REWL_OK;
}

int rewl_get_walker(rewl_ctx *h, int w, int8_t *spins, int64_t *E, uint64_t *t, int *flat,
                    double *lng, uint32_t *H, uint8_t *visited)
{
    if (!h || w < 0 || w >= h->g.nw) return fail(REWL_EINVAL, "bad handle or walker");
    const int k = w / h->p.walkers_per_window;
    const size_t W = (size_t)(h->g.hi[k] - h->g.lo[k] + 1);
    int rc = REWL_OK;
    if (spins) rc = d2h(h, spins, h->l.spins + (size_t)w * h->g.Npad, (size_t)h->g.N);
    if (!rc && E) {
        int e;
        rc = d2h(h, &e, h->l.E + 4 * (size_t)w, 1);
        *E = e;
    }
    if (!rc && t) {
        unsigned long long v;
        rc = d2h(h, &v, h->l.t + 8 * (size_t)w, 1);
        *t = v;
    }
    if (!rc && flat) rc = d2h(h, flat, h->l.flat + 4 * (size_t)w, 1);
    std::vector<double> g;
    if (!rc && (lng || visited)) {
        g.resize(W);
        rc = d2h(h, g.data(), h->l.lng + 8 * (size_t)w * h->g.Wmax, W);
        if (lng) std::memcpy(lng, g.data(), W * 8);
        if (visited)
            for (size_t b = 0; b < W; ++b) visited[b] = g[b] > 0.0;
    }
    if (!rc && H) rc = d2h(h, H, h->l.H + 4 * (size_t)w * h->g.Wmax, W);
    return rc;
}

int rewl_get_lng(rewl_ctx *h, double *out, int64_t cap, int64_t *n_bins, int64_t *e_min,
                 int64_t *e_step)
{
    if (!h) return fail(REWL_EINVAL, "bad handle");
    Claim claim(h->batch);
    if (h->batch && !claim) return fail(REWL_EBUSY, "the run is in use by another thread");
    return get_lng_impl(h, out, cap, n_bins, e_min, e_step);
}

int rewl_get_info(rewl_ctx *h, int64_t *n_bins, int64_t *e_min, int64_t *e_step, int *n_windows,
                  int *walkers_per_window, int *n_sites, int64_t *rounds, uint64_t *attempts,
                  uint64_t *accepts, uint64_t *ex_prop, uint64_t *ex_acc)
{
    if (!h) return fail(REWL_EINVAL, "bad handle");
    Claim claim(h->batch);
    if (h->batch && !claim) return fail(REWL_EBUSY, "the run is in use by another thread");
    if (n_bins) *n_bins = h->g.B;
    if (e_min) *e_min = h->g.e_min;
    if (e_step) *e_step = h->g.step;
    if (n_windows) *n_windows = h->p.n_windows;
    if (walkers_per_window) *walkers_per_window = h->p.walkers_per_window;
    if (n_sites) *n_sites = h->g.N;
    const size_t nw = (size_t)h->g.nw, H = (size_t)h->p.n_windows;
    std::vector<unsigned long long> a(nw), c(nw), xp(H), xa(H);
    long long r = 0;
    int rc = d2h(h, a.data(), h->l.t, nw);
    if (!rc) rc = d2h(h, c.data(), h->l.n_acc, nw);
    if (!rc) rc = d2h(h, xp.data(), h->l.ex_prop, H);
    if (!rc) rc = d2h(h, xa.data(), h->l.ex_acc, H);
    if (!rc) rc = d2h(h, &r, h->l.round, 1);
    if (rc) return rc;
    if (rounds) *rounds = r;
    auto sum = [](const std::vector<unsigned long long> &v) {
        unsigned long long s = 0;
        for (auto x : v) s += x;
        return (uint64_t)s;
    };
    if (attempts) *attempts = sum(a);
    if (accepts) *accepts = sum(c);
    if (ex_prop) *ex_prop = sum(xp);
    if (ex_acc) *ex_acc = sum(xa);
    return REWL_OK;
}

// ------------------------------------------------------------------ batches
int rewl_batch_create(rewl_batch **out, const rewl_params *runs, int n_runs, int walkers_per_wave,
                      void *hip_stream)
{
    if (!out || !runs || n_runs < 1) return fail(REWL_EINVAL, "bad arguments");
    *out = nullptr;
    const int P = walkers_per_wave > 0 ? walkers_per_wave : 1;
    if (!valid_P(P)) return fail(REWL_EINVAL, "walkers_per_wave must be 1, 2, 4 or 8");
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    rewl_batch *b = new_batch(stream, P);
    if (!b) return fail(REWL_ENOMEM, "host allocation failed");
    b->owns_runs = true;
    for (int i = 0; i < n_runs; ++i) {
        rewl_ctx *h = nullptr;
        int rc = make_run(&h, &runs[i], nullptr, 0, stream);
        if (rc) {
            free_batch(b);
            return rc;
        }
        h->batch = b;
        b->runs.push_back(h);
    }
    int rc = rebuild(b);
    if (rc) {
        free_batch(b);
        return rc;
    }
    *out = b;
    return REWL_OK;
}

int rewl_batch_get_run(rewl_batch *b, int i, rewl_ctx **run)
{
    if (!b || !run || i < 0 || i >= (int)b->runs.size() || !b->runs[i])
        return fail(REWL_EINVAL, "bad batch or run index");
    *run = b->runs[i];
    return REWL_OK;
}

int rewl_batch_set_walkers_per_wave(rewl_batch *b, int walkers_per_wave)
{
    if (!b || !valid_P(walkers_per_wave)) return fail(REWL_EINVAL, "walkers_per_wave must be 1, 2, 4 or 8");
    int rc = bsync(b);
    if (rc) return rc;
    const int old = b->P;
    b->P = walkers_per_wave;
    b->dirty = true;
    rc = rebuild(b);
    if (rc) {
        b->P = old;
        b->dirty = true;
        (void)rebuild(b);
    }
    return rc;
}

int rewl_batch_set_form(rewl_batch *b, int form)
{
    if (!b || (form != REWL_FORM_ROUNDS && form != REWL_FORM_PERSISTENT))
        return fail(REWL_EINVAL, "form must be REWL_FORM_ROUNDS or REWL_FORM_PERSISTENT");
    int rc = bsync(b);
    if (rc) return rc;
    const int old = b->form;
    b->form = form;
    b->dirty = true;
    rc = rebuild(b);
    if (rc) {
        const std::string why(g_err);
        b->form = old;
        b->dirty = true;
        (void)rebuild(b);
        return fail(rc, why);
    }
    return REWL_OK;
}

int rewl_batch_set_graph(rewl_batch *b, int rounds_per_graph)
{
    if (!b || rounds_per_graph < 0) return fail(REWL_EINVAL, "bad arguments");
    int rc = bsync(b);
    if (rc) return rc;
    drop_graph(b);
    b->graph_rounds = rounds_per_graph;
    return REWL_OK;
}

int rewl_batch_step(rewl_batch *b, int64_t rounds)
{
    if (!b) return fail(REWL_EINVAL, "bad batch");
    Claim c(b);
    if (!c) return fail(REWL_EBUSY, "the batch is in use by another thread");
    return batch_step(b, rounds);
}

int rewl_batch_run(rewl_batch *b, int64_t max_rounds, int64_t *rounds_issued)
{
    if (!b) return fail(REWL_EINVAL, "bad batch");
    Claim c(b);
    if (!c) return fail(REWL_EBUSY, "the batch is in use by another thread");
    bool done = false;
    int rc = batch_run(b, max_rounds, &done);
    if (rc) return rc;
    if (rounds_issued) *rounds_issued = b->rounds;
    return done ? REWL_OK : REWL_NOT_CONVERGED;
}

int rewl_batch_done(rewl_batch *b, int *flags, int cap)
{
    if (!b || !flags) return fail(REWL_EINVAL, "bad arguments");
    Claim c(b);
    if (!c) return fail(REWL_EBUSY, "the batch is in use by another thread");
    std::vector<int> f;
    int rc = batch_done(b, f);
    if (rc) return rc;
    if (cap < (int)f.size()) return fail(REWL_EINVAL, "flags capacity below the number of runs");
    for (size_t i = 0; i < f.size(); ++i) flags[i] = f[i];
    return REWL_OK;
}

int rewl_batch_set_timing(rewl_batch *b, int on)
{
    if (!b) return fail(REWL_EINVAL, "bad batch");
    int rc = bsync(b);
    if (rc) return rc;
    b->timing = on != 0;
    b->sweep_ms = 0.0;
    b->sweep_launches = 0;
    return REWL_OK;
}

int rewl_batch_get_timing(rewl_batch *b, double *sweep_ms, int64_t *sweep_launches)
{
    if (!b) return fail(REWL_EINVAL, "bad batch");
    int rc = bsync(b);
    if (rc) return rc;
    if (sweep_ms) *sweep_ms = b->sweep_ms;
    if (sweep_launches) *sweep_launches = b->sweep_launches;
    return REWL_OK;
}

void rewl_batch_destroy(rewl_batch *b) { free_batch(b); }

// ------------------------------------------------- allocation-free entry point
int rewl_run_noalloc(const rewl_params *p, int64_t rounds, int32_t *E, int8_t *spins,
                     int64_t spins_stride, double *lng, uint32_t *H, int64_t bins_stride,
                     void *hip_stream)
{
    if (!p || rounds < 0 || !E || !spins || !lng || !H)
        return fail(REWL_EINVAL, "rewl_run_noalloc: NULL argument or negative rounds");
    if (p->n_windows < 1 || p->n_windows > kNoAllocMaxWindows)
        return fail(REWL_EINVAL, "rewl_run_noalloc: n_windows must be in [1, 64]");
    Geometry g;  // its window vectors stay empty: the windows live in lo / hi
    int64_t lo[kNoAllocMaxWindows], hi[kNoAllocMaxWindows];
    int rc = validate_into(p, g, lo, hi);
    if (rc) return rc;
    if (spins_stride < g.N || spins_stride % 4 || bins_stride < g.Wmax)
        return fail(REWL_EINVAL, "rewl_run_noalloc: spins_stride must be a multiple of 4 and "
                                 ">= the sites, bins_stride >= the widest window's bins");
    if ((uintptr_t)E % 4 || (uintptr_t)spins % 4 || (uintptr_t)lng % 8 || (uintptr_t)H % 4)
        return fail(REWL_EINVAL, "rewl_run_noalloc: misaligned output array");
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    // the scratch layout: launch tables, then the run's bookkeeping
    const size_t nw = (size_t)g.nw, h = (size_t)p->n_windows, N = (size_t)g.N;
    const bool glass = p->model == REWL_EA || p->model == REWL_EA3;
    const size_t j_raw = glass ? (size_t)bonds_per_site(p->model) * N : 0;
    const size_t j_words = (size_t)model_j_words(p->model);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + std::max<size_t>(bytes, 4), 256);
        return at;
    };
    const size_t o_desc = take(sizeof(RunDesc)), o_sweep = take(nw * sizeof(SweepItem));
    const size_t o_win = take(h * sizeof(WinItem)), o_pair = take(h / 2 * sizeof(WinItem));
    const size_t o_t = take(nw * 8), o_flat = take(nw * 4), o_acc = take(nw * 8);
    const size_t o_lnf = take(h * 8), o_done = take(h * 4), o_phase = take(h * 4);
    const size_t o_fin = take(h * 8), o_first = take(h * 8), o_lo = take(h * 4), o_hi = take(h * 4);
    const size_t o_exp = take(h * 8), o_exa = take(h * 8);
    const size_t o_jraw = take(j_raw), o_j4 = take(j_words * 4 * N);
    const size_t o_round = take(8), o_status = take(4);
    if (off > kNoAllocScratch)
        return fail(REWL_EINVAL, "rewl_run_noalloc: the run needs more than the 128 KiB of "
                                 "device scratch (about 36 bytes per walker, 80 per window, "
                                 "6 per site of a 2D glass, 11 of a 3D one)");
    void *base = nullptr;
    if (rewl_noalloc_scratch(&base)) return fail(REWL_EDEVICE, "rewl_run_noalloc: scratch lookup");
    char *sc = (char *)base;
    NoAllocSetup s{};
    RunDesc &d = s.d;
    fill_desc(d, p, g);
    d.Npad = (int)spins_stride;
    d.Wmax = (int)bins_stride;
    d.spins = spins;
    d.E = E;
    d.lng = lng;
    d.H = H;
    d.t = (unsigned long long *)(sc + o_t);
    d.flat = (int *)(sc + o_flat);
    d.n_acc = (unsigned long long *)(sc + o_acc);
    d.lnf = (double *)(sc + o_lnf);
    d.done = (int *)(sc + o_done);
    d.phase = (int *)(sc + o_phase);
    d.finish = (long long *)(sc + o_fin);
    d.first = (long long *)(sc + o_first);
    d.lo = (int *)(sc + o_lo);
    d.hi = (int *)(sc + o_hi);
    d.ex_prop = (unsigned long long *)(sc + o_exp);
    d.ex_acc = (unsigned long long *)(sc + o_exa);
    d.J4 = (uint32_t *)(sc + o_j4);
    d.round = (long long *)(sc + o_round);
    d.status = (int *)(sc + o_status);
    s.desc = (RunDesc *)(sc + o_desc);
    s.sweep = (SweepItem *)(sc + o_sweep);
    s.win = (WinItem *)(sc + o_win);
    s.pair = (WinItem *)(sc + o_pair);
    s.J_raw = (const int8_t *)(sc + o_jraw);
    s.lnf_init = p->lnf_init;
    for (int k = 0; k < p->n_windows; ++k) {
        s.lo[k] = (int)lo[k];
        s.hi[k] = (int)hi[k];
    }
    // the couplings as given (the caller's host array stays valid: this call
    // waits for the stream before it returns from the start-up)
    if (glass) HIP_TRY(hipMemcpyAsync(sc + o_jraw, p->couplings, j_raw, hipMemcpyHostToDevice, stream));
    if (rewl_launch_noalloc_setup(s, stream)) return fail(REWL_EDEVICE, "rewl_run_noalloc: set-up launch");
    if (rewl_launch_init(d, stream)) return fail(REWL_EDEVICE, "rewl_run_noalloc: start-up launch");
    int status = 0;
    HIP_TRY(hipMemcpyAsync(&status, d.status, 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (status) return fail(REWL_EINIT, "rewl_run_noalloc: a walker could not reach its window");
    BatchDev bd{};
    bd.runs = s.desc;
    bd.sweep = s.sweep;
    bd.win = s.win;
    bd.pair = s.pair;
    bd.n_runs = 1;
    bd.n_sweep = (int)nw;
    bd.n_win = (int)h;
    bd.n_pair = (int)(h / 2);
    bd.P = 1;
    bd.max_N = g.N;
    bd.max_W = g.Wmax;
    bd.j_words = (int)j_words;
    bd.region = (int)sweep_region(g.Wmax, g.N, kWave);
    for (int64_t r = 0; r < rounds; ++r) {
        rc = rewl_launch_round(bd, stream, nullptr, nullptr);
        if (rc) return fail(rc == -1 ? REWL_EINVAL : REWL_EDEVICE, "rewl_run_noalloc: round launch");
    }
    return REWL_OK;
}
// ------------------------------------------------------------------- server
}  // extern "C"

struct rewl_server {
    rewl_batch *batch = nullptr;        // running runs (slots reused)
    size_t budget = 0, used = 0;        // device bytes
    int rounds_per_tick = 8;
    int64_t next_id = 0;
    struct Pending {
        int64_t id;
        rewl_params p;
        std::vector<int8_t> couplings;
        std::vector<int64_t> wlo, whi;  // windows (explicit or equal partition)
        size_t bytes;
    };
    std::vector<Pending> queue;         // FIFO
    struct Finished {
        std::vector<double> lng;
        int64_t n_bins, e_min, e_step, rounds;
        int status;
        std::string what;  // why the run failed (status < 0)
    };
    std::map<int64_t, Finished> results;
    std::vector<int64_t> done_order;    // finished ids not yet popped
};

namespace {

// retire finished runs: stitch on the host, free their slabs and slots
int server_retire(rewl_server *s)
{
    rewl_batch *b = s->batch;
    std::vector<int> flags;
    int rc = batch_done(b, flags);
    if (rc) return rc;
    int live = 0;
    for (size_t i = 0; i < b->runs.size(); ++i) {
        rewl_ctx *h = b->runs[i];
        if (!h) continue;
        const int f = flags[live++];
        if (!f) continue;
        rewl_server::Finished fin;
        fin.lng.assign((size_t)h->g.B, 0.0);
        fin.status = get_lng_impl(h, fin.lng.data(), h->g.B, &fin.n_bins, &fin.e_min, &fin.e_step);
        std::vector<long long> fr(h->p.n_windows);
        rc = d2h(h, fr.data(), h->l.finish, fr.size());
        if (rc) return rc;
        fin.rounds = *std::max_element(fr.begin(), fr.end()) + 1;
        s->results[h->id] = std::move(fin);
        s->done_order.push_back(h->id);
        s->used -= h->l.total;
        free_run(h);
        b->runs[i] = nullptr;
        b->dirty = true;
    }
    return REWL_OK;
}

// largest walkers-per-wave <= want whose LDS footprint fits all runs
int fit_P(rewl_batch *b, int want, int extra_W, int extra_N, int extra_j_words)
{
    int max_W = extra_W, max_N = extra_N, jw = extra_j_words;
    for (rewl_ctx *h : b->runs) {
        if (!h) continue;
        max_W = std::max(max_W, h->g.Wmax);
        max_N = std::max(max_N, h->g.N);
        jw = std::max(jw, model_j_words(h->p.model));
    }
    for (int P = want; P >= 1; P /= 2)
        if (sweep_lds_bytes(P, max_W, max_N, jw) <= kMaxLds) return P;
    return 0;
}

// admit queued runs in arrival order while they fit the device budget
int server_admit(rewl_server *s, int want_P)
{
    rewl_batch *b = s->batch;
    while (!s->queue.empty()) {
        rewl_server::Pending &q = s->queue.front();
        if (s->used + q.bytes > s->budget) break;
        Geometry g;
        int rc = validate(&q.p, g);
        const int P = rc ? 1 : fit_P(b, want_P, g.Wmax, g.N, model_j_words(q.p.model));
        if (P == 0) break;
        rewl_ctx *h = nullptr;
        if (!rc) rc = make_run(&h, &q.p, nullptr, 0, b->stream);
        if (rc == REWL_EINIT || rc == REWL_EINVAL) {
            // the request itself cannot run (a walker cannot reach its
            // window): it finishes at once with that status, the others go on
            rewl_server::Finished fin;
            fin.n_bins = fin.e_min = fin.e_step = fin.rounds = 0;
            fin.status = rc;
            fin.what = rewl_last_error();
            s->results[q.id] = std::move(fin);
            s->done_order.push_back(q.id);
            s->queue.erase(s->queue.begin());
            continue;
        }
        if (rc) return rc;
        h->batch = b;
        h->id = q.id;
        h->admit_round = b->rounds;
        s->used += h->l.total;
        size_t slot = 0;
        while (slot < b->runs.size() && b->runs[slot]) ++slot;
        if (slot == b->runs.size()) b->runs.push_back(h);
        else b->runs[slot] = h;
        b->P = P;
        b->dirty = true;
        s->queue.erase(s->queue.begin());
    }
    return REWL_OK;
}

}  // namespace

extern "C" {

int rewl_server_create(rewl_server **out, size_t device_budget_bytes, int walkers_per_wave,
                       int rounds_per_tick, void *hip_stream)
{
    if (!out || device_budget_bytes == 0 || rounds_per_tick < 1 ||
        !valid_P(walkers_per_wave > 0 ? walkers_per_wave : 1))
        return fail(REWL_EINVAL, "bad server arguments");
    *out = nullptr;
    rewl_server *s = new (std::nothrow) rewl_server();
    if (!s) return fail(REWL_ENOMEM, "host allocation failed");
    s->batch = new_batch(reinterpret_cast<hipStream_t>(hip_stream),
                         walkers_per_wave > 0 ? walkers_per_wave : 1);
    if (!s->batch) {
        delete s;
        return fail(REWL_ENOMEM, "host allocation failed");
    }
    s->batch->owns_runs = true;
    s->budget = device_budget_bytes;
    s->rounds_per_tick = rounds_per_tick;
    *out = s;
    return REWL_OK;
}

int rewl_server_submit(rewl_server *s, const rewl_params *p, int64_t *id)
{
    if (!s || !p) return fail(REWL_EINVAL, "bad arguments");
    Geometry g;
    int rc = validate(p, g);
    if (rc) return rc;
    rewl_server::Pending q;
    q.id = s->next_id++;
    q.p = *p;
    q.wlo = g.lo;
    q.whi = g.hi;
    if (p->model == REWL_EA || p->model == REWL_EA3) {
        q.couplings.assign(p->couplings,
                           p->couplings + (size_t)bonds_per_site(p->model) * (size_t)g.N);
        q.p.couplings = q.couplings.data();
    } else {
        q.p.couplings = nullptr;
    }
    q.bytes = layout(p, g).total;
    if (q.bytes > s->budget) return fail(REWL_EBUSY, "run larger than the server's device budget");
    s->queue.push_back(std::move(q));
    // vector growth moved the copies; point each entry at its own again
    for (auto &e : s->queue) {
        if (e.p.model == REWL_EA || e.p.model == REWL_EA3) e.p.couplings = e.couplings.data();
        e.p.window_lo = e.wlo.data();
        e.p.window_hi = e.whi.data();
    }
    if (id) *id = s->queue.back().id;
    return REWL_OK;
}

int rewl_server_tick(rewl_server *s, int *n_running, int *n_queued)
{
    if (!s) return fail(REWL_EINVAL, "bad server");
    rewl_batch *b = s->batch;
    Claim c(b);
    if (!c) return fail(REWL_EBUSY, "the server is in use by another thread");
    int rc = server_retire(s);
    if (!rc) rc = server_admit(s, b->P > 0 ? b->P : 1);
    if (!rc) rc = batch_step(b, s->rounds_per_tick);
    if (rc) return rc;
    int running = 0;
    for (rewl_ctx *h : b->runs) running += h != nullptr;
    if (n_running) *n_running = running;
    if (n_queued) *n_queued = (int)s->queue.size();
    return REWL_OK;
}

int rewl_server_next_done(rewl_server *s, int64_t *id, int64_t *rounds)
{
    if (!s || !id) return fail(REWL_EINVAL, "bad arguments");
    if (s->done_order.empty()) return REWL_NOT_CONVERGED;
    *id = s->done_order.front();
    s->done_order.erase(s->done_order.begin());
    if (rounds) *rounds = s->results[*id].rounds;
    return REWL_OK;
}

int rewl_server_result(rewl_server *s, int64_t id, double *out, int64_t cap, int64_t *n_bins,
                       int64_t *e_min, int64_t *e_step)
{
    if (!s) return fail(REWL_EINVAL, "bad server");
    auto it = s->results.find(id);
    if (it == s->results.end()) return fail(REWL_EINVAL, "unknown or unfinished request id");
    const rewl_server::Finished &f = it->second;
    if (f.status < 0) return fail(f.status, f.what.c_str());
    if (n_bins) *n_bins = f.n_bins;
    if (e_min) *e_min = f.e_min;
    if (e_step) *e_step = f.e_step;
    if (out) {
        if (cap < f.n_bins) return fail(REWL_EINVAL, "output capacity below n_bins");
        std::memcpy(out, f.lng.data(), (size_t)f.n_bins * sizeof(double));
    }
    return f.status;
}

int rewl_server_release(rewl_server *s, int64_t id)
{
    if (!s) return fail(REWL_EINVAL, "bad server");
    s->results.erase(id);
    return REWL_OK;
}

void rewl_server_destroy(rewl_server *s)
{
    if (!s) return;
    free_batch(s->batch);
    delete s;
}

int rewl_selftest_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int n)
{
    if (n <= 0 || !ctr || !key || !out) return fail(REWL_EINVAL, "bad arguments");
    uint32_t *dc = nullptr, *dout = nullptr;
    hipError_t e = hipMalloc(&dc, (size_t)n * 16);
    if (e == hipSuccess) e = hipMalloc(&dout, (size_t)n * 16);
    if (e == hipSuccess) e = hipMemcpy(dc, ctr, (size_t)n * 16, hipMemcpyHostToDevice);
    int rc = (e == hipSuccess) ? rewl_launch_selftest_philox(dc, key[0], key[1], dout, n) : 0;
    if (e == hipSuccess && !rc) e = hipMemcpy(out, dout, (size_t)n * 16, hipMemcpyDeviceToHost);
    if (dc) (void)hipFree(dc);
    if (dout) (void)hipFree(dout);
    if (e != hipSuccess) return hip_fail(e, "selftest");
    return rc ? fail(rc, "selftest launch failed") : REWL_OK;
}

int rewl_selftest_ln_u(const uint32_t *words, double *out, int n)
{
    if (n <= 0 || !words || !out) return fail(REWL_EINVAL, "bad arguments");
    uint32_t *dw = nullptr;
    double *dout = nullptr;
    hipError_t e = hipMalloc(&dw, (size_t)n * 8);
    if (e == hipSuccess) e = hipMalloc(&dout, (size_t)n * 8);
    if (e == hipSuccess) e = hipMemcpy(dw, words, (size_t)n * 8, hipMemcpyHostToDevice);
    int rc = (e == hipSuccess) ? rewl_launch_selftest_ln_u(dw, dout, n) : 0;
    if (e == hipSuccess && !rc) e = hipMemcpy(out, dout, (size_t)n * 8, hipMemcpyDeviceToHost);
    if (dw) (void)hipFree(dw);
    if (dout) (void)hipFree(dout);
    if (e != hipSuccess) return hip_fail(e, "selftest");
    return rc ? fail(rc, "selftest launch failed") : REWL_OK;
}

}  // extern "C"
