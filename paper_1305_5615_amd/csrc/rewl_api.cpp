// rewl_api.cpp -- host runtime and C ABI of the REWL library (include/rewl.h).
//
// The host validates parameters, lays the energy range out in windows,
// carves one device allocation into the run's arrays, queues the kernels of
// rewl_kernels.hip on the run's stream and, at the end, joins the window pieces
// of ln g.  It never computes a Monte Carlo step itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rewl.h"
#include "rewl_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(REWL_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                  \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

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
int make_windows(int64_t B, int h, double o, std::vector<int64_t> &lo, std::vector<int64_t> &hi)
{
    lo.assign(h, 0);
    hi.assign(h, 0);
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

int validate(const rewl_params *p, Geometry &g)
{
    if (!p) return fail(REWL_EINVAL, "params is NULL");
    if (p->model < 0 || p->model > 2) return fail(REWL_EINVAL, "unknown model");
    if (p->L < 3 || p->L > 256) return fail(REWL_EINVAL, "L must be in [3, 256]");
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
    const int64_t N = (int64_t)p->L * p->L;
    g.N = (int)N;
    g.step = (p->model == REWL_POTTS) ? 1 : 4;
    const int64_t lo_full = -2 * N, hi_full = (p->model == REWL_POTTS) ? 0 : 2 * N;
    int64_t cls = 0;
    if (p->model == REWL_EA) {
        if (!p->couplings) return fail(REWL_EINVAL, "EA model needs couplings");
        int64_t n_neg = 0;
        for (int64_t i = 0; i < 2 * N; ++i) {
            const int8_t c = p->couplings[i];
            if (c != 1 && c != -1) return fail(REWL_EINVAL, "couplings must be +-1");
            n_neg += c < 0;
        }
        cls = -2 * N + 2 * n_neg;
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
    int rc = make_windows(g.B, p->n_windows, p->overlap, g.lo, g.hi);
    if (rc) return rc;
    g.Wmax = 0;
    for (int k = 0; k < p->n_windows; ++k)
        g.Wmax = std::max<int>(g.Wmax, (int)(g.hi[k] - g.lo[k] + 1));
    g.nw = p->n_windows * p->walkers_per_window;
    g.Npad = (int)align_up((size_t)N, 16);
    if (sweep_lds_bytes(p->model, g.Wmax, g.N) > kMaxLds)
        return fail(REWL_EINVAL, "one walker's window does not fit the LDS of a CU");
    return REWL_OK;
}

// Byte offsets of the arrays inside the device allocation.
struct Layout {
    size_t spins, E, t, flat, lng, H, n_acc, lnf, done, finish, lo, hi, ex_prop, ex_acc, J4,
        status, total;
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
    l.finish = take(h * 8);
    l.lo = take(h * 4);
    l.hi = take(h * 4);
    l.ex_prop = take(h * 8);
    l.ex_acc = take(h * 8);
    l.J4 = take(p->model == REWL_EA ? (size_t)g.N * 4 : 4);
    l.status = take(4);
    l.total = off;
    return l;
}

}  // namespace

struct rewl_ctx {
    rewl_params p{};
    std::vector<int8_t> couplings;
    Geometry g;
    Layout l{};
    void *base = nullptr;
    bool owns = false;
    hipStream_t stream = nullptr;
    RunDev dev{};
    int64_t rounds = 0;
    int *pinned = nullptr; // done flags, polled by rewl_run
    // optional timing of the sweep launches with events on the run's stream
    bool timing = false;
    std::vector<hipEvent_t> ev_free, ev_pending; // pending: start/stop pairs
    double sweep_ms = 0.0;
    int64_t sweep_launches = 0;
};

namespace {

// Fold finished start/stop event pairs into the sweep time (stream synced).
int collect_timing(rewl_ctx *h)
{
    for (size_t i = 0; i + 1 < h->ev_pending.size(); i += 2) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, h->ev_pending[i], h->ev_pending[i + 1]));
        h->sweep_ms += ms;
        h->sweep_launches += 1;
        h->ev_free.push_back(h->ev_pending[i]);
        h->ev_free.push_back(h->ev_pending[i + 1]);
    }
    h->ev_pending.clear();
    return REWL_OK;
}

int sync(rewl_ctx *h)
{
    HIP_TRY(hipStreamSynchronize(h->stream));
    return h->timing ? collect_timing(h) : REWL_OK;
}

int take_event(rewl_ctx *h, hipEvent_t *e)
{
    if (h->ev_free.empty()) {
        hipEvent_t ev;
        HIP_TRY(hipEventCreate(&ev));
        h->ev_free.push_back(ev);
    }
    *e = h->ev_free.back();
    h->ev_free.pop_back();
    h->ev_pending.push_back(*e);
    return REWL_OK;
}

template <class T>
int d2h(rewl_ctx *h, T *dst, size_t off, size_t count)
{
    HIP_TRY(hipMemcpyAsync(dst, (char *)h->base + off, count * sizeof(T), hipMemcpyDeviceToHost,
                           h->stream));
    return sync(h);
}

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
    if (h->p.model != REWL_EA && g.full_lo && std::isfinite(out[0])) {
        ref = out[0];
        target = std::log(h->p.model == REWL_POTTS ? (double)h->p.q : 2.0);
    } else if (h->p.model == REWL_EA && g.full_lo && g.full_hi) {
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

int all_done(rewl_ctx *h, bool *done)
{
    const int n = h->p.n_windows;
    HIP_TRY(hipMemcpyAsync(h->pinned, (char *)h->base + h->l.done, (size_t)n * 4,
                           hipMemcpyDeviceToHost, h->stream));
    int rc = sync(h);
    if (rc) return rc;
    bool all = true;
    for (int k = 0; k < n; ++k) all = all && h->pinned[k] != 0;
    *done = all;
    return REWL_OK;
}

}  // namespace

extern "C" {

const char *rewl_last_error(void) { return g_err.c_str(); }

int rewl_footprint(const rewl_params *p, size_t *device_bytes, size_t *lds_bytes)
{
    Geometry g;
    int rc = validate(p, g);
    if (rc) return rc;
    if (device_bytes) *device_bytes = layout(p, g).total;
    if (lds_bytes) *lds_bytes = sweep_lds_bytes(p->model, g.Wmax, g.N);
    return REWL_OK;
}

void rewl_destroy(rewl_ctx *h)
{
    if (!h) return;
    if (h->stream || h->base) (void)hipStreamSynchronize(h->stream);
    if (h->owns && h->base) (void)hipFree(h->base);
    if (h->pinned) (void)hipHostFree(h->pinned);
    for (hipEvent_t e : h->ev_free) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->ev_pending) (void)hipEventDestroy(e);
    delete h;
}

int rewl_create_ex(rewl_ctx **out, const rewl_params *p, void *device_buffer, size_t buffer_bytes,
                   void *hip_stream)
{
    if (!out) return fail(REWL_EINVAL, "out is NULL");
    *out = nullptr;
    Geometry g;
    int rc = validate(p, g);
    if (rc) return rc;
    rewl_ctx *h = new (std::nothrow) rewl_ctx();
    if (!h) return fail(REWL_ENOMEM, "host allocation failed");
    h->p = *p;
    h->g = g;
    h->l = layout(p, g);
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (p->model == REWL_EA) {
        h->couplings.assign(p->couplings, p->couplings + 2 * (size_t)g.N);
        h->p.couplings = h->couplings.data();
    } else {
        h->p.couplings = nullptr;
    }
    auto bail = [&](int code) {
        rewl_destroy(h);
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
    if (hipHostMalloc((void **)&h->pinned, (size_t)p->n_windows * 4) != hipSuccess)
        return bail(fail(REWL_ENOMEM, "pinned allocation failed"));

    char *b = (char *)h->base;
    RunDev &d = h->dev;
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
    d.S = p->attempts_per_round;
    d.key0 = (uint32_t)p->seed;
    d.key1 = (uint32_t)(p->seed >> 32);
    d.flat_p = p->flatness;
    d.lnf_final = p->lnf_final;
    d.spins = (int8_t *)(b + h->l.spins);
    d.E = (int *)(b + h->l.E);
    d.t = (unsigned long long *)(b + h->l.t);
    d.flat = (int *)(b + h->l.flat);
    d.lng = (double *)(b + h->l.lng);
    d.H = (uint32_t *)(b + h->l.H);
    d.n_acc = (unsigned long long *)(b + h->l.n_acc);
    d.lnf = (double *)(b + h->l.lnf);
    d.done = (int *)(b + h->l.done);
    d.finish = (long long *)(b + h->l.finish);
    d.lo = (int *)(b + h->l.lo);
    d.hi = (int *)(b + h->l.hi);
    d.ex_prop = (unsigned long long *)(b + h->l.ex_prop);
    d.ex_acc = (unsigned long long *)(b + h->l.ex_acc);
    d.J4 = (uint32_t *)(b + h->l.J4);
    d.status = (int *)(b + h->l.status);

    // host-side images of the small per-window arrays and the EA couplings
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
    }
    hipError_t e = hipMemsetAsync(h->base, 0, h->l.total, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d.lnf, lnf.data(), H * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d.finish, fin.data(), H * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.lo, lo.data(), H * 4, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.hi, hi.data(), H * 4, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && !J4.empty())
        e = hipMemcpyAsync(d.J4, J4.data(), (size_t)N * 4, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "upload of the run parameters"));
    rc = rewl_launch_init(d, h->stream);
    if (rc) return bail(fail(rc, "launch of the start-up kernel failed"));
    int status = 0;
    e = hipMemcpyAsync(&status, d.status, 4, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "start-up"));
    if (status) return bail(fail(REWL_EINIT, "a walker could not reach its window"));
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
    return rewl_create_ex(out, &p, nullptr, 0, nullptr);
}

int rewl_step(rewl_ctx *h, int64_t rounds)
{
    if (!h || rounds < 0) return fail(REWL_EINVAL, "bad handle or negative rounds");
    for (int64_t i = 0; i < rounds; ++i) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (h->timing) {
            int rc = take_event(h, &e0);
            if (!rc) rc = take_event(h, &e1);
            if (rc) return rc;
        }
        int rc = rewl_launch_round(h->dev, h->rounds, h->stream, e0, e1);
        if (rc) return fail(rc, "kernel launch failed");
        h->rounds += 1;
    }
    return REWL_OK;
}

int rewl_set_timing(rewl_ctx *h, int on)
{
    if (!h) return fail(REWL_EINVAL, "bad handle");
    int rc = sync(h);
    if (rc) return rc;
    h->timing = on != 0;
    h->sweep_ms = 0.0;
    h->sweep_launches = 0;
    return REWL_OK;
}

int rewl_get_timing(rewl_ctx *h, double *sweep_ms, int64_t *sweep_launches)
{
    if (!h) return fail(REWL_EINVAL, "bad handle");
    int rc = sync(h);
    if (rc) return rc;
    if (sweep_ms) *sweep_ms = h->sweep_ms;
    if (sweep_launches) *sweep_launches = h->sweep_launches;
    return REWL_OK;
}

int rewl_run(rewl_ctx *h, int64_t max_rounds, int64_t *rounds_done)
{
    if (!h) return fail(REWL_EINVAL, "bad handle");
    bool done = false;
    int rc = all_done(h, &done);
    if (rc) return rc;
    int64_t issued = 0, chunk = 4;
    while (!done && (max_rounds < 0 || issued < max_rounds)) {
        int64_t n = chunk;
        if (max_rounds >= 0) n = std::min(n, max_rounds - issued);
        rc = rewl_step(h, n);
        if (rc) return rc;
        issued += n;
        rc = all_done(h, &done);
        if (rc) return rc;
        chunk = std::min<int64_t>(chunk * 2, 64);
    }
    if (rounds_done) {
        *rounds_done = h->rounds;
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
    bool done = false;
    rc = all_done(h, &done);
    if (rc) return rc;
    return done ? REWL_OK : REWL_NOT_CONVERGED;
}

int rewl_get_info(rewl_ctx *h, int64_t *n_bins, int64_t *e_min, int64_t *e_step, int *n_windows,
                  int *walkers_per_window, int *n_sites, int64_t *rounds, uint64_t *attempts,
                  uint64_t *accepts, uint64_t *ex_prop, uint64_t *ex_acc)
{
    if (!h) return fail(REWL_EINVAL, "bad handle");
    if (n_bins) *n_bins = h->g.B;
    if (e_min) *e_min = h->g.e_min;
    if (e_step) *e_step = h->g.step;
    if (n_windows) *n_windows = h->p.n_windows;
    if (walkers_per_window) *walkers_per_window = h->p.walkers_per_window;
    if (n_sites) *n_sites = h->g.N;
    if (rounds) *rounds = h->rounds;
    const size_t nw = (size_t)h->g.nw, H = (size_t)h->p.n_windows;
    std::vector<unsigned long long> a(nw), c(nw), xp(H), xa(H);
    int rc = d2h(h, a.data(), h->l.t, nw);
    if (!rc) rc = d2h(h, c.data(), h->l.n_acc, nw);
    if (!rc) rc = d2h(h, xp.data(), h->l.ex_prop, H);
    if (!rc) rc = d2h(h, xa.data(), h->l.ex_acc, H);
    if (rc) return rc;
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

int rewl_selftest_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int n)
{
    if (n <= 0 || !ctr || !key || !out) return fail(REWL_EINVAL, "bad arguments");
    uint32_t *dc = nullptr, *dout = nullptr;
    HIP_TRY(hipMalloc(&dc, (size_t)n * 16));
    HIP_TRY(hipMalloc(&dout, (size_t)n * 16));
    HIP_TRY(hipMemcpy(dc, ctr, (size_t)n * 16, hipMemcpyHostToDevice));
    int rc = rewl_launch_selftest_philox(dc, key[0], key[1], dout, n);
    if (!rc) HIP_TRY(hipMemcpy(out, dout, (size_t)n * 16, hipMemcpyDeviceToHost));
    (void)hipFree(dc);
    (void)hipFree(dout);
    return rc ? fail(rc, "selftest launch failed") : REWL_OK;
}

int rewl_selftest_ln_u(const uint32_t *words, double *out, int n)
{
    if (n <= 0 || !words || !out) return fail(REWL_EINVAL, "bad arguments");
    uint32_t *dw = nullptr;
    double *dout = nullptr;
    HIP_TRY(hipMalloc(&dw, (size_t)n * 8));
    HIP_TRY(hipMalloc(&dout, (size_t)n * 8));
    HIP_TRY(hipMemcpy(dw, words, (size_t)n * 8, hipMemcpyHostToDevice));
    int rc = rewl_launch_selftest_ln_u(dw, dout, n);
    if (!rc) HIP_TRY(hipMemcpy(out, dout, (size_t)n * 8, hipMemcpyDeviceToHost));
    (void)hipFree(dw);
    (void)hipFree(dout);
    return rc ? fail(rc, "selftest launch failed") : REWL_OK;
}

}  // extern "C"
