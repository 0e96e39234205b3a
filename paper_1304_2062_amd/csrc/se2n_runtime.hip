// Host runtime of libse2n: plans, argument validation, the per-frequency
// propagator cache, workspace layout and the C ABI of include/se2n.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/se2n.h"
#include "se2n_internal.hpp"
#include "se2n_host.hpp"

using namespace se2n;

namespace se2n {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(SE2N_EHIP, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_last_error.clear(); }

// Allocation-failure injection: -1 disables it; k >= 0 lets k allocations
// succeed and fails every later one until reset.
std::atomic<long> g_alloc_budget{-1};

static bool alloc_allowed() {
    long k = g_alloc_budget.load();
    while (k >= 0) {
        if (k == 0) return false;
        if (g_alloc_budget.compare_exchange_weak(k, k - 1)) return true;
    }
    return true;
}

hipError_t dev_malloc(void** p, size_t bytes) {
    if (!alloc_allowed()) return hipErrorOutOfMemory;
    return hipMalloc(p, bytes);
}

hipError_t pinned_malloc(void** p, size_t bytes) {
    if (!alloc_allowed()) return hipErrorOutOfMemory;
    return hipHostMalloc(p, bytes, hipHostMallocDefault);
}

bool is_2a3b(int M, int* twos, int* threes) {
    int a = 0, b = 0, m = M;
    while (m % 2 == 0) { m /= 2; ++a; }
    while (m % 3 == 0) { m /= 3; ++b; }
    if (twos) *twos = a;
    if (threes) *threes = b;
    return m == 1;
}

// Radix sequence of a length-L transform, L = 2^a 3^b dividing M: radix 8
// where possible, then 4 (or 4,4 in place of 8,2), then radix 3.
FftPlan make_fft_plan(int L, int M) {
    FftPlan p{};
    p.L = L;
    int a = 0, b = 0;
    is_2a3b(L, &a, &b);
    int rad[16], n = 0;
    int q = a / 3, r = a % 3;
    if (r == 1 && q >= 1) {
        for (int i = 0; i < q - 1; ++i) rad[n++] = 8;
        rad[n++] = 4;
        rad[n++] = 4;
    } else {
        for (int i = 0; i < q; ++i) rad[n++] = 8;
        if (r == 1) rad[n++] = 2;
        if (r == 2) rad[n++] = 4;
    }
    for (int i = 0; i < b; ++i) rad[n++] = 3;
    p.nstages = n;
    int Ns = 1;
    for (int i = 0; i < n; ++i) {
        FftStage& s = p.st[i];
        s.radix = rad[i];
        s.nb = L / rad[i];
        s.Ns = Ns;
        s.twstep = M / (Ns * rad[i]);
        s.inv_nb = 1.0f / (float)s.nb;
        s.inv_Ns = 1.0f / (float)Ns;
        s.lg_Ns = (Ns & (Ns - 1)) == 0 ? __builtin_ctz((unsigned)Ns) : -1;
        Ns *= rad[i];
    }
    return p;
}

// Quarter table w_M^m = exp(-2 pi i m / M), m in [0, M/4], evaluated in
// extended precision before rounding to R.
template <class R>
std::vector<C2<R>> quarter_twiddles(int M) {
    const int n = M / 4 + 1;
    std::vector<C2<R>> h(n);
    for (int m = 0; m < n; ++m) {
        const long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)M;
        h[m].x = (R)(double)cosl(a);
        h[m].y = (R)(double)(-sinl(a));
    }
    return h;
}
template std::vector<C2<float>> quarter_twiddles<float>(int);
template std::vector<C2<double>> quarter_twiddles<double>(int);

// The orientation step's two Fourier multipliers per axis: the Gaussian
// G_k = exp(-2 pi^2 sigma^2 kbar^2 / M^2) (kbar = k wrapped to [-M/2, M/2))
// and G_k times the central-difference symbol i sqrt(M) sin(2 pi k/M).
// Their inverse DFTs, in FP64, are the smoothing kernel
//     g[x] = (1/M) sum_k G_k cos(2 pi k x/M)
// and the smoothed difference kernel
//     d[x] = -(sqrt(M)/M) sum_k sin(2 pi k/M) G_k sin(2 pi k x/M),
// (even and odd in x).  The convolution out = d (*) in becomes the
// correlation out[y] = sum_j d[-j] in[y + j], hence the reflected taps.
int orient_stencil_taps(int M, double sigma, OrientTaps* taps) {
    const double two_pi = 6.283185307179586476925;
    std::vector<double> G(M), c(M), s(M), g(M, 0.0), d(M, 0.0);
    for (int k = 0; k < M; ++k) {
        const double kb = (double)(((k + M / 2) % M) - M / 2);
        G[k] = std::exp(-0.5 * two_pi * two_pi * sigma * sigma * kb * kb / ((double)M * M));
        c[k] = std::cos(two_pi * k / M);
        s[k] = std::sin(two_pi * k / M);
    }
    // the M/2 + 1 sums are independent: large sides split them over a few
    // host threads (each sum is the same sequence of operations, so the taps
    // do not depend on the split)
    auto sums = [&](int x0, int x1) {
        for (int x = x0; x < x1; ++x) {
            double sg = 0.0, sd = 0.0;
            int idx = 0;  // k x mod M
            for (int k = 0; k < M; ++k) {
                sg += G[k] * c[idx];
                sd += s[k] * G[k] * s[idx];
                idx += x;
                if (idx >= M) idx -= M;
            }
            g[x] = sg / M;
            d[x] = -std::sqrt((double)M) / M * sd;
            if (x > 0 && x < M - x) {
                g[M - x] = g[x];
                d[M - x] = -d[x];
            }
        }
    };
    const int nx = M / 2 + 1;
    const unsigned hw = std::thread::hardware_concurrency();
    const int nt = M < 512 ? 1 : (int)std::min<unsigned>(8u, hw ? hw : 1u);
    if (nt <= 1) {
        sums(0, nx);
    } else {
        std::vector<std::thread> pool;
        for (int t = 0; t < nt; ++t) {
            const int x0 = (int)((long)nx * t / nt), x1 = (int)((long)nx * (t + 1) / nt);
            pool.emplace_back(sums, x0, x1);
        }
        for (auto& th : pool) th.join();
    }
    // absolute mass at circular distance r, then the smallest radius whose
    // dropped tail is below 2^-26 of the kernel's absolute sum
    const int H = M / 2;
    std::vector<double> mg(H + 1), md(H + 1);
    double tg = 0.0, td = 0.0;
    for (int r = 0; r <= H; ++r) {
        mg[r] = std::fabs(g[r]) + ((r > 0 && r < M - r) ? std::fabs(g[M - r]) : 0.0);
        md[r] = std::fabs(d[r]) + ((r > 0 && r < M - r) ? std::fabs(d[M - r]) : 0.0);
        tg += mg[r];
        td += md[r];
    }
    const double tol = std::ldexp(1.0, -26);
    int need = H;  // the whole circle
    double tail_g = 0.0, tail_d = 0.0;
    for (int R = H; R >= 1; --R) {
        tail_g += mg[R];
        tail_d += md[R];
        if (tail_g > tol * tg || tail_d > tol * td) break;
        need = R - 1;
    }
    const bool circle = need >= H;
    int rad = 0;
    for (int rv : kOrientRadii) {
        if (rv >= (circle ? H : need)) {
            rad = rv;
            break;
        }
    }
    if (rad == 0) return 0;
    std::memset(taps, 0, sizeof *taps);
    const int lo = circle ? -(H - 1) : -need;
    const int hi = circle ? H : need;
    for (int j = lo; j <= hi; ++j) {
        const int m = ((-j) % M + M) % M;
        taps->g[j + rad] = (float)g[m];
        taps->d[j + rad] = (float)d[m];
    }
    return rad;
}

int orient_stencil_taps_cached(int M, double sigma, OrientTaps* taps) {
    static std::mutex mu;
    static std::map<std::pair<int, uint64_t>, std::pair<int, OrientTaps>> memo;
    uint64_t bits;
    std::memcpy(&bits, &sigma, sizeof bits);
    const auto key = std::make_pair(M, bits);
    std::lock_guard<std::mutex> lock(mu);
    auto it = memo.find(key);
    if (it == memo.end()) {
        std::pair<int, OrientTaps> v;
        v.first = orient_stencil_taps(M, sigma, &v.second);
        it = memo.emplace(key, v).first;
    }
    if (taps) *taps = it->second.second;
    return it->second.first;
}

}  // namespace se2n

namespace {

struct CacheKey {
    double T, beta;
    int n, scheme;
    bool operator==(const CacheKey& o) const {
        return std::memcmp(&T, &o.T, sizeof T) == 0 && std::memcmp(&beta, &o.beta, sizeof beta) == 0 &&
               n == o.n && scheme == o.scheme;
    }
};

struct CacheEntry {
    CacheKey key;
    void* dptr;
    size_t bytes;
};

}  // namespace

struct se2n_plan_s {
    int M = 0, N = 0;
    se2n_dtype dt = SE2N_F32;
    int device = 0;
    void* tw = nullptr;  // w_M^m, m <= M/4, in the plan dtype
    FftPlan planH{}, planM{};
    LaunchGeom geom{};
    std::list<CacheEntry> cache;  // most recently used first
    // orientation stencil taps for the last sigma (FP32 plans); radius 0 = FFT route
    bool ot_valid = false;
    double ot_sigma = 0.0;
    int ot_radius = 0;
    OrientTaps ot{};
    size_t cache_bytes = 0;
    size_t cache_limit = (size_t)16 << 30;
    std::mutex mu;
    bool alive = true;
    // kernel timing
    bool prof_on = false;
    bool prof_hold = false;  // set while a call that may not create events runs
    // SE2N_KEEP_NEGLIGIBLE set at plan creation: no class is taken as
    // negligible (measurement of the passes without the skip)
    bool keep_negligible = false;
    // solver schedule of the CN diffusion: collapsed propagator or iterated
    // steps (se2n_set_schedule); requests per uncached key for the automatic choice
    se2n_schedule schedule = SE2N_SCHEDULE_PROPAGATOR;
    se2n_schedule last_schedule = SE2N_SCHEDULE_AUTO;
    std::map<std::tuple<uint64_t, uint64_t, int>, int> misses;
    struct ProfRec {
        const char* name;
        hipEvent_t a, b;
    };
    std::vector<ProfRec> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    std::map<std::string, std::pair<int, double>> prof_acc;

    size_t real_size() const { return dt == SE2N_F32 ? 4 : 8; }
    size_t cplx_size() const { return 2 * real_size(); }
    int K() const { return M / 2 + 1; }
    size_t spec_bytes() const { return align256((size_t)N * K() * M * cplx_size()); }
    // second spectrum: the inverse column pass's result in the row-blocked
    // layout, where the compiled passes support it (row_blocked)
    bool blk_ok = false;
    size_t blk_bytes() const { return blk_ok ? spec_bytes() : 0; }
    size_t enc_bytes() const { return align256((size_t)M * M * real_size()); }
    size_t rmap_bytes() const { return align256((size_t)M * M); }
    size_t workspace() const { return spec_bytes() + blk_bytes() + enc_bytes() + rmap_bytes(); }
    size_t workspace_unblocked() const { return spec_bytes() + enc_bytes() + rmap_bytes(); }
    // restoration: the above, the real volume, h, h_ref and the join map
    size_t vol_bytes() const { return align256((size_t)N * M * M * real_size()); }
    size_t restore_workspace() const {
        return workspace() + vol_bytes() + 2 * enc_bytes() + align256((size_t)M * M * sizeof(int16_t));
    }
    // class-major propagators + one flag byte per class (padded rows)
    size_t table_bytes() const { return se2n::table_bytes(M, N, (int)real_size()); }
};

namespace {

hipEvent_t prof_event(se2n_plan p) {
    if (!p->prof_pool.empty()) {
        hipEvent_t e = p->prof_pool.back();
        p->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one launch with events on its stream while timing is enabled.
struct ProfScope {
    se2n_plan p;
    const char* name;
    hipStream_t st;
    hipEvent_t a = nullptr;
    ProfScope(se2n_plan p_, const char* name_, hipStream_t st_) : p(p_), name(name_), st(st_) {
        if (p->prof_on && !p->prof_hold) {
            a = prof_event(p);
            if (a) (void)hipEventRecord(a, st);
        }
    }
    ~ProfScope() {
        if (a) {
            hipEvent_t b = prof_event(p);
            if (b) {
                (void)hipEventRecord(b, st);
                p->prof_pending.push_back({name, a, b});
            } else {
                p->prof_pool.push_back(a);
            }
        }
    }
};

#define SE2N_TIMED(plan, name, st, call, what) \
    do {                                       \
        ProfScope ps_(plan, name, st);         \
        SE2N_HIP(call, what);                  \
    } while (0)

template <class R>
LaunchGeom make_geom(int M, int N, int num_cu) {
    const GeomCore c = geom_core<R>(M);
    LaunchGeom g{};
    g.rows = c.rows;
    g.row_threads = c.row_threads;
    g.row_ept = c.row_ept;
    g.cols = c.cols;
    g.col_threads = c.col_threads;
    g.col_ept = c.col_ept;
    g.ocols = c.ocols;
    g.ocol_threads = c.ocol_threads;
    g.ocol_ept = c.ocol_ept;
    g.pcols = c.pcols;
    g.pcol_threads = c.pcol_threads;
    g.pcol_ept = c.pcol_ept;
    g.tw_full = c.tw_full;
    g.tw_full_col = c.tw_full_col;
    const int row_blocks = M / c.rows;
    // slice groups of the row passes: the fewest that give every compute unit
    // a workgroup (a row pass workgroup fills a CU's registers); fewer groups
    // read the lift sources fewer times and combine fewer maxima through
    // atomics (SE2N_ROW_GROUPS / SE2N_INV_GROUPS override the choice)
    int groups = (num_cu + row_blocks - 1) / row_blocks;
    int inv_groups = groups;
    if (const char* v = std::getenv("SE2N_ROW_GROUPS")) groups = std::atoi(v);
    if (const char* v = std::getenv("SE2N_INV_GROUPS")) inv_groups = std::atoi(v);
    groups = std::max(1, std::min(groups, N));
    inv_groups = std::max(1, std::min(inv_groups, N));
    g.row_slices = (N + groups - 1) / groups;
    g.inv_slices = (N + inv_groups - 1) / inv_groups;
    g.xcd_pair = 1;
    if (const char* v = std::getenv("SE2N_TW_FULL")) g.tw_full = std::atoi(v) != 0 && g.tw_full;
    if (const char* v = std::getenv("SE2N_XCD_PAIR")) g.xcd_pair = std::atoi(v);
    g.static_ok = std::getenv("SE2N_NO_STATIC") == nullptr;
    return g;
}

// Invariants the kernels rely on; a violation is a library bug, reported as
// SE2N_EUNSUPPORTED instead of launching.
template <class R>
int check_geom(const LaunchGeom& g, int M) {
    const int H = M / 2;
    const size_t cs = sizeof(C2<R>);
    const size_t lds_max = 160 * 1024;
    const bool ok =
        g.rows >= 1 && (g.rows & (g.rows - 1)) == 0 && M % g.rows == 0 && g.row_slices >= 1 &&
        g.inv_slices >= 1 && g.row_threads >= 1 && g.row_threads <= 1024 && g.row_threads % g.rows == 0 &&
        g.rows * H <= g.row_ept * g.row_threads && g.cols >= 1 && g.col_threads >= 1 && g.col_threads <= 1024 &&
        g.cols * M <= g.col_ept * g.col_threads && g.ocols >= 1 && g.ocol_threads >= 1 && g.ocol_threads <= 1024 &&
        2 * g.ocols * M <= g.ocol_ept * g.ocol_threads &&
        (size_t)(tw_elems(M, g.tw_full) + lds_padded_size(g.rows * (H + 2))) * cs <= lds_max &&
        (size_t)(tw_elems(M, g.tw_full_col) + lds_padded_size(2 * g.ocols * M)) * cs <= lds_max &&
        (size_t)(tw_elems(M, g.tw_full_col) + lds_padded_size(g.cols * M)) * cs <= lds_max &&
        g.pcols >= 2 && g.pcols % 2 == 0 && g.pcol_threads >= 1 && g.pcol_threads <= 1024 &&
        g.pcols * M <= g.pcol_ept * g.pcol_threads &&
        (size_t)(tw_elems(M, false) + lds_padded_size(g.pcols * M)) * cs <= lds_max;
    return ok ? SE2N_OK : fail(SE2N_EUNSUPPORTED, "internal launch geometry invalid for M=%d", M);
}

int check_plan(se2n_plan p) {
    if (!p) return fail(SE2N_EINVAL, "plan is NULL");
    if (!p->alive) return fail(SE2N_ESTATE, "plan was destroyed");
    return SE2N_OK;
}

int check_diffusion_params(double T, double beta, int n_steps, se2n_scheme scheme) {
    if (!(T >= 0.0) || !std::isfinite(T)) return fail(SE2N_EINVAL, "T must be finite and >= 0 (got %g)", T);
    if (!(beta >= 0.0) || !std::isfinite(beta))
        return fail(SE2N_EINVAL, "beta must be finite and >= 0 (got %g)", beta);
    if (scheme != SE2N_CN && scheme != SE2N_EXACT) return fail(SE2N_EINVAL, "unknown scheme %d", (int)scheme);
    if (scheme == SE2N_CN && n_steps < 1) return fail(SE2N_EINVAL, "n_steps must be >= 1 (got %d)", n_steps);
    return SE2N_OK;
}

// Look up (or compute on `st`) the propagator table for the given parameters.
int get_propagators(se2n_plan p, double T, double beta, int n_steps, se2n_scheme scheme, hipStream_t st,
                    const void** out) {
    CacheKey key{T, beta, scheme == SE2N_CN ? n_steps : 0, (int)scheme};
    std::lock_guard<std::mutex> lock(p->mu);
    for (auto it = p->cache.begin(); it != p->cache.end(); ++it) {
        if (it->key == key) {
            p->cache.splice(p->cache.begin(), p->cache, it);
            *out = p->cache.front().dptr;
            return SE2N_OK;
        }
    }
    const size_t bytes = p->table_bytes();
    // evict least recently used entries to stay under the limit
    while (!p->cache.empty() && p->cache_bytes + bytes > p->cache_limit) {
        SE2N_HIP(hipStreamSynchronize(st), "hipStreamSynchronize before cache eviction");
        SE2N_HIP(hipFree(p->cache.back().dptr), "hipFree of an evicted propagator table");
        p->cache_bytes -= p->cache.back().bytes;
        p->cache.pop_back();
    }
    void* d = nullptr;
    hipError_t e = dev_malloc(&d, bytes);
    if (e != hipSuccess) return fail(SE2N_ENOMEM, "hipMalloc of %zu bytes for propagators: %s", bytes,
                                     hipGetErrorString(e));
    {
        ProfScope ps(p, "precompute", st);
        if (p->dt == SE2N_F32)
            e = launch_precompute<float>((float*)d, p->M, p->N, beta, T, n_steps, (int)scheme, st, p->keep_negligible);
        else
            e = launch_precompute<double>((double*)d, p->M, p->N, beta, T, n_steps, (int)scheme, st,
                                          p->keep_negligible);
    }
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(e, "propagator precompute launch");
    }
    p->cache.push_front(CacheEntry{key, d, bytes});
    p->cache_bytes += bytes;
    *out = d;
    return SE2N_OK;
}

// The cached propagator table for the given parameters, or NULL (no
// allocation, no launch).
const void* find_propagators(se2n_plan p, double T, double beta, int n_steps, se2n_scheme scheme) {
    CacheKey key{T, beta, scheme == SE2N_CN ? n_steps : 0, (int)scheme};
    std::lock_guard<std::mutex> lock(p->mu);
    for (auto it = p->cache.begin(); it != p->cache.end(); ++it) {
        if (it->key == key) {
            p->cache.splice(p->cache.begin(), p->cache, it);
            return p->cache.front().dptr;
        }
    }
    return nullptr;
}

// Estimated milliseconds of the two CN schedules on MI355X, from measured
// per-unit costs: the iterated kernel per mode and step, the FP64 propagator
// build per class (it grows with (N/2)^3 and with the binary powering's
// log2 n products).  Used only to choose a schedule for an uncached key.
// (FP32, 2048^2, N = 32: 6.66 ms for 400 iterated steps; the 400-step table
// takes 2.6 ms on the matrix cores (blocks of 9..16), 8.6 ms on the scalar
// path, whose cost grows with (N/2)^3.)
double est_iterated_ms(int M, int N, int n) {
    return 8.0e-9 * (double)(M / 2 + 1) * M * n * (N / 32.0);
}
double est_precompute_ms(int M, int N, int n) {
    const double h = N / 2.0;
    const double classes = (double)table_slots(M, N);  // one build per stored class
    const double products = (std::log2((double)n) + 3.0) / 11.6;
    if (h > 8 && h <= 16) return 1.0e-5 * classes * products;
    return 3.3e-5 * classes * (h * h * h / 4096.0) * products;
}

// Whether this CN diffusion runs the iterated schedule.  AUTO: a cached
// propagator table is always used; for an uncached key the iterated steps
// run while they are estimated cheaper than building the table, until the
// key has been asked for a second time (a table then pays for itself).
bool use_iterated(se2n_plan p, double T, double beta, int n_steps, se2n_scheme scheme) {
    if (scheme != SE2N_CN || (p->N & 1)) return false;  // the iterated kernel splits even N into p/q blocks
    if (p->schedule == SE2N_SCHEDULE_ITERATED) return true;
    if (p->schedule == SE2N_SCHEDULE_PROPAGATOR) return false;
    if (find_propagators(p, T, beta, n_steps, scheme)) return false;
    uint64_t tb, bb;
    std::memcpy(&tb, &T, sizeof tb);
    std::memcpy(&bb, &beta, sizeof bb);
    std::lock_guard<std::mutex> lock(p->mu);
    const int seen = p->misses[std::make_tuple(tb, bb, n_steps)]++;
    return seen == 0 && est_iterated_ms(p->M, p->N, n_steps) < est_precompute_ms(p->M, p->N, n_steps);
}

template <class R>
int spectral_middle_iter(se2n_plan p, C2<R>* spec, C2<R>* blk, double T, double beta, int n_steps, hipStream_t st) {
    const C2<R>* tw = (const C2<R>*)p->tw;
    const long ncols = (long)p->N * p->K();
    SE2N_TIMED(p, "col_fft_fwd", st, launch_col_fft<R>(false, spec, ncols, p->M, p->geom, p->planM, tw, st, nullptr),
               "forward column FFT");
    SE2N_TIMED(p, "solve_iter", st, launch_solve_iter<R>(spec, p->M, p->N, beta, T, n_steps, st),
               "iterated per-mode Crank-Nicolson");
    SE2N_TIMED(p, "col_fft_inv", st,
               launch_col_inv_paired<R>(spec, p->M, p->N, p->geom, p->planM, tw, st, nullptr, blk),
               "inverse column FFT");
    return SE2N_OK;
}

// Workspace: the half spectrum, the row-blocked copy the inverse column pass
// writes for the inverse row pass (blk_ok plans; left out of a workspace of
// workspace_unblocked() bytes), the max-combining buffer and the map.
template <class R>
struct Ws {
    C2<R>* spec;
    C2<R>* blk;  // null: the inverse passes work in place on spec
    typename Enc<R>::U* enc;
    uint8_t* rmap;
    const C2<R>* rows() const { return blk ? blk : spec; }  // what the inverse row pass reads
};

template <class R>
Ws<R> split_workspace(se2n_plan p, void* ws, bool use_blk = true) {
    char* b = (char*)ws;
    Ws<R> w;
    w.spec = (C2<R>*)b;
    const size_t bb = use_blk ? p->blk_bytes() : 0;
    w.blk = bb ? (C2<R>*)(b + p->spec_bytes()) : nullptr;
    w.enc = (typename Enc<R>::U*)(b + p->spec_bytes() + bb);
    w.rmap = (uint8_t*)(b + p->spec_bytes() + bb + p->enc_bytes());
    return w;
}

// Stencil radius for sigma (0: the FFT route) and a copy of its taps.  FP64
// plans always take the FFT route: the periodic kernels' aliasing floor
// (about exp(-pi^2 sigma^2 / 2)) keeps their tails above FP64 rounding.
int orient_radius(se2n_plan p, double sigma, OrientTaps* taps) {
    if (p->dt != SE2N_F32) return 0;
    std::lock_guard<std::mutex> lock(p->mu);
    if (!p->ot_valid || std::memcmp(&p->ot_sigma, &sigma, sizeof sigma) != 0) {
        p->ot_radius = orient_stencil_taps(p->M, sigma, &p->ot);
        p->ot_sigma = sigma;
        p->ot_valid = true;
    }
    if (taps) *taps = p->ot;
    return p->ot_radius;
}

template <class R>
int orient_impl(se2n_plan p, const R* f, const uint8_t* mask, double sigma, uint8_t* rmap, C2<R>* spec,
                hipStream_t st) {
    const C2<R>* tw = (const C2<R>*)p->tw;
    const int M = p->M;
    if constexpr (std::is_same<R, float>::value) {
        OrientTaps taps;
        const int rad = orient_radius(p, sigma, &taps);
        if (rad > 0) {
            SE2N_TIMED(p, "orient_stencil", st, launch_orient_stencil(f, mask, rmap, M, p->N, rad, taps, st),
                       "orientation stencil");
            return SE2N_OK;
        }
    }
    SE2N_TIMED(p, "orient_row_fwd", st,
               launch_row_fwd<R>(SRC_IMAGE, f, mask, nullptr, nullptr, spec, M, 1, p->geom, p->planH, tw, st),
               "orient row pass");
    SE2N_TIMED(p, "orient_col", st, launch_col_orient<R>(spec, M, p->geom, p->planM, tw, sigma, st),
               "orient column pass");
    SE2N_TIMED(p, "orient_row_inv", st,
               launch_row_inv<R>(DST_ORIENT, spec, nullptr, nullptr, rmap, M, 2, p->N, R(1), p->geom, 2,
                                 p->planH, tw, st),
               "orient inverse row pass");
    return SE2N_OK;
}

// spec holds the forward half spectrum of all slices; propagate it (in place,
// or into blk in the row-blocked layout when blk is set).
// The forward column pass does not store the modes of negligible classes;
// the solve writes their zeros unless the inverse column pass takes them as
// zero without reading them.  The inverse column pass runs on column pairs
// and leaves the pairing step of the real inverse row transform done (the
// row pass is then `paired`).
template <class R>
int spectral_middle(se2n_plan p, C2<R>* spec, C2<R>* blk, const void* P, hipStream_t st) {
    const C2<R>* tw = (const C2<R>*)p->tw;
    const long ncols = (long)p->N * p->K();
    const uint8_t* negf = table_flags(P, p->M, p->N, (int)sizeof(R));
    // the inverse column pass takes negligible modes as zero where it can do
    // so cheaply; the solve then does not store their zeros
    const bool masked = col_inv_masks<R>(p->M, p->geom);
    SE2N_TIMED(p, "col_fft_fwd", st, launch_col_fft<R>(false, spec, ncols, p->M, p->geom, p->planM, tw, st, negf),
               "forward column FFT");
    SE2N_TIMED(p, "solve", st, launch_solve<R>(spec, (const R*)P, p->M, p->N, st, !masked), "per-mode solve");
    SE2N_TIMED(p, "col_fft_inv", st,
               launch_col_inv_paired<R>(spec, p->M, p->N, p->geom, p->planM, tw, st, masked ? negf : nullptr, blk),
               "inverse column FFT");
    return SE2N_OK;
}

// spec: the paired spectrum, row-blocked if `blocked`.
template <class R>
int project_spec(se2n_plan p, const C2<R>* spec, bool blocked, typename Enc<R>::U* enc, se2n_proj mode, R* out,
                 hipStream_t st) {
    const C2<R>* tw = (const C2<R>*)p->tw;
    const int M = p->M, N = p->N;
    const long MM = (long)M * M;
    if (mode == SE2N_PROJ_MEAN) {
        SE2N_TIMED(p, "row_inv_mean", st,
                   launch_row_inv<R>(DST_SUM, spec, out, nullptr, nullptr, M, N, N, R(1) / (R)N, p->geom, N,
                                     p->planH, tw, st, true, blocked),
                   "inverse row pass (mean)");
        return SE2N_OK;
    }
    if (p->geom.inv_slices >= N) {
        SE2N_TIMED(p, "row_inv_max", st,
                   launch_row_inv<R>(DST_MAX, spec, out, nullptr, nullptr, M, N, N, R(1), p->geom, N, p->planH,
                                     tw, st, true, blocked),
                   "inverse row pass (max)");
        return SE2N_OK;
    }
    SE2N_TIMED(p, "fill_max", st, launch_fill_enc<R>(enc, MM, st), "clear max buffer");
    SE2N_TIMED(p, "row_inv_max", st,
               launch_row_inv<R>(DST_MAX, spec, nullptr, enc, nullptr, M, N, N, R(1), p->geom,
                                 p->geom.inv_slices, p->planH, tw, st, true, blocked),
               "inverse row pass (max)");
    SE2N_TIMED(p, "decode_max", st, launch_decode_enc<R>(enc, out, MM, st), "decode max buffer");
    return SE2N_OK;
}

template <class R>
int inpaint_impl(se2n_plan p, const R* f, const uint8_t* mask, double sigma, double T, double beta,
                 int n_steps, se2n_scheme scheme, se2n_proj mode, const uint8_t* rmap_in, uint8_t* rmap_out,
                 R* out, void* workspace, hipStream_t st, const void* P = nullptr, bool use_blk = true) {
    int rc = SE2N_OK;
    const bool iter = !P && use_iterated(p, T, beta, n_steps, scheme);
    if (!P && !iter) rc = get_propagators(p, T, beta, n_steps, scheme, st, &P);
    if (rc) return rc;
    p->last_schedule = iter ? SE2N_SCHEDULE_ITERATED : SE2N_SCHEDULE_PROPAGATOR;
    Ws<R> w = split_workspace<R>(p, workspace, use_blk);
    const uint8_t* rmap = rmap_in;
    if (!rmap_in) {
        uint8_t* dst = rmap_out ? rmap_out : w.rmap;
        rc = orient_impl<R>(p, f, mask, sigma, dst, w.spec, st);
        if (rc) return rc;
        rmap = dst;
    } else if (rmap_out && rmap_out != rmap_in) {
        SE2N_HIP(hipMemcpyAsync(rmap_out, rmap_in, (size_t)p->M * p->M, hipMemcpyDeviceToDevice, st),
                 "copy of rmap_in to rmap_out");
    }
    const C2<R>* tw = (const C2<R>*)p->tw;
    SE2N_TIMED(p, "lift_row_fwd", st,
               launch_row_fwd<R>(SRC_LIFT, f, mask, rmap, nullptr, w.spec, p->M, p->N, p->geom, p->planH, tw, st),
               "lift + row FFT");
    rc = iter ? spectral_middle_iter<R>(p, w.spec, w.blk, T, beta, n_steps, st)
              : spectral_middle<R>(p, w.spec, w.blk, P, st);
    if (rc) return rc;
    return project_spec<R>(p, w.rows(), w.blk != nullptr, w.enc, mode, out, st);
}

template <class R>
int diffuse_impl(se2n_plan p, R* psi, double T, double beta, int n_steps, se2n_scheme scheme, void* workspace,
                 hipStream_t st) {
    const void* P = nullptr;
    const bool iter = use_iterated(p, T, beta, n_steps, scheme);
    int rc = iter ? SE2N_OK : get_propagators(p, T, beta, n_steps, scheme, st, &P);
    if (rc) return rc;
    p->last_schedule = iter ? SE2N_SCHEDULE_ITERATED : SE2N_SCHEDULE_PROPAGATOR;
    Ws<R> w = split_workspace<R>(p, workspace);
    const C2<R>* tw = (const C2<R>*)p->tw;
    SE2N_TIMED(p, "row_fwd", st,
               launch_row_fwd<R>(SRC_VOLUME, nullptr, nullptr, nullptr, psi, w.spec, p->M, p->N, p->geom,
                                 p->planH, tw, st),
               "row FFT");
    rc = iter ? spectral_middle_iter<R>(p, w.spec, w.blk, T, beta, n_steps, st)
              : spectral_middle<R>(p, w.spec, w.blk, P, st);
    if (rc) return rc;
    SE2N_TIMED(p, "row_inv_volume", st,
               launch_row_inv<R>(DST_VOLUME, w.rows(), psi, nullptr, nullptr, p->M, p->N, p->N, R(1), p->geom,
                                 p->geom.inv_slices, p->planH, tw, st, true, w.blk != nullptr),
               "inverse row FFT");
    return SE2N_OK;
}

// Static / dynamic restoration (Sec. "Heuristic complements"): n intervals
// of tau = T/n, each integrated by the collapsed propagator of `substeps`
// Crank-Nicolson steps of tau/substeps (or e^{tau A}).  The state stays in
// the half spectrum; at mesh points t_1 .. t_{n-1} it is brought to a real
// volume, mixed on the good set (DR: after growing it), and transformed back.
template <class R>
int restore_impl(se2n_plan p, const R* f, const uint8_t* mask, double sigma, double T, double beta, int n_int,
                 int substeps, se2n_scheme scheme, double eps, bool dynamic, se2n_proj mode, const uint8_t* rmap_in,
                 uint8_t* rmap_out, int16_t* join_out, R* out, void* workspace, hipStream_t st) {
    const double tau = T / n_int;
    const void* P = nullptr;
    int rc = get_propagators(p, tau, beta, substeps, scheme, st, &P);
    if (rc) return rc;
    Ws<R> w = split_workspace<R>(p, workspace);
    char* b = (char*)workspace + p->workspace();
    R* vol = (R*)b;
    R* h = (R*)(b + p->vol_bytes());
    R* href = (R*)(b + p->vol_bytes() + p->enc_bytes());
    int16_t* join = (int16_t*)(b + p->vol_bytes() + 2 * p->enc_bytes());
    const uint8_t* rmap = rmap_in;
    if (!rmap_in) {
        uint8_t* dst = rmap_out ? rmap_out : w.rmap;
        rc = orient_impl<R>(p, f, mask, sigma, dst, w.spec, st);
        if (rc) return rc;
        rmap = dst;
    } else if (rmap_out && rmap_out != rmap_in) {
        SE2N_HIP(hipMemcpyAsync(rmap_out, rmap_in, (size_t)p->M * p->M, hipMemcpyDeviceToDevice, st),
                 "copy of rmap_in to rmap_out");
    }
    const C2<R>* tw = (const C2<R>*)p->tw;
    if (dynamic) SE2N_TIMED(p, "dr_init", st, launch_dr_init<R>(join, href, f, mask, p->M, st), "DR set-up");
    SE2N_TIMED(p, "lift_row_fwd", st,
               launch_row_fwd<R>(SRC_LIFT, f, mask, rmap, nullptr, w.spec, p->M, p->N, p->geom, p->planH, tw, st),
               "lift + row FFT");
    for (int i = 0; i < n_int; ++i) {
        if (i > 0) {
            SE2N_TIMED(p, "row_inv_volume", st,
                       launch_row_inv<R>(DST_VOLUME, w.rows(), vol, nullptr, nullptr, p->M, p->N, p->N, R(1), p->geom,
                                         p->geom.inv_slices, p->planH, tw, st, true, w.blk != nullptr),
                       "inverse row FFT");
            if (dynamic)
                SE2N_TIMED(p, "dr_step", st, launch_dr_step<R>(vol, h, join, href, eps, i, p->M, p->N, st),
                           "DR growth and mix");
            else
                SE2N_TIMED(p, "sr_mix", st, launch_sr_mix<R>(vol, f, mask, eps, p->M, p->N, st), "SR mix");
            SE2N_TIMED(p, "row_fwd", st,
                       launch_row_fwd<R>(SRC_VOLUME, nullptr, nullptr, nullptr, vol, w.spec, p->M, p->N, p->geom,
                                         p->planH, tw, st),
                       "row FFT");
        }
        rc = spectral_middle<R>(p, w.spec, w.blk, P, st);
        if (rc) return rc;
    }
    rc = project_spec<R>(p, w.rows(), w.blk != nullptr, w.enc, mode, out, st);
    if (rc) return rc;
    if (join_out) {
        if (dynamic)
            SE2N_HIP(hipMemcpyAsync(join_out, join, (size_t)p->M * p->M * sizeof(int16_t), hipMemcpyDeviceToDevice, st),
                     "copy of the join map");
        else
            SE2N_TIMED(p, "dr_init", st, launch_dr_init<R>(join_out, href, f, mask, p->M, st), "SR join map");
    }
    return SE2N_OK;
}

template <class R>
int make_twiddles(se2n_plan p) {
    const std::vector<C2<R>> h = quarter_twiddles<R>(p->M);
    const hipError_t e = dev_malloc(&p->tw, h.size() * sizeof(C2<R>));
    if (e != hipSuccess) {
        p->tw = nullptr;
        return fail(SE2N_ENOMEM, "hipMalloc of the twiddle table: %s", hipGetErrorString(e));
    }
    SE2N_HIP(hipMemcpy(p->tw, h.data(), h.size() * sizeof(C2<R>), hipMemcpyHostToDevice), "twiddle upload");
    return SE2N_OK;
}

// Workspace of se2n_inpaint_noalloc: a file-scope device array, so that the
// call needs no allocation.  Every GPU holds its own copy at its own address
// until the process ends; in host code `scratch` names only a host-side
// stand-in, so kernels receive the device address that hipGetSymbolAddress
// returned for the current device, never the array's name.
static __device__ __align__(256) unsigned char scratch[SE2N_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Look up the scratch array's address on `device` (which must be current).
// Called once per device at plan creation; later calls return the stored result.
void scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device] || g_scratch_err[device] != hipSuccess) return;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
        return;
    }
    g_scratch_ptr[device] = ptr;
}

}  // namespace

extern "C" {

int se2n_plan_create(se2n_plan* out, int M, int N, se2n_dtype dtype) {
    g_last_error.clear();
    if (!out) return fail(SE2N_EINVAL, "out is NULL");
    int twos = 0;
    if (M < 16 || M > 4096 || !is_2a3b(M, &twos, nullptr) || twos < 2)
        return fail(SE2N_EINVAL, "M must be 2^a 3^b with a >= 2 and 16 <= M <= 4096 (got %d)", M);
    if (N < 4 || N > 64) return fail(SE2N_EINVAL, "N must lie in [4, 64] (got %d)", N);
    if (dtype != SE2N_F32 && dtype != SE2N_F64) return fail(SE2N_EINVAL, "unknown dtype %d", (int)dtype);
    se2n_plan p = new (std::nothrow) se2n_plan_s;
    if (!p) return fail(SE2N_ENOMEM, "host allocation of the plan failed");
    p->M = M;
    p->N = N;
    p->dt = dtype;
    (void)hipGetDevice(&p->device);
    int num_cu = 0;
    if (hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || num_cu < 1)
        num_cu = 256;
    scratch_init(p->device);
    p->keep_negligible = std::getenv("SE2N_KEEP_NEGLIGIBLE") != nullptr;
    p->planH = make_fft_plan(M / 2, M);
    p->planM = make_fft_plan(M, M);
    int rc;
    if (dtype == SE2N_F32) {
        p->geom = make_geom<float>(M, N, num_cu);
        rc = check_geom<float>(p->geom, M);
        if (!rc) rc = make_twiddles<float>(p);
        // SE2N_NO_ROW_BLOCKS: the inverse passes stay in place (measurement)
        p->blk_ok = row_blocked<float>(M, p->geom) && std::getenv("SE2N_NO_ROW_BLOCKS") == nullptr;
    } else {
        p->geom = make_geom<double>(M, N, num_cu);
        rc = check_geom<double>(p->geom, M);
        if (!rc) rc = make_twiddles<double>(p);
    }
    if (rc) {
        if (p->tw) (void)hipFree(p->tw);
        delete p;
        return rc;
    }
    *out = p;
    return SE2N_OK;
}

int se2n_plan_info(se2n_plan p, int* M, int* N, se2n_dtype* dtype) {
    g_last_error.clear();
    const int rc = check_plan(p);
    if (rc) return rc;
    if (M) *M = p->M;
    if (N) *N = p->N;
    if (dtype) *dtype = p->dt;
    return SE2N_OK;
}

int se2n_plan_destroy(se2n_plan p) {
    g_last_error.clear();
    if (!p) return fail(SE2N_EINVAL, "plan is NULL");
    (void)hipDeviceSynchronize();
    for (auto& e : p->cache) (void)hipFree(e.dptr);
    for (auto& r : p->prof_pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : p->prof_pool) (void)hipEventDestroy(e);
    if (p->tw) (void)hipFree(p->tw);
    p->alive = false;
    delete p;
    return SE2N_OK;
}

size_t se2n_workspace_bytes(se2n_plan p) {
    if (!p || !p->alive) return 0;
    return p->workspace();
}

int se2n_precompute(se2n_plan p, double T, double beta, int n_steps, se2n_scheme scheme, void* stream) {
    g_last_error.clear();
    int rc = check_plan(p);
    if (rc) return rc;
    rc = check_diffusion_params(T, beta, n_steps, scheme);
    if (rc) return rc;
    const void* P = nullptr;
    return get_propagators(p, T, beta, n_steps, scheme, (hipStream_t)stream, &P);
}

int se2n_propagator_flags(se2n_plan p, double T, double beta, int n_steps, se2n_scheme scheme, void* stream,
                          uint8_t* flags, long capacity, int* Q) {
    g_last_error.clear();
    int rc = check_plan(p);
    if (rc) return rc;
    rc = check_diffusion_params(T, beta, n_steps, scheme);
    if (rc) return rc;
    if (!Q) return fail(SE2N_EINVAL, "null pointer argument");
    const int q = p->M / 4 + 1;
    *Q = q;
    if (!flags) return SE2N_OK;
    if (capacity < (long)q * q) return fail(SE2N_EINVAL, "capacity %ld < Q*Q = %ld", capacity, (long)q * q);
    const void* P = nullptr;
    hipStream_t st = (hipStream_t)stream;
    rc = get_propagators(p, T, beta, n_steps, scheme, st, &P);
    if (rc) return rc;
    const int rs = (int)p->real_size();
    const size_t FS = (size_t)flag_stride(p->M);
    const uint8_t* dflags = table_flags(P, p->M, p->N, rs);
    // the precompute ran on `st`; copy the padded rows synchronously, then unpad
    SE2N_HIP(hipStreamSynchronize(st), "hipStreamSynchronize before the flag copy");
    std::vector<uint8_t> rows((size_t)q * FS);
    SE2N_HIP(hipMemcpy(rows.data(), dflags, rows.size(), hipMemcpyDeviceToHost), "copy of the class flags");
    for (int lx = 0; lx < q; ++lx) std::memcpy(flags + (size_t)lx * q, rows.data() + (size_t)lx * FS, (size_t)q);
    return SE2N_OK;
}

int se2n_orient(se2n_plan p, const void* f, const uint8_t* mask, double sigma, uint8_t* rmap, void* workspace,
                void* stream) {
    g_last_error.clear();
    int rc = check_plan(p);
    if (rc) return rc;
    if (!f || !mask || !rmap || !workspace) return fail(SE2N_EINVAL, "null pointer argument");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(SE2N_EINVAL, "sigma must be > 0 (got %g)", sigma);
    hipStream_t st = (hipStream_t)stream;
    if (p->dt == SE2N_F32)
        return orient_impl<float>(p, (const float*)f, mask, sigma, rmap, split_workspace<float>(p, workspace).spec, st);
    return orient_impl<double>(p, (const double*)f, mask, sigma, rmap, split_workspace<double>(p, workspace).spec,
                               st);
}

int se2n_orient_method(se2n_plan p, double sigma, int* radius) {
    g_last_error.clear();
    int rc = check_plan(p);
    if (rc) return rc;
    if (!radius) return fail(SE2N_EINVAL, "null pointer argument");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(SE2N_EINVAL, "sigma must be > 0 (got %g)", sigma);
    *radius = orient_radius(p, sigma, nullptr);
    return SE2N_OK;
}

int se2n_orient_stencil_taps(int M, double sigma, float* g, float* d, int* radius) {
    g_last_error.clear();
    if (!g || !d || !radius) return fail(SE2N_EINVAL, "null pointer argument");
    if (M < 16 || M > 4096 || !is_2a3b(M, nullptr, nullptr) || M % 4 != 0)
        return fail(SE2N_EINVAL, "M must be 2^a 3^b with a >= 2 in [16, 4096] (got %d)", M);
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(SE2N_EINVAL, "sigma must be > 0 (got %g)", sigma);
    OrientTaps t;
    const int rad = orient_stencil_taps(M, sigma, &t);
    *radius = rad;
    if (rad == 0) return SE2N_OK;
    const int R = kOrientMaxRadius;
    for (int j = -R; j <= R; ++j) {
        const bool in = j >= -rad && j <= rad;
        g[j + R] = in ? t.g[j + rad] : 0.0f;
        d[j + R] = in ? t.d[j + rad] : 0.0f;
    }
    return SE2N_OK;
}

int se2n_lift(se2n_plan p, const void* f, const uint8_t* mask, const uint8_t* rmap, void* psi, void* stream) {
    g_last_error.clear();
    int rc = check_plan(p);
    if (rc) return rc;
    if (!f || !mask || !rmap || !psi) return fail(SE2N_EINVAL, "null pointer argument");
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps(p, "lift", st);
    hipError_t e = p->dt == SE2N_F32
                       ? launch_lift<float>((const float*)f, mask, rmap, (float*)psi, p->M, p->N, st)
                       : launch_lift<double>((const double*)f, mask, rmap, (double*)psi, p->M, p->N, st);
    if (e != hipSuccess) return hip_fail(e, "lift launch");
    return SE2N_OK;
}

int se2n_diffuse(se2n_plan p, void* psi, double T, double beta, int n_steps, se2n_scheme scheme, void* workspace,
                 void* stream) {
    g_last_error.clear();
    int rc = check_plan(p);
    if (rc) return rc;
    if (!psi || !workspace) return fail(SE2N_EINVAL, "null pointer argument");
    rc = check_diffusion_params(T, beta, n_steps, scheme);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (p->dt == SE2N_F32) return diffuse_impl<float>(p, (float*)psi, T, beta, n_steps, scheme, workspace, st);
    return diffuse_impl<double>(p, (double*)psi, T, beta, n_steps, scheme, workspace, st);
}

int se2n_project(se2n_plan p, const void* psi, se2n_proj mode, void* out, void* stream) {
    g_last_error.clear();
    int rc = check_plan(p);
    if (rc) return rc;
    if (!psi || !out) return fail(SE2N_EINVAL, "null pointer argument");
    if (mode != SE2N_PROJ_MAX && mode != SE2N_PROJ_MEAN) return fail(SE2N_EINVAL, "unknown projection %d", (int)mode);
    hipStream_t st = (hipStream_t)stream;
    const bool mean = mode == SE2N_PROJ_MEAN;
    ProfScope ps(p, "project", st);
    hipError_t e = p->dt == SE2N_F32 ? launch_project<float>((const float*)psi, (float*)out, p->M, p->N, mean, st)
                                     : launch_project<double>((const double*)psi, (double*)out, p->M, p->N, mean, st);
    if (e != hipSuccess) return hip_fail(e, "project launch");
    return SE2N_OK;
}

int se2n_inpaint(se2n_plan p, const void* f, const uint8_t* mask, double sigma, double T, double beta, int n_steps,
                 se2n_scheme scheme, se2n_proj mode, const uint8_t* rmap_in, uint8_t* rmap_out, void* out,
                 void* workspace, void* stream) {
    g_last_error.clear();
    int rc = check_plan(p);
    if (rc) return rc;
    if (!f || !mask || !out || !workspace) return fail(SE2N_EINVAL, "null pointer argument");
    if (!rmap_in && (!(sigma > 0.0) || !std::isfinite(sigma)))
        return fail(SE2N_EINVAL, "sigma must be > 0 (got %g)", sigma);
    if (mode != SE2N_PROJ_MAX && mode != SE2N_PROJ_MEAN) return fail(SE2N_EINVAL, "unknown projection %d", (int)mode);
    rc = check_diffusion_params(T, beta, n_steps, scheme);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (p->dt == SE2N_F32)
        return inpaint_impl<float>(p, (const float*)f, mask, sigma, T, beta, n_steps, scheme, mode, rmap_in,
                                   rmap_out, (float*)out, workspace, st);
    return inpaint_impl<double>(p, (const double*)f, mask, sigma, T, beta, n_steps, scheme, mode, rmap_in, rmap_out,
                                (double*)out, workspace, st);
}

int se2n_inpaint_noalloc(se2n_plan p, const void* f, const uint8_t* mask, double sigma, double T, double beta,
                         int n_steps, se2n_scheme scheme, se2n_proj mode, const uint8_t* rmap_in, uint8_t* rmap_out,
                         void* out, void* stream) {
    g_last_error.clear();
    int rc = check_plan(p);
    if (rc) return rc;
    if (!f || !mask || !out) return fail(SE2N_EINVAL, "null pointer argument");
    if (!rmap_in && (!(sigma > 0.0) || !std::isfinite(sigma)))
        return fail(SE2N_EINVAL, "sigma must be > 0 (got %g)", sigma);
    if (mode != SE2N_PROJ_MAX && mode != SE2N_PROJ_MEAN) return fail(SE2N_EINVAL, "unknown projection %d", (int)mode);
    rc = check_diffusion_params(T, beta, n_steps, scheme);
    if (rc) return rc;
    // the row-blocked copy of the spectrum is used when it fits as well
    const bool use_blk = p->workspace() <= (size_t)SE2N_NOALLOC_MAX_BYTES;
    if (p->workspace_unblocked() > (size_t)SE2N_NOALLOC_MAX_BYTES)
        return fail(SE2N_EINVAL, "M=%d, N=%d needs %zu bytes of workspace, above the %zu-byte static scratch", p->M,
                    p->N, p->workspace_unblocked(), (size_t)SE2N_NOALLOC_MAX_BYTES);
    int dev = -1;
    SE2N_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev != p->device) return fail(SE2N_ESTATE, "the plan belongs to device %d, device %d is current", p->device, dev);
    void* ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (dev < 0 || dev >= kMaxDevices) return fail(SE2N_EUNSUPPORTED, "device index %d out of range", dev);
        if (g_scratch_err[dev] != hipSuccess) return hip_fail(g_scratch_err[dev], "hipGetSymbolAddress(scratch)");
        ws = g_scratch_ptr[dev];
    }
    if (!ws) return fail(SE2N_ESTATE, "static scratch of device %d not set up", dev);
    const bool iter = scheme == SE2N_CN && p->schedule == SE2N_SCHEDULE_ITERATED;
    const void* P = iter ? nullptr : find_propagators(p, T, beta, n_steps, scheme);
    if (!P && !iter)
        return fail(SE2N_ESTATE, "propagators for T=%g, beta=%g, n_steps=%d, scheme=%d are not cached: call "
                    "se2n_precompute first (or set the iterated schedule)", T, beta, n_steps, (int)scheme);
    if (!rmap_in && p->dt == SE2N_F32) {
        std::lock_guard<std::mutex> lock(p->mu);
        if (!p->ot_valid || std::memcmp(&p->ot_sigma, &sigma, sizeof sigma) != 0)
            return fail(SE2N_ESTATE, "orientation taps for sigma=%g are not prepared: call se2n_orient_method first",
                        sigma);
    }
    hipStream_t st = (hipStream_t)stream;
    p->prof_hold = true;  // timing events would be created on demand
    if (p->dt == SE2N_F32)
        rc = inpaint_impl<float>(p, (const float*)f, mask, sigma, T, beta, n_steps, scheme, mode, rmap_in, rmap_out,
                                 (float*)out, ws, st, P, use_blk);
    else
        rc = inpaint_impl<double>(p, (const double*)f, mask, sigma, T, beta, n_steps, scheme, mode, rmap_in,
                                  rmap_out, (double*)out, ws, st, P, use_blk);
    p->prof_hold = false;
    return rc;
}

size_t se2n_restore_workspace_bytes(se2n_plan p) {
    if (!p || !p->alive) return 0;
    return p->restore_workspace();
}

int se2n_restore(se2n_plan p, const void* f, const uint8_t* mask, double sigma, double T, double beta,
                 int n_intervals, int substeps, se2n_scheme scheme, double eps, int dynamic, se2n_proj mode,
                 const uint8_t* rmap_in, uint8_t* rmap_out, int16_t* join_out, void* out, void* workspace,
                 void* stream) {
    g_last_error.clear();
    int rc = check_plan(p);
    if (rc) return rc;
    if (!f || !mask || !out || !workspace) return fail(SE2N_EINVAL, "null pointer argument");
    if (!rmap_in && (!(sigma > 0.0) || !std::isfinite(sigma)))
        return fail(SE2N_EINVAL, "sigma must be > 0 (got %g)", sigma);
    if (mode != SE2N_PROJ_MAX && mode != SE2N_PROJ_MEAN) return fail(SE2N_EINVAL, "unknown projection %d", (int)mode);
    if (n_intervals < 1 || n_intervals > 32767)
        return fail(SE2N_EINVAL, "n_intervals must lie in [1, 32767] (got %d)", n_intervals);
    if (substeps < 1) return fail(SE2N_EINVAL, "substeps must be >= 1 (got %d)", substeps);
    if (!(eps >= 0.0 && eps <= 1.0)) return fail(SE2N_EINVAL, "eps must lie in [0, 1] (got %g)", eps);
    if (dynamic != 0 && dynamic != 1) return fail(SE2N_EINVAL, "dynamic must be 0 or 1 (got %d)", dynamic);
    rc = check_diffusion_params(T, beta, substeps, scheme);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (p->dt == SE2N_F32)
        return restore_impl<float>(p, (const float*)f, mask, sigma, T, beta, n_intervals, substeps, scheme, eps,
                                   dynamic != 0, mode, rmap_in, rmap_out, join_out, (float*)out, workspace, st);
    return restore_impl<double>(p, (const double*)f, mask, sigma, T, beta, n_intervals, substeps, scheme, eps,
                                dynamic != 0, mode, rmap_in, rmap_out, join_out, (double*)out, workspace, st);
}

int se2n_set_schedule(se2n_plan p, se2n_schedule schedule) {
    g_last_error.clear();
    int rc = check_plan(p);
    if (rc) return rc;
    if (schedule != SE2N_SCHEDULE_AUTO && schedule != SE2N_SCHEDULE_PROPAGATOR && schedule != SE2N_SCHEDULE_ITERATED)
        return fail(SE2N_EINVAL, "unknown schedule %d", (int)schedule);
    if (schedule == SE2N_SCHEDULE_ITERATED && (p->N & 1))
        return fail(SE2N_EUNSUPPORTED, "the iterated schedule needs even N (got %d)", p->N);
    p->schedule = schedule;
    return SE2N_OK;
}

int se2n_last_schedule(se2n_plan p, se2n_schedule* schedule) {
    g_last_error.clear();
    int rc = check_plan(p);
    if (rc) return rc;
    if (!schedule) return fail(SE2N_EINVAL, "schedule is NULL");
    *schedule = p->last_schedule;
    return SE2N_OK;
}

int se2n_profile(se2n_plan p, int enable) {
    g_last_error.clear();
    int rc = check_plan(p);
    if (rc) return rc;
    for (auto& r : p->prof_pending) {
        SE2N_HIP(hipEventSynchronize(r.b), "hipEventSynchronize");
        p->prof_pool.push_back(r.a);
        p->prof_pool.push_back(r.b);
    }
    p->prof_pending.clear();
    p->prof_acc.clear();
    p->prof_on = enable != 0;
    return SE2N_OK;
}

int se2n_profile_stats(se2n_plan p, se2n_kernel_stat* out, int capacity, int* count) {
    g_last_error.clear();
    int rc = check_plan(p);
    if (rc) return rc;
    if (!count) return fail(SE2N_EINVAL, "count is NULL");
    for (auto& r : p->prof_pending) {
        SE2N_HIP(hipEventSynchronize(r.b), "hipEventSynchronize");
        float ms = 0.f;
        SE2N_HIP(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
        auto& acc = p->prof_acc[r.name];
        acc.first += 1;
        acc.second += ms;
        p->prof_pool.push_back(r.a);
        p->prof_pool.push_back(r.b);
    }
    p->prof_pending.clear();
    int i = 0;
    for (auto& kv : p->prof_acc) {
        if (out && i < capacity) {
            std::snprintf(out[i].name, sizeof out[i].name, "%s", kv.first.c_str());
            out[i].launches = kv.second.first;
            out[i].total_ms = kv.second.second;
        }
        ++i;
    }
    *count = i;
    return SE2N_OK;
}

int se2n_debug_fail_allocations(long after) {
    g_last_error.clear();
    if (after < -1) return fail(SE2N_EINVAL, "after must be >= -1 (got %ld)", after);
    g_alloc_budget.store(after);
    return SE2N_OK;
}

const char* se2n_last_error(void) { return g_last_error.c_str(); }

const char* se2n_version(void) { return "se2n 0.1 (gfx950)"; }

}  // extern "C"
