// Host runtime of batched inpainting: batch plans (propagator tables, tile
// lists, the captured graph), the schedule autotuner and its table, and the
// C ABI of the batched calls in include/se2n.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/se2n.h"
#include "se2n_batch.hpp"
#include "se2n_orient.hpp"
#include "se2n_host.hpp"
#include "se2n_internal.hpp"

using namespace se2n;

namespace {

constexpr int kMaxItems = 4096;
constexpr int kMaxPlansPerDevice = 4;
constexpr int kPixelsPerTile = 8192;  // clear / decode tiles

// The pointer-free description of an item: what a batch plan is built for.
struct Shape {
    int M, N, n, scheme, proj;
    double T, beta, sigma;
};

std::string signature_of(const std::vector<Shape>& sh) {
    std::string s;
    char b[160];
    for (const Shape& x : sh) {
        snprintf(b, sizeof b, "%d,%d,%d,%d,%d,%a,%a,%a;", x.M, x.N, x.scheme == SE2N_CN ? x.n : 0, x.scheme, x.proj,
                 x.T, x.beta, x.sigma);
        s += b;
    }
    return s;
}

uint64_t fnv1a(const std::string& s) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

std::string hex64(uint64_t h) {
    char b[20];
    snprintf(b, sizeof b, "%016llx", (unsigned long long)h);
    return b;
}

int check_items(const se2n_item* items, int count, bool need_pointers) {
    if (!items) return fail(SE2N_EINVAL, "items is NULL");
    if (count < 1 || count > kMaxItems) return fail(SE2N_EINVAL, "count must lie in [1, %d] (got %d)", kMaxItems, count);
    for (int i = 0; i < count; ++i) {
        const se2n_item& it = items[i];
        int twos = 0;
        if (it.M < 16 || it.M > kBatchMaxM || !is_2a3b(it.M, &twos, nullptr) || twos < 3)
            return fail(SE2N_EINVAL, "item %d: M must be 2^a 3^b with a >= 3 and 16 <= M <= %d (got %d)", i,
                        kBatchMaxM, it.M);
        if (it.N < 4 || it.N > 64 || it.N % 2)
            return fail(SE2N_EINVAL, "item %d: N must be even in [4, 64] (got %d)", i, it.N);
        if (it.scheme != SE2N_CN && it.scheme != SE2N_EXACT)
            return fail(SE2N_EINVAL, "item %d: unknown scheme %d", i, it.scheme);
        if (it.proj != SE2N_PROJ_MAX && it.proj != SE2N_PROJ_MEAN)
            return fail(SE2N_EINVAL, "item %d: unknown projection %d", i, it.proj);
        if (it.scheme == SE2N_CN && it.n_steps < 1)
            return fail(SE2N_EINVAL, "item %d: n_steps must be >= 1 (got %d)", i, it.n_steps);
        if (!(it.T >= 0.0) || !std::isfinite(it.T)) return fail(SE2N_EINVAL, "item %d: T must be finite, >= 0", i);
        if (!(it.beta >= 0.0) || !std::isfinite(it.beta))
            return fail(SE2N_EINVAL, "item %d: beta must be finite, >= 0", i);
        if (!(it.sigma > 0.0) || !std::isfinite(it.sigma))
            return fail(SE2N_EINVAL, "item %d: sigma must be finite, > 0", i);
        if (need_pointers && (!it.f || !it.mask || !it.out))
            return fail(SE2N_EINVAL, "item %d: f, mask and out must be non-NULL", i);
    }
    return SE2N_OK;
}

std::vector<Shape> shapes_of(const se2n_item* items, int count) {
    std::vector<Shape> v(count);
    for (int i = 0; i < count; ++i) {
        const se2n_item& it = items[i];
        v[i] = Shape{it.M, it.N, it.scheme == SE2N_CN ? it.n_steps : 0, it.scheme, it.proj, it.T, it.beta, it.sigma};
    }
    return v;
}

int check_tune(const se2n_tune& t) {
    if (t.wg_per_cu < 0 || t.wg_per_cu > 16) return fail(SE2N_EINVAL, "wg_per_cu must lie in [0, 16]");
    if (t.order != 0 && t.order != 1) return fail(SE2N_EINVAL, "order must be 0 or 1");
    if (t.row_groups < 1 || t.row_groups > 64) return fail(SE2N_EINVAL, "row_groups must lie in [1, 64]");
    return SE2N_OK;
}

const se2n_tune kDefaultTune = {2, 0, 1, 0};

// ---------------------------------------------------------------------------
// Workspace layout and tiles (host only)
// ---------------------------------------------------------------------------
struct Layout {
    std::vector<size_t> spec, blk, enc, rmap;  // blk: SIZE_MAX where the side has none
    size_t bytes = 0;
};

Layout layout_of(const std::vector<Shape>& sh) {
    Layout L;
    size_t off = 0;
    for (const Shape& x : sh) {
        const size_t M = (size_t)x.M, K = M / 2 + 1;
        const size_t vol = align256((size_t)x.N * K * M * sizeof(C2<float>));
        L.spec.push_back(off);
        off += vol;
        if (batch_blocked(x.M)) {
            L.blk.push_back(off);
            off += vol;
        } else {
            L.blk.push_back(SIZE_MAX);
        }
        L.enc.push_back(off);
        off += align256(M * M * sizeof(unsigned));
        L.rmap.push_back(off);
        off += align256(M * M);
    }
    L.bytes = off;
    return L;
}

// Slice groups of an item's lift and inverse row passes under `t`.
int groups_of(const Shape& x, const se2n_tune& t) {
    if (x.proj == SE2N_PROJ_MEAN) return 1;  // the mean is written directly
    const int g = std::min(t.row_groups, x.N);
    const int spg = (x.N + g - 1) / g;
    return (x.N + spg - 1) / spg;
}

struct Tile {
    int4 v;
    double cost;
};

double lg2(int n) { return std::log2((double)std::max(n, 2)); }

// Tiles of one pass (see se2n_batch_tiles) before ordering.
std::vector<Tile> raw_tiles(const std::vector<Shape>& sh, const se2n_tune& t, int pass) {
    std::vector<Tile> out;
    for (int i = 0; i < (int)sh.size(); ++i) {
        const Shape& x = sh[i];
        const int M = x.M, H = M / 2, K = H + 1, N = x.N;
        const GeomCore g = geom_core<float>(M);
        const int nrb = M / g.rows;
        switch (pass) {
            case 0:
            case 2: {
                if (orient_stencil_taps_cached(M, x.sigma, nullptr) > 0) break;
                const int ns = pass == 0 ? 1 : 2;
                for (int rb = 0; rb < nrb; ++rb)
                    out.push_back({make_int4(i, rb, 0, ns), (double)ns * g.rows * H * lg2(H)});
                break;
            }
            case 1:
                if (orient_stencil_taps_cached(M, x.sigma, nullptr) > 0) break;
                for (int c = 0; c < K; c += g.ocols)
                    out.push_back({make_int4(i, c, 0, 0), 3.0 * std::min(g.ocols, K - c) * M * lg2(M)});
                break;
            case 9: {
                const int rad = orient_stencil_taps_cached(M, x.sigma, nullptr);
                if (rad == 0) break;
                for (int tt = 0; tt < orient_tiles(M); ++tt)
                    out.push_back({make_int4(i, tt, rad, 0), (double)kOrientTX * kOrientTY * (2 * rad + 1)});
                break;
            }
            case 3:
            case 6: {
                const int grp = groups_of(x, t);
                const int spg = (N + grp - 1) / grp;
                for (int gi = 0; gi < grp; ++gi) {
                    const int sb = gi * spg, se = std::min(N, sb + spg);
                    for (int rb = 0; rb < nrb; ++rb)
                        out.push_back({make_int4(i, rb, sb, se), (double)(se - sb) * g.rows * H * lg2(H)});
                }
                break;
            }
            case 4: {
                const long ncols = (long)N * K;
                for (long c = 0; c < ncols; c += g.cols)
                    out.push_back({make_int4(i, (int)c, 0, 0), (double)std::min<long>(g.cols, ncols - c) * M * lg2(M)});
                break;
            }
            case 5: {
                const int Q = M / 4 + 1;
                const int cls = solve_classes(N, 4);  // classes per tile of the solve instance for N
                for (int lx = 0; lx < Q; ++lx)
                    for (int ly = 0; ly < Q; ly += cls)
                        out.push_back({make_int4(i, lx, ly, N), (double)std::min(cls, Q - ly) * 8.0 * N * N});
                break;
            }
            case 8: {
                // inverse column pass on column pairs (k, H-k), k = 0 .. H/2,
                // pcols/2 pairs per tile; the tile is the linear index
                // slice * tiles_per_slice + pair block
                const int P = g.pcols / 2;
                const int tps = (H / 2 + 1 + P - 1) / P;
                for (int tt = 0; tt < N * tps; ++tt) {
                    const int np = std::min(P, H / 2 + 1 - (tt % tps) * P);
                    out.push_back({make_int4(i, tt, 0, 0), (double)2 * np * M * lg2(M)});
                }
                break;
            }
            case 7:
                if (x.proj == SE2N_PROJ_MAX && groups_of(x, t) > 1) {
                    const int npx = M * M;
                    for (int p = 0; p < npx; p += kPixelsPerTile)
                        out.push_back({make_int4(i, p, std::min(kPixelsPerTile, npx - p), 0),
                                       (double)std::min(kPixelsPerTile, npx - p)});
                }
                break;
            default:
                break;
        }
    }
    return out;
}

std::vector<int4> ordered_tiles(const std::vector<Shape>& sh, const se2n_tune& t, int pass) {
    std::vector<Tile> raw = raw_tiles(sh, t, pass);
    if (t.order == 0)
        std::stable_sort(raw.begin(), raw.end(), [](const Tile& a, const Tile& b) { return a.cost > b.cost; });
    std::vector<int4> v(raw.size());
    for (size_t k = 0; k < raw.size(); ++k) v[k] = raw[k].v;
    return v;
}

// ---------------------------------------------------------------------------
// Tuning table
// ---------------------------------------------------------------------------
std::mutex g_mu;  // guards everything below
std::map<std::string, se2n_tune> g_tune_set;    // se2n_batch_set_tune
std::map<std::string, se2n_tune> g_tune_table;  // loaded or autotuned
bool g_env_table_read = false;

std::string arch_of(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

std::string tune_key(const std::string& arch, uint64_t sig) { return arch + "|" + hex64(sig); }

bool json_str(const std::string& line, const char* key, std::string& out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = line.find(k);
    if (p == std::string::npos) return false;
    p = line.find(':', p + k.size());
    if (p == std::string::npos) return false;
    p = line.find('"', p);
    if (p == std::string::npos) return false;
    const size_t q = line.find('"', p + 1);
    if (q == std::string::npos) return false;
    out = line.substr(p + 1, q - p - 1);
    return true;
}

bool json_num(const std::string& line, const char* key, double& out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = line.find(k);
    if (p == std::string::npos) return false;
    p = line.find(':', p + k.size());
    if (p == std::string::npos) return false;
    char* end = nullptr;
    out = std::strtod(line.c_str() + p + 1, &end);
    return end != line.c_str() + p + 1;
}

int load_table_locked(const char* path) {
    std::ifstream in(path);
    if (!in) return fail(SE2N_EHIP, "cannot read tuning table %s", path);
    std::string line;
    while (std::getline(in, line)) {
        std::string arch, sig;
        double w, o, g;
        if (!json_str(line, "arch", arch) || !json_str(line, "signature", sig) || !json_num(line, "wg_per_cu", w) ||
            !json_num(line, "order", o) || !json_num(line, "row_groups", g))
            continue;
        se2n_tune t{(int)w, (int)o, (int)g, 0};
        if (check_tune(t) != SE2N_OK) {
            clear_error();
            continue;
        }
        g_tune_table[arch + "|" + sig] = t;
    }
    return SE2N_OK;
}

void read_env_table_locked() {
    if (g_env_table_read) return;
    g_env_table_read = true;
    if (const char* p = std::getenv("SE2N_TUNE_TABLE")) {
        if (load_table_locked(p) != SE2N_OK) clear_error();  // a missing table is not an error
    }
}

se2n_tune lookup_tune_locked(const std::string& key) {
    read_env_table_locked();
    auto a = g_tune_set.find(key);
    if (a != g_tune_set.end()) return a->second;
    auto b = g_tune_table.find(key);
    if (b != g_tune_table.end()) return b->second;
    return kDefaultTune;
}

int write_table_entry(const char* path, const std::string& arch, uint64_t sig, int count, const se2n_tune& t,
                      double ms) {
    std::vector<std::string> keep;
    {
        std::ifstream in(path);
        std::string line;
        const std::string want = hex64(sig);
        while (in && std::getline(in, line)) {
            std::string a, s;
            if (json_str(line, "arch", a) && json_str(line, "signature", s) && a == arch && s == want) continue;
            if (!line.empty()) keep.push_back(line);
        }
    }
    char b[384];
    snprintf(b, sizeof b,
             "{\"arch\": \"%s\", \"signature\": \"%s\", \"items\": %d, \"wg_per_cu\": %d, \"order\": %d, "
             "\"row_groups\": %d, \"ms\": %.4f}",
             arch.c_str(), hex64(sig).c_str(), count, t.wg_per_cu, t.order, t.row_groups, ms);
    keep.push_back(b);
    std::ofstream out(path, std::ios::trunc);
    if (!out) return fail(SE2N_EHIP, "cannot write tuning table %s", path);
    for (const std::string& l : keep) out << l << "\n";
    return out.good() ? SE2N_OK : fail(SE2N_EHIP, "write to tuning table %s failed", path);
}

// ---------------------------------------------------------------------------
// Batch plans
// ---------------------------------------------------------------------------
struct TableKey {
    int M, N, n, scheme;
    double T, beta;
    bool operator<(const TableKey& o) const {
        return std::tie(M, N, n, scheme, T, beta) < std::tie(o.M, o.N, o.n, o.scheme, o.T, o.beta);
    }
};

struct Launch {
    int kind, N, cls;
    const char* name;
    int ntiles, grid;
    size_t lds;
    size_t tile_off;  // into the plan's tile buffer, in int4
    OrientTaps taps;  // BK_ORIENT_STENCIL only
};

const char* kind_name(int kind, int N) {
    static const char* solve_names[33] = {};
    static char buf[33][24];
    switch (kind) {
        case BK_ORIENT_ROW: return "b_orient_row_fwd";
        case BK_ORIENT_COL: return "b_orient_col";
        case BK_ORIENT_INV: return "b_orient_row_inv";
        case BK_LIFT_ROW: return "b_lift_row_fwd";
        case BK_COL_FWD: return "b_col_fft_fwd";
        case BK_COL_INV: return "b_col_fft_inv";
        case BK_FILL: return "b_fill_max";
        case BK_ROW_INV_MAX: return "b_row_inv_max";
        case BK_ROW_INV_MEAN: return "b_row_inv_mean";
        case BK_DECODE: return "b_decode_max";
        case BK_ORIENT_STENCIL: return "b_orient_stencil";
        case BK_SOLVE:
            if (N >= 4 && N <= 64 && N % 2 == 0) {
                const int k = N / 2;
                if (!solve_names[k]) {
                    snprintf(buf[k], sizeof buf[k], "b_solve_N%d", N);
                    solve_names[k] = buf[k];
                }
                return solve_names[k];
            }
            return "b_solve";
        default: return "b_unknown";
    }
}

struct BatchPlan {
    int device = 0;
    std::string sig;
    uint64_t hash = 0;
    std::vector<Shape> shapes;
    se2n_tune tune = kDefaultTune;
    Layout layout;
    int num_cu = 0;
    std::map<TableKey, void*> tables;
    std::map<int, void*> twiddles;
    std::vector<BItem> items;  // host copy (pointers as last uploaded)
    BItem* d_items = nullptr;
    bool uploaded = false;
    BItem* pinned[2] = {nullptr, nullptr};
    hipEvent_t pinned_ev[2] = {nullptr, nullptr};
    int ring = 0;
    std::vector<Launch> launches;
    int4* d_tiles = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    void drop_schedule() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d_tiles) (void)hipFree(d_tiles);
        exec = nullptr;
        graph = nullptr;
        d_tiles = nullptr;
        launches.clear();
    }
    ~BatchPlan() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        (void)hipDeviceSynchronize();
        drop_schedule();
        for (auto& kv : tables) (void)hipFree(kv.second);
        for (auto& kv : twiddles) (void)hipFree(kv.second);
        if (d_items) (void)hipFree(d_items);
        for (int k = 0; k < 2; ++k) {
            if (pinned[k]) (void)hipHostFree(pinned[k]);
            if (pinned_ev[k]) (void)hipEventDestroy(pinned_ev[k]);
        }
        if (cap) (void)hipStreamDestroy(cap);
        (void)hipSetDevice(cur);
    }
};

std::list<std::unique_ptr<BatchPlan>> g_plans;  // most recently used first

// Profiling of eager batched runs.
struct ProfRec {
    const char* name;
    hipEvent_t a, b;
};
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
std::map<std::string, std::pair<int, double>> g_prof_acc;

int build_schedule(BatchPlan& bp) {
    bp.drop_schedule();
    // tile lists per launch: pass x size class (x N for the solve, x projection for the inverse rows)
    struct Part {
        int kind, N, cls;
        std::vector<int4> tiles;
        OrientTaps taps;
    };
    std::vector<Part> parts;
    auto add_pass_fwd = [&](int kind, int pass) {
        std::vector<int4> all = ordered_tiles(bp.shapes, bp.tune, pass);
        if (kind == BK_ORIENT_STENCIL) {
            // one launch per (M, sigma), largest sides first
            std::vector<std::pair<int, double>> keys;
            for (const int4& t : all) {
                const std::pair<int, double> k(bp.shapes[t.x].M, bp.shapes[t.x].sigma);
                if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
            }
            std::stable_sort(keys.begin(), keys.end(),
                             [](const std::pair<int, double>& a, const std::pair<int, double>& b) {
                                 return a.first > b.first;
                             });
            for (const auto& k : keys) {
                Part p{kind, 0, 0, {}, {}};
                p.cls = orient_stencil_taps_cached(k.first, k.second, &p.taps);
                for (const int4& t : all)
                    if (bp.shapes[t.x].M == k.first && bp.shapes[t.x].sigma == k.second) p.tiles.push_back(t);
                parts.push_back(std::move(p));
            }
            return;
        }
        if (kind == BK_SOLVE) {
            std::vector<int> Ns;
            for (const int4& t : all)
                if (std::find(Ns.begin(), Ns.end(), t.w) == Ns.end()) Ns.push_back(t.w);
            std::sort(Ns.begin(), Ns.end());
            for (int N : Ns) {
                Part p{kind, N, 0, {}, {}};
                for (const int4& t : all)
                    if (t.w == N) p.tiles.push_back(t);
                parts.push_back(std::move(p));
            }
            return;
        }
        if (kind == BK_ORIENT_COL || kind == BK_FILL || kind == BK_DECODE) {
            if (!all.empty()) parts.push_back(Part{kind, 0, 0, std::move(all), {}});
            return;
        }
        for (int cls = kBatchClasses - 1; cls >= 0; --cls) {
            const int kinds[2] = {kind == BK_ROW_INV_MAX ? BK_ROW_INV_MAX : kind,
                                  kind == BK_ROW_INV_MAX ? BK_ROW_INV_MEAN : -1};
            for (int k : kinds) {
                if (k < 0) continue;
                Part p{k, 0, cls, {}, {}};
                for (const int4& t : all) {
                    const Shape& x = bp.shapes[t.x];
                    if (batch_class(x.M) != cls) continue;
                    if (k == BK_ROW_INV_MAX && x.proj != SE2N_PROJ_MAX) continue;
                    if (k == BK_ROW_INV_MEAN && x.proj != SE2N_PROJ_MEAN) continue;
                    p.tiles.push_back(t);
                }
                if (!p.tiles.empty()) parts.push_back(std::move(p));
            }
        }
    };
    // reverse: the pass's launches and tiles run in the opposite order, so
    // that it starts on the images the previous pass finished with (the
    // memory-side cache still holds their most recent lines)
    auto add_pass = [&](int kind, int pass, bool reverse = false) {
        const size_t first = parts.size();
        add_pass_fwd(kind, pass);
        if (reverse) {
            std::reverse(parts.begin() + first, parts.end());
            for (size_t k = first; k < parts.size(); ++k) std::reverse(parts[k].tiles.begin(), parts[k].tiles.end());
        }
    };
    add_pass(BK_ORIENT_STENCIL, 9);
    add_pass(BK_ORIENT_ROW, 0);
    add_pass(BK_ORIENT_COL, 1);
    add_pass(BK_ORIENT_INV, 2);
    add_pass(BK_LIFT_ROW, 3);
    add_pass(BK_COL_FWD, 4, true);
    add_pass(BK_SOLVE, 5);
    add_pass(BK_COL_INV, 8, true);
    add_pass(BK_FILL, 7);
    add_pass(BK_ROW_INV_MAX, 6);
    add_pass(BK_DECODE, 7);

    size_t total = 0;
    for (const Part& p : parts) total += p.tiles.size();
    std::vector<int4> flat;
    flat.reserve(total);
    for (const Part& p : parts) {
        Launch L{};
        L.kind = p.kind;
        L.N = p.N;
        L.cls = p.cls;
        L.name = kind_name(p.kind, p.N);
        L.ntiles = (int)p.tiles.size();
        L.tile_off = flat.size();
        L.taps = p.taps;
        // LDS: the largest need of the part's images
        size_t lds = 0;
        for (const int4& t : p.tiles) {
            const Shape& x = bp.shapes[t.x];
            const int M = x.M, H = M / 2;
            const GeomCore g = geom_core<float>(M);
            size_t need = 0;
            switch (p.kind) {
                case BK_ORIENT_INV:
                    need = (size_t)(tw_elems(M, true) + lds_padded_size(g.rows * (H + 2))) * sizeof(C2<float>);
                    break;
                case BK_ORIENT_ROW:
                case BK_LIFT_ROW:
                case BK_ROW_INV_MAX:
                case BK_ROW_INV_MEAN:
                    // two row buffers where the compiled stages run between them
                    need = batch_two_buf(M)
                               ? (size_t)(tw_elems(M, true) + 2 * row_buf_elems(M, g.rows)) * sizeof(C2<float>)
                               : (size_t)(tw_elems(M, true) + lds_padded_size(g.rows * (H + 2))) * sizeof(C2<float>);
                    break;
                case BK_COL_FWD:
                    need = (size_t)(tw_elems(M, false) + lds_padded_size(g.cols * M)) * sizeof(C2<float>);
                    break;
                case BK_COL_INV:
                    need = (size_t)(tw_elems(M, false) + lds_padded_size(g.pcols * M)) * sizeof(C2<float>);
                    break;
                case BK_ORIENT_COL:
                    need = (size_t)(tw_elems(M, false) + lds_padded_size(2 * g.ocols * M)) * sizeof(C2<float>);
                    break;
                case BK_SOLVE: {
                    need = (size_t)solve_lds_stride(x.N, 4) * solve_classes(x.N, 4) * sizeof(float);
                    break;
                }
                default:
                    break;
            }
            lds = std::max(lds, need);
        }
        if (lds > 160 * 1024) return fail(SE2N_EUNSUPPORTED, "batched pass %s needs %zu bytes of LDS", L.name, lds);
        L.lds = lds;
        int grid = L.ntiles;
        if (bp.tune.wg_per_cu > 0) {
            int occ = 0;
            SE2N_HIP(batch_occupancy(L.kind, L.N, L.cls, lds, &occ), "occupancy query of a batched kernel");
            if (occ < 1) return fail(SE2N_EUNSUPPORTED, "batched pass %s cannot be resident", L.name);
            grid = std::min(L.ntiles, std::min(bp.tune.wg_per_cu, occ) * bp.num_cu);
        }
        L.grid = std::max(grid, 1);
        bp.launches.push_back(L);
        flat.insert(flat.end(), p.tiles.begin(), p.tiles.end());
    }
    if (dev_malloc((void**)&bp.d_tiles, std::max<size_t>(flat.size(), 1) * sizeof(int4)) != hipSuccess) {
        bp.d_tiles = nullptr;
        return fail(SE2N_ENOMEM, "hipMalloc of the batch tiles failed");
    }
    SE2N_HIP(hipMemcpy(bp.d_tiles, flat.data(), flat.size() * sizeof(int4), hipMemcpyHostToDevice),
             "upload of batch tiles");

    // capture the launches into a graph (kernel nodes only)
    SE2N_HIP(hipStreamBeginCapture(bp.cap, hipStreamCaptureModeRelaxed), "begin graph capture");
    hipError_t le = hipSuccess;
    for (const Launch& L : bp.launches) {
        le = launch_batch(L.kind, L.N, L.cls, bp.d_items, bp.d_tiles + L.tile_off, L.ntiles, L.grid, L.lds, bp.cap,
                          &L.taps);
        if (le != hipSuccess) break;
    }
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(bp.cap, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le, "batched kernel launch during capture");
    }
    SE2N_HIP(ee, "end graph capture");
    bp.graph = g;
    SE2N_HIP(hipGraphInstantiate(&bp.exec, bp.graph, nullptr, nullptr, 0), "graph instantiate");
    return SE2N_OK;
}

int build_plan(BatchPlan& bp, const se2n_item* items, int count, hipStream_t st) {
    bp.shapes = shapes_of(items, count);
    bp.sig = signature_of(bp.shapes);
    bp.hash = fnv1a(bp.sig);
    SE2N_HIP(hipGetDevice(&bp.device), "hipGetDevice");
    SE2N_HIP(hipDeviceGetAttribute(&bp.num_cu, hipDeviceAttributeMultiprocessorCount, bp.device),
             "compute unit count");
    bp.tune = lookup_tune_locked(tune_key(arch_of(bp.device), bp.hash));
    bp.layout = layout_of(bp.shapes);
    SE2N_HIP(hipStreamCreateWithFlags(&bp.cap, hipStreamNonBlocking), "capture stream");
    for (int k = 0; k < 2; ++k) {
        if (pinned_malloc((void**)&bp.pinned[k], (size_t)count * sizeof(BItem)) != hipSuccess) {
            bp.pinned[k] = nullptr;
            return fail(SE2N_ENOMEM, "pinned allocation of the item staging failed");
        }
        SE2N_HIP(hipEventCreateWithFlags(&bp.pinned_ev[k], hipEventDisableTiming), "staging event");
    }
    if (dev_malloc((void**)&bp.d_items, (size_t)count * sizeof(BItem)) != hipSuccess) {
        bp.d_items = nullptr;
        return fail(SE2N_ENOMEM, "hipMalloc of the batch items failed");
    }

    bp.items.assign(count, BItem{});
    for (int i = 0; i < count; ++i) {
        const Shape& x = bp.shapes[i];
        const int M = x.M;
        // twiddles, one table per side
        if (!bp.twiddles.count(M)) {
            const std::vector<C2<float>> h = quarter_twiddles<float>(M);
            void* d = nullptr;
            if (dev_malloc(&d, h.size() * sizeof(C2<float>)) != hipSuccess)
                return fail(SE2N_ENOMEM, "hipMalloc of a twiddle table failed");
            bp.twiddles[M] = d;
            SE2N_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(C2<float>), hipMemcpyHostToDevice), "twiddle upload");
        }
        // propagators, one table per distinct parameter set (computed on the caller's stream)
        const TableKey tk{M, x.N, x.n, x.scheme, x.T, x.beta};
        if (!bp.tables.count(tk)) {
            void* d = nullptr;
            const hipError_t e = dev_malloc(&d, table_bytes(M, x.N, 4));  // class-major propagators + class flags
            if (e != hipSuccess) return fail(SE2N_ENOMEM, "hipMalloc of a propagator table: %s", hipGetErrorString(e));
            bp.tables[tk] = d;
            SE2N_HIP(launch_precompute<float>((float*)d, M, x.N, x.beta, x.T, x.n, x.scheme, st),
                     "propagator precompute launch");
        }
        const GeomCore g = geom_core<float>(M);
        BItem& b = bp.items[i];
        b.P = (const float*)bp.tables[tk];
        b.tw = (const C2<float>*)bp.twiddles[M];
        b.M = M;
        b.N = x.N;
        b.K = M / 2 + 1;
        b.rows = g.rows;
        b.cols = g.cols;
        b.ocols = g.ocols;
        b.pcols = g.pcols;
        b.proj = x.proj;
        b.groups = groups_of(x, bp.tune);
        b.Q = M / 4 + 1;
        b.FS = flag_stride(M);
        {
            const int side = kBatchSides[batch_class(M)];  // compiled side of the item's column kernels (0: generic)
            b.imask = side != 0 && col_skip_shape(side, geom_core<float>(side).pcol_threads) ? 1 : 0;
        }
        b.ocoef = (float)(-2.0 * 9.869604401089358619 * x.sigma * x.sigma / ((double)M * M));
        b.oscale = (float)(std::sqrt((double)M) / ((double)M * M));
        b.planH = make_fft_plan(M / 2, M);
        b.planM = make_fft_plan(M, M);
        // the invariants the batched bodies rely on (512 threads, 8 elements each)
        const int H = M / 2;
        if (g.rows * H > 8 * kBatchThreads || g.cols * M > 8 * kBatchThreads ||
            2 * g.ocols * M > 8 * kBatchThreads || g.pcols * M > 8 * kBatchThreads ||
            kBatchThreads % g.rows != 0 || g.tw_full != 1)
            return fail(SE2N_EUNSUPPORTED, "item %d: no batched geometry for M=%d", i, M);
    }
    return build_schedule(bp);
}

// Refresh the device item table if the caller's buffers differ from the last upload.
int upload_items(BatchPlan& bp, const se2n_item* items, void* ws, hipStream_t st) {
    bool changed = !bp.uploaded;
    char* base = (char*)ws;
    for (size_t i = 0; i < bp.items.size(); ++i) {
        BItem& b = bp.items[i];
        const se2n_item& it = items[i];
        BItem n = b;
        n.f = it.f;
        n.mask = it.mask;
        n.out = it.out;
        n.rmap = it.rmap_out ? it.rmap_out : (uint8_t*)(base + bp.layout.rmap[i]);
        n.spec = (C2<float>*)(base + bp.layout.spec[i]);
        n.blk = bp.layout.blk[i] == SIZE_MAX ? nullptr : (C2<float>*)(base + bp.layout.blk[i]);
        n.enc = (unsigned*)(base + bp.layout.enc[i]);
        n.groups = groups_of(bp.shapes[i], bp.tune);
        if (std::memcmp(&n, &b, sizeof(BItem)) != 0) {
            b = n;
            changed = true;
        }
    }
    if (!changed) return SE2N_OK;
    const int k = bp.ring;
    bp.ring ^= 1;
    // the staging buffer is reused only after its previous copy has run
    SE2N_HIP(hipEventSynchronize(bp.pinned_ev[k]), "wait for item staging");
    std::memcpy(bp.pinned[k], bp.items.data(), bp.items.size() * sizeof(BItem));
    SE2N_HIP(hipMemcpyAsync(bp.d_items, bp.pinned[k], bp.items.size() * sizeof(BItem), hipMemcpyHostToDevice, st),
             "item table upload");
    SE2N_HIP(hipEventRecord(bp.pinned_ev[k], st), "staging event record");
    bp.uploaded = true;
    return SE2N_OK;
}

hipEvent_t new_event() {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int run_plan(BatchPlan& bp, const se2n_item* items, void* ws, hipStream_t st) {
    int rc = upload_items(bp, items, ws, st);
    if (rc) return rc;
    if (!g_prof_on) {
        SE2N_HIP(hipGraphLaunch(bp.exec, st), "batch graph launch");
        return SE2N_OK;
    }
    for (const Launch& L : bp.launches) {
        hipEvent_t a = new_event(), b = new_event();
        if (a) (void)hipEventRecord(a, st);
        const hipError_t e =
            launch_batch(L.kind, L.N, L.cls, bp.d_items, bp.d_tiles + L.tile_off, L.ntiles, L.grid, L.lds, st,
                         &L.taps);
        if (b) (void)hipEventRecord(b, st);
        if (a && b) g_prof_pending.push_back({L.name, a, b});
        if (e != hipSuccess) return hip_fail(e, "batched kernel launch");
    }
    return SE2N_OK;
}

// Find or build the plan for these items on the current device (g_mu held).
int get_plan(const se2n_item* items, int count, hipStream_t st, BatchPlan** out) {
    int dev = 0;
    SE2N_HIP(hipGetDevice(&dev), "hipGetDevice");
    const std::string sig = signature_of(shapes_of(items, count));
    for (auto it = g_plans.begin(); it != g_plans.end(); ++it) {
        if ((*it)->device == dev && (*it)->sig == sig) {
            g_plans.splice(g_plans.begin(), g_plans, it);
            *out = g_plans.front().get();
            return SE2N_OK;
        }
    }
    std::unique_ptr<BatchPlan> bp(new (std::nothrow) BatchPlan);
    if (!bp) return fail(SE2N_ENOMEM, "host allocation of a batch plan failed");
    const int rc = build_plan(*bp, items, count, st);
    if (rc) return rc;  // bp's destructor frees what was allocated
    // keep at most kMaxPlansPerDevice plans per device
    int n_dev = 0;
    for (auto it = g_plans.begin(); it != g_plans.end();) {
        if ((*it)->device == dev && ++n_dev >= kMaxPlansPerDevice) it = g_plans.erase(it);
        else ++it;
    }
    g_plans.push_front(std::move(bp));
    *out = g_plans.front().get();
    return SE2N_OK;
}

void drop_plan_locked(int dev, const std::string& sig) {
    for (auto it = g_plans.begin(); it != g_plans.end(); ++it) {
        if ((*it)->device == dev && (*it)->sig == sig) {
            g_plans.erase(it);
            return;
        }
    }
}

}  // namespace

extern "C" {

size_t se2n_batch_workspace_bytes(const se2n_item* items, int count) {
    clear_error();
    if (check_items(items, count, false)) return 0;
    return layout_of(shapes_of(items, count)).bytes;
}

int se2n_inpaint_batched(const se2n_item* items, int count, void* workspace, void* stream) {
    clear_error();
    int rc = check_items(items, count, true);
    if (rc) return rc;
    if (!workspace) return fail(SE2N_EINVAL, "workspace is NULL");
    std::lock_guard<std::mutex> lock(g_mu);
    BatchPlan* bp = nullptr;
    rc = get_plan(items, count, (hipStream_t)stream, &bp);
    if (rc) return rc;
    return run_plan(*bp, items, workspace, (hipStream_t)stream);
}

int se2n_batch_autotune(const se2n_item* items, int count, void* workspace, void* stream, int reps,
                        const char* table_path, se2n_tune* best, double* best_ms) {
    clear_error();
    int rc = check_items(items, count, true);
    if (rc) return rc;
    if (!workspace) return fail(SE2N_EINVAL, "workspace is NULL");
    if (reps < 1) return fail(SE2N_EINVAL, "reps must be >= 1 (got %d)", reps);
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(g_mu);
    BatchPlan* bp = nullptr;
    rc = get_plan(items, count, st, &bp);
    if (rc) return rc;
    const bool prof = g_prof_on;
    g_prof_on = false;  // time graph launches
    hipEvent_t e0 = new_event(), e1 = new_event();
    if (!e0 || !e1) {
        g_prof_on = prof;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return fail(SE2N_EHIP, "event creation for the autotuner failed");
    }
    se2n_tune win = bp->tune;
    double win_ms = 1e300;
    const int wgs[4] = {0, 1, 2, 4};
    const int groups[3] = {1, 2, 4};
    for (int w : wgs) {
        for (int o = 0; o < 2 && rc == SE2N_OK; ++o) {
            for (int g : groups) {
                se2n_tune t{w, o, g, 0};
                rc = hipStreamSynchronize(st) == hipSuccess ? SE2N_OK : fail(SE2N_EHIP, "stream synchronise");
                if (rc) break;
                bp->tune = t;
                rc = build_schedule(*bp);
                if (!rc) rc = run_plan(*bp, items, workspace, st);  // warm-up (and item upload)
                if (rc) break;
                (void)hipEventRecord(e0, st);
                for (int r = 0; r < reps && !rc; ++r) rc = run_plan(*bp, items, workspace, st);
                (void)hipEventRecord(e1, st);
                if (rc) break;
                if (hipEventSynchronize(e1) != hipSuccess) {
                    rc = fail(SE2N_EHIP, "autotune timing");
                    break;
                }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                const double per = ms / reps;
                if (per < win_ms) {
                    win_ms = per;
                    win = t;
                }
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g_prof_on = prof;
    if (rc) return rc;
    SE2N_HIP(hipStreamSynchronize(st), "stream synchronise");
    bp->tune = win;
    rc = build_schedule(*bp);
    if (rc) return rc;
    const std::string arch = arch_of(bp->device);
    g_tune_table[tune_key(arch, bp->hash)] = win;
    if (table_path) {
        rc = write_table_entry(table_path, arch, bp->hash, count, win, win_ms);
        if (rc) return rc;
    }
    if (best) *best = win;
    if (best_ms) *best_ms = win_ms;
    return SE2N_OK;
}

int se2n_batch_load_tune_table(const char* path) {
    clear_error();
    if (!path) return fail(SE2N_EINVAL, "path is NULL");
    std::lock_guard<std::mutex> lock(g_mu);
    return load_table_locked(path);
}

int se2n_batch_set_tune(const se2n_item* items, int count, const se2n_tune* tune) {
    clear_error();
    int rc = check_items(items, count, false);
    if (rc) return rc;
    if (!tune) return fail(SE2N_EINVAL, "tune is NULL");
    rc = check_tune(*tune);
    if (rc) return rc;
    int dev = 0;
    SE2N_HIP(hipGetDevice(&dev), "hipGetDevice");
    const std::vector<Shape> sh = shapes_of(items, count);
    const std::string sig = signature_of(sh);
    std::lock_guard<std::mutex> lock(g_mu);
    g_tune_set[tune_key(arch_of(dev), fnv1a(sig))] = *tune;
    drop_plan_locked(dev, sig);
    return SE2N_OK;
}

int se2n_batch_get_tune(const se2n_item* items, int count, se2n_tune* out) {
    clear_error();
    int rc = check_items(items, count, false);
    if (rc) return rc;
    if (!out) return fail(SE2N_EINVAL, "out is NULL");
    int dev = 0;
    SE2N_HIP(hipGetDevice(&dev), "hipGetDevice");
    const std::string sig = signature_of(shapes_of(items, count));
    std::lock_guard<std::mutex> lock(g_mu);
    for (const auto& p : g_plans) {
        if (p->device == dev && p->sig == sig) {
            *out = p->tune;
            return SE2N_OK;
        }
    }
    *out = lookup_tune_locked(tune_key(arch_of(dev), fnv1a(sig)));
    return SE2N_OK;
}

int se2n_batch_tiles(const se2n_item* items, int count, const se2n_tune* tune, int pass, int* tiles, int capacity,
                     int* ntiles) {
    clear_error();
    int rc = check_items(items, count, false);
    if (rc) return rc;
    if (!ntiles) return fail(SE2N_EINVAL, "ntiles is NULL");
    if (pass < 0 || pass > 9) return fail(SE2N_EINVAL, "pass must lie in [0, 9] (got %d)", pass);
    if (tiles && capacity < 0) return fail(SE2N_EINVAL, "capacity must be >= 0");
    se2n_tune t = kDefaultTune;
    if (tune) {
        rc = check_tune(*tune);
        if (rc) return rc;
        t = *tune;
    }
    const std::vector<int4> v = ordered_tiles(shapes_of(items, count), t, pass);
    *ntiles = (int)v.size();
    if (tiles) {
        const int n = std::min(capacity, (int)v.size());
        for (int k = 0; k < n; ++k) {
            tiles[4 * k + 0] = v[k].x;
            tiles[4 * k + 1] = v[k].y;
            tiles[4 * k + 2] = v[k].z;
            tiles[4 * k + 3] = v[k].w;
        }
    }
    return SE2N_OK;
}

int se2n_batch_profile(int enable) {
    clear_error();
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto& r : g_prof_pending) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
    g_prof_acc.clear();
    g_prof_on = enable != 0;
    return SE2N_OK;
}

int se2n_batch_profile_stats(se2n_kernel_stat* out, int capacity, int* count) {
    clear_error();
    if (!count) return fail(SE2N_EINVAL, "count is NULL");
    if (out && capacity < 0) return fail(SE2N_EINVAL, "capacity must be >= 0");
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto& r : g_prof_pending) {
        SE2N_HIP(hipEventSynchronize(r.b), "wait for timing events");
        float ms = 0.f;
        SE2N_HIP(hipEventElapsedTime(&ms, r.a, r.b), "event elapsed time");
        auto& acc = g_prof_acc[r.name];
        acc.first += 1;
        acc.second += ms;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
    *count = (int)g_prof_acc.size();
    if (out) {
        int k = 0;
        for (const auto& kv : g_prof_acc) {
            if (k >= capacity) break;
            std::memset(&out[k], 0, sizeof out[k]);
            snprintf(out[k].name, sizeof out[k].name, "%s", kv.first.c_str());
            out[k].launches = kv.second.first;
            out[k].total_ms = kv.second.second;
            ++k;
        }
    }
    return SE2N_OK;
}

int se2n_batch_clear(void) {
    clear_error();
    std::lock_guard<std::mutex> lock(g_mu);
    g_plans.clear();
    return SE2N_OK;
}

}  // extern "C"
