// Host side of libgc.so: graph handles, CSR validation, workspace layout and
// the Greedy++ driver (Section 4 of Bergamini, Gonser, Meyerhenke).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "gc.h"
#include "gc_kernels.h"
#include "gc_mlp.h"
#include "gc_bits.h"
#include "gc_internal.h"
#include "gc_weighted.h"

using namespace gck;

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_OK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(GC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
    } while (0)

extern "C" const char *gc_strerror(int code) {
    switch (code) {
    case GC_OK: return "ok";
    case GC_EINVAL: return "invalid argument";
    case GC_ENOTSYM: return "adjacency is not symmetric";
    case GC_EDISCONNECTED: return "graph is not connected";
    case GC_ERANGE: return "distance exceeds the distance width";
    case GC_EWORKSPACE: return "workspace missing or too small";
    case GC_ENOMEM: return "host allocation failed";
    case GC_EDEVICE: return "HIP runtime error";
    default: return "unknown error";
    }
}

extern "C" const char *gc_last_error(void) { return g_last_error.c_str(); }

// Optional HIP-event timing of the gain kernels (gc_timing_enable).
static thread_local bool g_timing = false;
static thread_local float g_timing_ms = -1.f;
static thread_local hipEvent_t g_ev0 = nullptr, g_ev1 = nullptr;

extern "C" int gc_timing_enable(int on) {
    g_timing = on != 0;
    if (g_timing && !g_ev0) {
        if (hipEventCreate(&g_ev0) != hipSuccess || hipEventCreate(&g_ev1) != hipSuccess) {
            g_timing = false;
            g_last_error = "hipEventCreate failed";
            return GC_EDEVICE;
        }
    }
    g_timing_ms = -1.f;
    return GC_OK;
}

extern "C" double gc_timing_last_ms(void) { return (double)g_timing_ms; }

static double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------- graph

struct gc_graph {
    int32_t n;
    int64_t nnz;
    const int32_t *d_rp;
    const int32_t *d_ci;
    std::vector<int32_t> h_rp;  // host copy of row_ptr (degrees, orders)
    std::vector<int32_t> by_degree;  // nodes by decreasing degree, ties ascending id
    // source order of the closeness search and of the first gain round: balls
    // of 64 nearby nodes (GC_BALLS=0: the degree order and ascending ids)
    std::vector<int32_t> by_ball;
    std::vector<int32_t> ball_rank;  // position of every node in by_ball
    // the row split's chunks of the rows of more than kSplitLongRow entries:
    // pairs {row, index of the row's first pair}, one per kSplitChunk entries
    std::vector<int32_t> split_chunks;
    int32_t max_deg;
    int32_t num_cu;
    // tuning read once at load time so the workspace layout never changes
    int64_t vis_budget;     // GC_VIS_BUDGET_MB (bytes)
    int64_t log_entries;    // GC_LOG_ENTRIES
    int64_t touch_entries;  // GC_TOUCH_ENTRIES (0: n per batch, at most 64M)
    int32_t level_wgs_per_cu;  // GC_LEVEL_WGS (workgroups per CU of a level kernel)
    int32_t unroll;         // GC_UNROLL (4 or 8)
    int32_t min_edges;      // GC_MIN_EDGES (adjacency entries per workgroup)
    // the same two for gain launches of at most 1024 sources (later rounds)
    // and the d(S,.) updates:
    // GC_UNROLL_SMALL, GC_MIN_EDGES_SMALL
    int32_t unroll_small;
    int32_t min_edges_small;
    int32_t learned_pool_pct;  // GC_LEARNED_POOL_PCT: the learned order ranks the
                               // largest bounds, this many percent of a block (110..1600)
    bool balls;                // GC_BALLS (default on)
    bool directed;             // GC_DIRECTED: rows are out-neighbour lists
    // weighted graphs (gc_load_csr_weighted): the caller's uint8 lengths, the
    // largest one, the bucket widths of the gain and closeness searches
    // (GC_WDELTA, GC_WDELTA_CLOSE) and the number of search slots (GC_WSLOTS)
    // watchdogs (GC_LEVEL_CAP, GC_ROUND_CAP; 0 = none): a BFS that needs more
    // levels, or a weighted search more near-list rounds, fails the call
    // with GC_EDEVICE instead of running on
    int32_t level_cap = 0;
    uint32_t wround_cap = 0;
    bool weighted = false;
    const uint8_t *d_w = nullptr;
    int32_t wmax = 0;
    int32_t wdelta_gain = 0;
    int32_t wdelta_close = 0;
    int32_t wslots = 0;
    int32_t wclose_threads = 1024; // GC_WCLOSE_THREADS: workgroup of a closeness search (256 or 1024)
    int32_t wclose_slots = 256;    // GC_WCLOSE_SLOTS: closeness searches in flight (<= wslots)
    bool wdelta_close_env = false; // GC_WDELTA_CLOSE given (else from the first search's mean distance)
    const std::vector<int32_t> &search_order() const { return balls ? by_ball : by_degree; }
};

extern "C" int32_t gc_graph_n(const gc_graph *g) { return g ? g->n : -1; }
extern "C" int64_t gc_graph_nnz(const gc_graph *g) { return g ? g->nnz : -1; }

// weighted graphs: every distance, at most 255 (n - 1), fits int32
constexpr int32_t kWeightedMaxN = 1 << 23;

// the level watchdog: GC_EDEVICE once a BFS has reached `levels` levels
// beyond the cap (the call's device state is then undefined)
static int level_cap_check(const gc_graph *g, int64_t levels) {
    if (g->level_cap > 0 && levels > g->level_cap)
        return fail(GC_EDEVICE, "a BFS passed the level cap (GC_LEVEL_CAP = %d)", g->level_cap);
    return GC_OK;
}

// GC_EINVAL for a weighted graph in a call that only the unweighted engine has
static int unweighted_only(const gc_graph *g, const char *what) {
    return g && g->weighted ? fail(GC_EINVAL, "%s: unweighted graphs only", what) : GC_OK;
}

static int hw_threads() {
    unsigned t = std::thread::hardware_concurrency();
    if (t == 0) t = 1;
    if (t > 16) t = 16;
    return (int)t;
}

template <typename F>
static void parallel_for(int64_t n, F f) {
    const int nt = (int)std::min<int64_t>(hw_threads(), std::max<int64_t>(1, n / 65536));
    if (nt <= 1) {
        f(0, n);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) {
        int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
        th.emplace_back([=] { f(lo, hi); });
    }
    for (auto &x : th) x.join();
}

// CSR contract of the method's input (Section 2: connected, undirected,
// unweighted): ranges, sorted rows, no self-loops or duplicates, symmetry,
// one component.
static int validate_csr(int32_t n, int64_t nnz, const std::vector<int32_t> &rp,
                        const std::vector<int32_t> &ci, bool directed) {
    std::atomic<int> bad{GC_OK};
    std::atomic<int64_t> where{-1};
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t u = lo; u < hi && bad.load(std::memory_order_relaxed) == GC_OK; ++u) {
            for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
                const int32_t v = ci[e];
                if (v < 0 || v >= n || v == u || (e > rp[u] && ci[e - 1] >= v)) {
                    bad = GC_EINVAL;
                    where = u;
                    break;
                }
                if (!directed && !std::binary_search(ci.begin() + rp[v], ci.begin() + rp[v + 1], (int32_t)u)) {
                    int exp = GC_OK;
                    bad.compare_exchange_strong(exp, GC_ENOTSYM);
                    where = u;
                    break;
                }
            }
        }
    });
    if (bad != GC_OK) {
        if (bad == GC_ENOTSYM)
            return fail(GC_ENOTSYM, "row %lld has an edge without its reverse", (long long)where.load());
        return fail(GC_EINVAL, "row %lld: id out of range, self-loop, unsorted or duplicate entry",
                    (long long)where.load());
    }
    std::vector<uint8_t> seen((size_t)n, 0);
    std::vector<int32_t> q((size_t)n);
    int64_t h = 0, t = 0;
    q[t++] = 0;
    seen[0] = 1;
    while (h < t) {
        int32_t x = q[h++];
        for (int32_t e = rp[x]; e < rp[x + 1]; ++e)
            if (!seen[ci[e]]) {
                seen[ci[e]] = 1;
                q[t++] = ci[e];
            }
    }
    if (t != n) return fail(GC_EDISCONNECTED, "graph has %lld of %d nodes in the component of node 0",
                            (long long)t, n);
    if (directed) {
        // strongly connected: node 0 is also reached along the reversed arcs
        std::vector<int32_t> trp((size_t)n + 1, 0), tci((size_t)nnz);
        for (int64_t e = 0; e < nnz; ++e) trp[(size_t)ci[e] + 1]++;
        for (int32_t v = 0; v < n; ++v) trp[(size_t)v + 1] += trp[v];
        std::vector<int32_t> fillp(trp.begin(), trp.end() - 1);
        for (int32_t u = 0; u < n; ++u)
            for (int32_t e = rp[u]; e < rp[u + 1]; ++e) tci[(size_t)fillp[ci[e]]++] = u;
        std::fill(seen.begin(), seen.end(), 0);
        h = 0;
        t = 0;
        q[t++] = 0;
        seen[0] = 1;
        while (h < t) {
            int32_t x = q[h++];
            for (int32_t e = trp[x]; e < trp[x + 1]; ++e)
                if (!seen[tci[e]]) {
                    seen[tci[e]] = 1;
                    q[t++] = tci[e];
                }
        }
        if (t != n)
            return fail(GC_EDISCONNECTED, "directed graph: %lld of %d nodes reach node 0 (not strongly connected)",
                        (long long)t, n);
    }
    return GC_OK;
}

// Nodes grouped into balls of up to 64: the first ball grows breadth-first
// from the node of largest degree over nodes not yet taken, the next from the
// largest-degree node left, and so on.  Sources of one 64-bit batch then lie
// close together, so a node is reached by them at few distinct distances and
// enters the batch's frontier few times (on a grid, a diamond of radius ~6
// instead of a row segment of 64).  Any order gives the same exact results.
static void ball_order(int32_t n, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                       const std::vector<int32_t> &by_degree, std::vector<int32_t> &out,
                       std::vector<int32_t> &rank) {
    out.clear();
    out.reserve((size_t)n);
    std::vector<uint8_t> taken((size_t)n, 0);
    for (const int32_t seed : by_degree) {
        if (taken[seed]) continue;
        const size_t b0 = out.size();
        taken[seed] = 1;
        out.push_back(seed);
        for (size_t h = b0; h < out.size() && out.size() - b0 < 64; ++h) {
            const int32_t u = out[h];
            for (int32_t e = rp[u]; e < rp[u + 1] && out.size() - b0 < 64; ++e) {
                const int32_t v = ci[e];
                if (!taken[v]) {
                    taken[v] = 1;
                    out.push_back(v);
                }
            }
        }
    }
    rank.assign((size_t)n, 0);
    for (int32_t i = 0; i < n; ++i) rank[(size_t)out[i]] = i;
}

// every length >= 1 and, undirected, both rows of an edge with the same length
static int validate_weights(int32_t n, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                            const std::vector<uint8_t> &w, bool directed) {
    for (int32_t u = 0; u < n; ++u)
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            if (w[(size_t)e] == 0) return fail(GC_EINVAL, "row %d: an edge of length 0", u);
            if (directed) continue;
            const int32_t v = ci[(size_t)e];
            const auto it = std::lower_bound(ci.begin() + rp[v], ci.begin() + rp[v + 1], u);
            if (w[(size_t)(it - ci.begin())] != w[(size_t)e])
                return fail(GC_ENOTSYM, "edge %d-%d has different lengths in its two rows", u, v);
        }
    return GC_OK;
}

static int load_graph(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                      bool weighted, const uint8_t *d_weight, uint32_t flags, hipStream_t stream,
                      gc_graph **out) {
    if (!out) return fail(GC_EINVAL, "out is NULL");
    if (n < 1) return fail(GC_EINVAL, "n must be >= 1 (got %d)", n);
    if (nnz < 0 || nnz >= (int64_t)INT32_MAX) return fail(GC_EINVAL, "nnz out of range");
    if (!d_row_ptr || (nnz > 0 && !d_col_idx)) return fail(GC_EINVAL, "NULL CSR array");
    if (weighted && n >= kWeightedMaxN)
        return fail(GC_ERANGE, "weighted graphs: n must be below 2^23 (distances stay below 2^31)");
    gc_graph *g = new (std::nothrow) gc_graph();
    if (!g) return fail(GC_ENOMEM, "no memory for the handle");
    g->n = n;
    g->nnz = nnz;
    g->d_rp = d_row_ptr;
    g->d_ci = d_col_idx;
    g->weighted = weighted;
    g->d_w = d_weight;
    try {
        g->h_rp.resize((size_t)n + 1);
    } catch (...) {
        delete g;
        return fail(GC_ENOMEM, "no memory for row_ptr copy");
    }
    hipError_t e = hipMemcpyAsync(g->h_rp.data(), d_row_ptr, sizeof(int32_t) * ((size_t)n + 1),
                                  hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        delete g;
        return fail(GC_EDEVICE, "copying row_ptr: %s", hipGetErrorString(e));
    }
    const auto &rp = g->h_rp;
    if (rp[0] != 0 || rp[n] != nnz) {
        delete g;
        return fail(GC_EINVAL, "row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
    }
    int32_t md = 0;
    for (int32_t u = 0; u < n; ++u) {
        if (rp[u + 1] < rp[u]) {
            delete g;
            return fail(GC_EINVAL, "row_ptr decreases at row %d", u);
        }
        md = std::max(md, rp[u + 1] - rp[u]);
    }
    g->max_deg = md;
    g->balls = !weighted;  // the balls batch the bit-parallel searches only
    if (const char *e = getenv("GC_BALLS")) g->balls = g->balls && strcmp(e, "0") != 0;
    std::vector<int32_t> ci;
    if ((flags & GC_VALIDATE) || g->balls) {
        try {
            ci.resize((size_t)nnz);
        } catch (...) {
            delete g;
            return fail(GC_ENOMEM, "no memory for the validation copy");
        }
        if (nnz > 0) {
            e = hipMemcpyAsync(ci.data(), d_col_idx, sizeof(int32_t) * (size_t)nnz,
                               hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) {
                delete g;
                return fail(GC_EDEVICE, "copying col_idx: %s", hipGetErrorString(e));
            }
        }
    }
    g->directed = (flags & GC_DIRECTED) != 0;
    if (flags & GC_VALIDATE) {
        int rc = validate_csr(n, nnz, rp, ci, g->directed);
        if (rc != GC_OK) {
            delete g;
            return rc;
        }
    }
    if (weighted) {
        std::vector<uint8_t> hw;
        try {
            hw.resize((size_t)nnz);
        } catch (...) {
            delete g;
            return fail(GC_ENOMEM, "no memory for the length copy");
        }
        if (nnz > 0) {
            e = hipMemcpyAsync(hw.data(), d_weight, (size_t)nnz, hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) {
                delete g;
                return fail(GC_EDEVICE, "copying the lengths: %s", hipGetErrorString(e));
            }
        }
        if (flags & GC_VALIDATE) {
            int rc = validate_weights(n, rp, ci, hw, g->directed);
            if (rc != GC_OK) {
                delete g;
                return rc;
            }
        }
        int32_t wmax = 1;
        for (uint8_t x : hw) wmax = std::max<int32_t>(wmax, x);
        g->wmax = wmax;
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    g->num_cu = cus;
    try {
        g->by_degree.resize((size_t)n);
    } catch (...) {
        delete g;
        return fail(GC_ENOMEM, "no memory for the degree order");
    }
    std::iota(g->by_degree.begin(), g->by_degree.end(), 0);
    std::stable_sort(g->by_degree.begin(), g->by_degree.end(), [&](int32_t x, int32_t y) {
        return (rp[x + 1] - rp[x]) > (rp[y + 1] - rp[y]);
    });
    for (int32_t v = 0; v < n; ++v) {
        const int32_t d = rp[v + 1] - rp[v];
        if (d <= kSplitLongRow) continue;
        const int32_t first = (int32_t)(g->split_chunks.size() / 2);
        for (int32_t c = 0; c < (d + kSplitChunk - 1) / kSplitChunk; ++c) {
            g->split_chunks.push_back(v);
            g->split_chunks.push_back(first);
        }
    }
    if (g->balls) {
        try {
            ball_order(n, rp, ci, g->by_degree, g->by_ball, g->ball_rank);
        } catch (...) {
            delete g;
            return fail(GC_ENOMEM, "no memory for the ball order");
        }
    }
    g->vis_budget = (int64_t)64 << 30;
    if (const char *e = getenv("GC_VIS_BUDGET_MB")) {
        long long v = strtoll(e, nullptr, 10);
        if (v > 0) g->vis_budget = (int64_t)v << 20;
    }
    g->level_wgs_per_cu = 4;
    if (const char *e = getenv("GC_LEVEL_WGS")) {
        long v = strtol(e, nullptr, 10);
        if (v >= 1 && v <= 64) g->level_wgs_per_cu = (int32_t)v;
    }
    g->unroll = 8;
    if (const char *e = getenv("GC_UNROLL")) {
        const long v = strtol(e, nullptr, 10);
        g->unroll = v >= 16 ? 16 : (v >= 8 ? 8 : 4);
    }
    g->learned_pool_pct = 110;
    if (const char *e = getenv("GC_LEARNED_POOL_PCT")) {
        const long v = strtol(e, nullptr, 10);
        if (v >= 110 && v <= 1600) g->learned_pool_pct = (int32_t)v;
    }
    g->min_edges = 512;
    if (const char *e = getenv("GC_MIN_EDGES")) {
        long v = strtol(e, nullptr, 10);
        if (v >= 16) g->min_edges = (int32_t)v;
    }
    g->unroll_small = 4;
    if (const char *e = getenv("GC_UNROLL_SMALL")) g->unroll_small = strtol(e, nullptr, 10) >= 8 ? 8 : 4;
    // adjacency entries per workgroup of small launches: graphs below 2^24 CSR
    // entries (small territories, levels of a few thousand entries) gain from
    // spreading a level over twice the workgroups; large ones (hub rows, more
    // work per workgroup) do not
    g->min_edges_small = nnz < (1LL << 24) ? 256 : 512;
    if (const char *e = getenv("GC_MIN_EDGES_SMALL")) {
        long v = strtol(e, nullptr, 10);
        if (v >= 16) g->min_edges_small = (int32_t)v;
    }
    // frontier log: 16 entries per node, between 8M and 256M entries (20 bytes each)
    g->log_entries = std::min<int64_t>((int64_t)256 << 20, std::max<int64_t>((int64_t)8 << 20, 16LL * n));
    if (const char *e = getenv("GC_LOG_ENTRIES")) {
        long long v = strtoll(e, nullptr, 10);
        if (v > 0) g->log_entries = v;
    }
    if (const char *e = getenv("GC_LEVEL_CAP")) {
        const long v = strtol(e, nullptr, 10);
        if (v >= 1) g->level_cap = (int32_t)std::min<long>(v, INT32_MAX);
    }
    if (const char *e = getenv("GC_ROUND_CAP")) {
        const long long v = strtoll(e, nullptr, 10);
        if (v >= 1) g->wround_cap = (uint32_t)std::min<long long>(v, UINT32_MAX);
    }
    g->touch_entries = 0;
    if (const char *e = getenv("GC_TOUCH_ENTRIES")) {
        long long v = strtoll(e, nullptr, 10);
        if (v > 0) g->touch_entries = v;
    }
    if (weighted) {
        // bucket widths: the gain searches are short and pay per phase, so one
        // phase spans twice the longest edge; the closeness search checks its
        // bound once per phase, so its width comes from the first search's
        // mean distance (this value only when GC_WDELTA_CLOSE sets it)
        g->wdelta_gain = std::min(2 * g->wmax, 65535);
        g->wdelta_close = std::max(1, g->wmax / 2);
        if (const char *e = getenv("GC_WDELTA")) {
            const long v = strtol(e, nullptr, 10);
            if (v >= 1 && v <= 65535) g->wdelta_gain = (int32_t)v;
        }
        if (const char *e = getenv("GC_WDELTA_CLOSE")) {
            const long v = strtol(e, nullptr, 10);
            if (v >= 1 && v <= 65535) {
                g->wdelta_close = (int32_t)v;
                g->wdelta_close_env = true;
            }
        }
        // one slot per resident workgroup of 256 threads (8 per CU), within the record budget
        const int64_t per_slot = (int64_t)kWSlotBytesPerNode * n;
        int64_t slots = std::min<int64_t>(8LL * g->num_cu, std::max<int64_t>(1, g->vis_budget / per_slot));
        if (const char *e = getenv("GC_WSLOTS")) {
            const long long v = strtoll(e, nullptr, 10);
            if (v >= 1 && v <= 65536) slots = v;
        }
        g->wslots = (int32_t)slots;
        if (const char *e = getenv("GC_WCLOSE_THREADS")) g->wclose_threads = strtol(e, nullptr, 10) == 256 ? 256 : 1024;
        // the closeness searches are full SSSPs: fewer, wider workgroups keep
        // per-node state (20 bytes per node each) closer to the caches
        g->wclose_slots = 256;
        if (const char *e = getenv("GC_WCLOSE_SLOTS")) {
            const long long v = strtoll(e, nullptr, 10);
            if (v >= 1 && v <= 65536) g->wclose_slots = (int32_t)v;
        }
        g->wclose_slots = std::min(g->wclose_slots, g->wslots);
    }
    *out = g;
    return GC_OK;
}

extern "C" int gc_load_csr(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                           uint32_t flags, hipStream_t stream, gc_graph **out) {
    return load_graph(n, nnz, d_row_ptr, d_col_idx, false, nullptr, flags, stream, out);
}

extern "C" int gc_load_csr_weighted(int32_t n, int64_t nnz, const int32_t *d_row_ptr,
                                    const int32_t *d_col_idx, const uint8_t *d_weight, uint32_t flags,
                                    hipStream_t stream, gc_graph **out) {
    if (!d_weight && nnz > 0) return fail(GC_EINVAL, "NULL length array");
    return load_graph(n, nnz, d_row_ptr, d_col_idx, true, d_weight, flags, stream, out);
}

extern "C" void gc_free_graph(gc_graph *g) { delete g; }

extern "C" int gc_get_tuning(const gc_graph *g, gc_tuning *out) {
    if (!g || !out) return fail(GC_EINVAL, "NULL argument");
    gc_tuning t{};
    t.unroll = g->unroll;
    t.unroll_small = g->unroll_small;
    t.min_edges = g->min_edges;
    t.min_edges_small = g->min_edges_small;
    t.level_wgs_per_cu = g->level_wgs_per_cu;
    *out = t;
    return GC_OK;
}

extern "C" int gc_set_tuning(gc_graph *g, const gc_tuning *t) {
    if (!g || !t) return fail(GC_EINVAL, "NULL argument");
    if (t->unroll != 4 && t->unroll != 8 && t->unroll != 16)
        return fail(GC_EINVAL, "unroll must be 4, 8 or 16 (got %d)", t->unroll);
    if (t->unroll_small != 4 && t->unroll_small != 8)
        return fail(GC_EINVAL, "unroll_small must be 4 or 8 (got %d)", t->unroll_small);
    if (t->min_edges < 16 || t->min_edges_small < 16)
        return fail(GC_EINVAL, "min_edges and min_edges_small must be >= 16");
    if (t->level_wgs_per_cu < 1 || t->level_wgs_per_cu > 64)
        return fail(GC_EINVAL, "level_wgs_per_cu must be 1..64 (got %d)", t->level_wgs_per_cu);
    g->unroll = t->unroll;
    g->unroll_small = t->unroll_small;
    g->min_edges = t->min_edges;
    g->min_edges_small = t->min_edges_small;
    g->level_wgs_per_cu = t->level_wgs_per_cu;
    return GC_OK;
}

// --------------------------------------------------------------- workspace

namespace {

constexpr size_t kCtrBytes = 4096;

struct WsLayout {
    size_t ctr, dist16, dist8, far, cand, gain, aux, aux2, q0, q1, claim;
    size_t wvis, ly, lr, lb, lo, lz, lvl, act, cutprev, farout, cisplit, rinfo, dist1, order, two,
        tails, total;
    int64_t kmax;       // batches per launch of the device-wide gain engine
    size_t vis_stride;  // words per batch
    int64_t cap;        // frontier log entries (a ring: a power of two)
    int64_t zcap;       // clean-up list entries
    size_t lchunk = 0, lcnt = 0;  // long rows' chunk list and part sizes of the row split
    int64_t nchunk = 0;           // chunks the layout has room for (0: none)
    size_t acc = 0;               // level-0 sums of launch_wide_first (0: no room)
};

constexpr int32_t kMaxLevels = 65536;  // 16-bit distances: at most 65534 levels
constexpr int kFlagSlot = 16;          // int32 counter slot of the overflow flag
constexpr int kMaxdSlot = 17;          // int32 counter slot for max d(S,.)



size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

WsLayout ws_layout(const gc_graph *g) {
    WsLayout L;
    const size_t n = (size_t)g->n;
    size_t o = 0;
    L.ctr = o; o += kCtrBytes;
    L.dist16 = o; o += al256(n * 2 + 4);
    L.dist8 = o; o += al256(n + 4);
    L.far = o; o += 256;
    L.cand = o; o += al256(n * 4);
    L.gain = o; o += al256(n * 8);
    L.aux = o; o += al256(n * 8);
    L.aux2 = o; o += al256(n * 4);
    L.q0 = o; o += al256(n * 4);
    L.q1 = o; o += al256(n * 4);
    L.claim = o; o += al256(((n + 31) / 32) * 4);
    // device-wide engine: per-(batch, node) 32-byte records (visited word and
    // three rotating frontier words) and the frontier log
    L.vis_stride = (n + 31) & ~(size_t)31;
    const int64_t nb_all = ((int64_t)n + 63) / 64;
    const size_t vis_budget = (size_t)g->vis_budget;
    int64_t kmax = (int64_t)(vis_budget / (L.vis_stride * 32));
    kmax = std::max<int64_t>(1, std::min<int64_t>(kmax, nb_all));
    L.kmax = kmax;
    int64_t cap = g->log_entries;
    cap = std::min<int64_t>(cap, 64LL * kmax * (int64_t)n + 128);
    cap = std::max<int64_t>(cap, (int64_t)n + 128);
    // (a level holds fewer than 2^27 entries and 2^35 adjacency entries: the
    // append flags more as an overflow)
    int64_t ring = 1;
    while (ring < cap) ring <<= 1;
    L.cap = ring;
    // the clean-up list names every touched record once: at most n per batch
    L.zcap = g->touch_entries > 0 ? std::max<int64_t>(g->touch_entries, (int64_t)n + 128)
                                  : std::max<int64_t>(cap, std::min<int64_t>(kmax * (int64_t)n, (int64_t)64 << 20));
    L.wvis = o; o += al256((size_t)kmax * L.vis_stride * 32);
    L.ly = o; o += al256((size_t)L.cap * 4);
    L.lr = o; o += al256((size_t)L.cap * 4);
    L.lb = o; o += al256((size_t)L.cap * 4);
    L.lo = o; o += al256((size_t)L.cap * 8);
    L.lz = o; o += al256((size_t)L.zcap * 8);
    L.lvl = o; o += al256((size_t)(kMaxLevels + 2) * sizeof(WideLevel));
    // level-0 sums of launches that fold the roots into level 0 (zero between launches)
    L.acc = o; o += al256((size_t)kFirstMaxSrc * 8);
    L.act = o; o += al256((size_t)kmax * 8);
    L.cutprev = o; o += al256(n * 16);
    L.farout = o; o += al256(n * 8);
    // rows split by d(S,.) at the first gain round (see WideArgs::rinfo)
    L.cisplit = o; o += al256((size_t)g->nnz * 4 + 4);
    L.rinfo = o; o += al256(n * 16);
    L.dist1 = o; o += al256(n * 2 + 4);
    // graph tables written by gc_workspace_init: the closeness search order
    // and the sum of neighbour degrees of every node
    L.order = o; o += al256(n * 4);
    L.two = o; o += al256(n * 8);
    // early exit: a histogram of d(S,.) and the bound's tail table T
    L.tails = o; o += al256((size_t)2 * (kMaxLevels + 2) * 8);
    // the row split's chunks of long rows (see launch_row_split)
    L.nchunk = (int64_t)g->split_chunks.size() / 2;
    L.lchunk = o; o += al256((size_t)L.nchunk * 8);
    L.lcnt = o; o += al256((size_t)L.nchunk * 8);
    L.total = o;
    return L;
}

struct Ws {
    WsLayout L;
    char *base;
    size_t bytes;
    int32_t *ctr() const { return reinterpret_cast<int32_t *>(base + L.ctr); }
    uint16_t *dist16() const { return reinterpret_cast<uint16_t *>(base + L.dist16); }
    uint8_t *dist8() const { return reinterpret_cast<uint8_t *>(base + L.dist8); }
    int64_t *far() const { return reinterpret_cast<int64_t *>(base + L.far); }
    int32_t *cand() const { return reinterpret_cast<int32_t *>(base + L.cand); }
    int64_t *gain() const { return reinterpret_cast<int64_t *>(base + L.gain); }
    int64_t *aux() const { return reinterpret_cast<int64_t *>(base + L.aux); }
    int32_t *aux2() const { return reinterpret_cast<int32_t *>(base + L.aux2); }
    int32_t *flags() const { return ctr() + kFlagSlot; }
    // learned-order region (after the main layout; see gc_mlp_ws_bytes)
    struct Mlp {
        float *feat;
        float *score;
        int64_t *ub;
        int32_t *last_eval;
        uint16_t *dist_at_eval;
    };
    Mlp mlp(int64_t n) const {
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        char *p = base + L.total;
        Mlp m;
        m.feat = reinterpret_cast<float *>(p); p += al((size_t)n * 8 * 4);
        m.score = reinterpret_cast<float *>(p); p += al((size_t)n * 4);
        m.ub = reinterpret_cast<int64_t *>(p); p += al((size_t)n * 8);
        m.last_eval = reinterpret_cast<int32_t *>(p); p += al((size_t)n * 4);
        m.dist_at_eval = reinterpret_cast<uint16_t *>(p);
        return m;
    }
    int32_t *maxd() const { return ctr() + kMaxdSlot; }
    int64_t *words() const { return reinterpret_cast<int64_t *>(ctr() + C_I64_BASE) + L_WORDS; }
    int64_t *zcnt() const { return reinterpret_cast<int64_t *>(ctr() + C_I64_BASE) + L_TOUCHED; }
    int64_t *cuts() const { return reinterpret_cast<int64_t *>(ctr() + C_I64_BASE) + L_CUTS; }
    unsigned long long *tail_hist() const { return reinterpret_cast<unsigned long long *>(base + L.tails); }
    int64_t *tail_T() const {
        return reinterpret_cast<int64_t *>(base + L.tails + (size_t)(kMaxLevels + 2) * 8);
    }
    int64_t *hdr() const { return reinterpret_cast<int64_t *>(ctr() + C_I64_BASE) + L_HDR; }
    int32_t *order() const { return reinterpret_cast<int32_t *>(base + L.order); }
    int64_t *two() const { return reinterpret_cast<int64_t *>(base + L.two); }
    WideArgs wide() const {
        WideArgs a{};
        a.vis = reinterpret_cast<uint64_t *>(base + L.wvis);
        a.vis_stride = L.vis_stride;
        a.ly = reinterpret_cast<int32_t *>(base + L.ly);
        a.lr = reinterpret_cast<int32_t *>(base + L.lr);
        a.lb = reinterpret_cast<int32_t *>(base + L.lb);
        a.lo = reinterpret_cast<int64_t *>(base + L.lo);
        a.lz = reinterpret_cast<int64_t *>(base + L.lz);
        a.zcnt = reinterpret_cast<unsigned long long *>(zcnt());
        a.cap = L.cap;
        a.zcap = L.zcap;
        a.lvl = reinterpret_cast<WideLevel *>(base + L.lvl);
        a.flags = flags();
        a.min_edges = 1024;
        return a;
    }
};

int get_ws(const gc_graph *g, void *d_ws, size_t ws_bytes, Ws *w) {
    if (!g) return fail(GC_EINVAL, "graph is NULL");
    w->L = ws_layout(g);
    if (!d_ws) return fail(GC_EWORKSPACE, "workspace is NULL");
    if (((uintptr_t)d_ws & 255) != 0) return fail(GC_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < w->L.total)
        return fail(GC_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, w->L.total);
    w->bytes = ws_bytes;
    w->base = reinterpret_cast<char *>(d_ws);
    return GC_OK;
}

// ---- weighted graphs: workspace of the per-workgroup searches
// counter block (256 bytes): work counter, flags, best farness, argmin
// result, sum, one node id, F(S); then d(S,.) (int32), per-candidate outputs,
// the candidate list, and the slots (records, then work lists)
struct WLayout {
    size_t ctr, dist, out, edges, vis, cand, d0, t0, hist, enc, rec, lists, total;
    int64_t t0_cap;  // entries of the closeness bound's tail table
};

WLayout wlayout(const gc_graph *g) {
    WLayout L{};
    const size_t n = (size_t)g->n, slots = (size_t)g->wslots;
    size_t o = 0;
    L.ctr = o; o += 256;
    L.dist = o; o += al256(n * 4);
    L.out = o; o += al256(n * 8);
    L.edges = o; o += al256(n * 8);
    L.vis = o; o += al256(n * 4);
    L.cand = o; o += al256(n * 4);
    // the landmark distances of the closeness search and their tail sums,
    // for distances up to min(255 (n - 1), 2^22)
    L.t0_cap = std::min<int64_t>(255LL * (int64_t)(n - 1) + 2, (int64_t)1 << 22);
    L.d0 = o; o += al256(n * 4);
    L.t0 = o; o += al256((size_t)L.t0_cap * 8);
    L.hist = o; o += al256((size_t)L.t0_cap * 4);
    L.enc = o; o += al256(slots * n * 4);
    L.rec = o; o += al256(slots * n * sizeof(WRec));
    L.lists = o; o += al256(slots * n * kWLists * 4);
    L.total = o;
    return L;
}

struct WWs {
    WLayout L;
    char *base;
    uint32_t *next() const { return reinterpret_cast<uint32_t *>(base + L.ctr); }
    int32_t *flags() const { return reinterpret_cast<int32_t *>(base + L.ctr + 4); }
    unsigned long long *best() const { return reinterpret_cast<unsigned long long *>(base + L.ctr + 8); }
    int64_t *res() const { return reinterpret_cast<int64_t *>(base + L.ctr + 16); }
    unsigned long long *sum() const { return reinterpret_cast<unsigned long long *>(base + L.ctr + 32); }
    int32_t *one() const { return reinterpret_cast<int32_t *>(base + L.ctr + 40); }
    int64_t *far() const { return reinterpret_cast<int64_t *>(base + L.ctr + 48); }
    int32_t *dist() const { return reinterpret_cast<int32_t *>(base + L.dist); }
    int64_t *out() const { return reinterpret_cast<int64_t *>(base + L.out); }
    int64_t *edges() const { return reinterpret_cast<int64_t *>(base + L.edges); }
    int32_t *vis() const { return reinterpret_cast<int32_t *>(base + L.vis); }
    int32_t *cand() const { return reinterpret_cast<int32_t *>(base + L.cand); }
    int32_t *d0() const { return reinterpret_cast<int32_t *>(base + L.d0); }
    int64_t *t0() const { return reinterpret_cast<int64_t *>(base + L.t0); }
    uint32_t *hist() const { return reinterpret_cast<uint32_t *>(base + L.hist); }
    int32_t *maxd0() const { return reinterpret_cast<int32_t *>(base + L.ctr + 56); }
    uint32_t *enc() const { return reinterpret_cast<uint32_t *>(base + L.enc); }
    WRec *rec() const { return reinterpret_cast<WRec *>(base + L.rec); }
    int32_t *lists() const { return reinterpret_cast<int32_t *>(base + L.lists); }
};

int get_wws(const gc_graph *g, void *d_ws, size_t ws_bytes, WWs *w) {
    if (!g) return fail(GC_EINVAL, "graph is NULL");
    w->L = wlayout(g);
    if (!d_ws) return fail(GC_EWORKSPACE, "workspace is NULL");
    if (((uintptr_t)d_ws & 255) != 0) return fail(GC_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < w->L.total)
        return fail(GC_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, w->L.total);
    w->base = reinterpret_cast<char *>(d_ws);
    return GC_OK;
}

// ---------------------------------------------------------- weighted graphs
//
// The same operations on a graph with integer edge lengths: every search is
// one workgroup's bucketed search (gc_weighted.hip) and d(S,.) is int32.

struct WClose {
    int32_t delta = 0;          // bucket width (0: the graph's default)
    const int32_t *d0 = nullptr;
    const int64_t *t0 = nullptr;
    int32_t t0_len = 0;
};

int wlaunch(const gc_graph *g, const WWs &w, int32_t mode, int32_t *dS, const int32_t *cand, int32_t count,
            int64_t *out, int64_t *edges, int32_t *vis, int64_t thr, unsigned long long *best, bool one,
            hipStream_t s, const WClose *wc = nullptr) {
    if (count <= 0) return GC_OK;
    HIP_OK(launch_fill_u32(w.next(), 1, 0u, s));
    WArgs a{};
    a.rp = g->d_rp;
    a.ci = g->d_ci;
    a.w = g->d_w;
    a.n = g->n;
    a.mode = mode;
    a.dS = dS;
    a.cand = cand;
    a.count = count;
    a.next = w.next();
    a.out = out;
    a.edges = edges;
    a.visited = vis;
    a.enc = w.enc();
    a.rec = w.rec();
    a.lists = w.lists();
    a.delta = mode == W_CLOSE ? g->wdelta_close : g->wdelta_gain;
    a.thr = thr;
    a.best = best;
    a.flags = w.flags();
    a.max_rounds = g->wround_cap;
    if (wc) {
        if (wc->delta > 0) a.delta = wc->delta;
        a.d0 = wc->d0;
        a.t0 = wc->t0;
        a.t0_len = wc->t0_len;
    }
    HIP_OK(one ? launch_wsearch_one(a, s)
               : mode == W_CLOSE ? launch_wsearch(a, g->wclose_slots, g->wclose_threads, s)
                                 : launch_wsearch(a, g->wslots, 256, s));
    return GC_OK;
}

// The k nodes of least F({v}) (Section 3.1 with k >= 1), in increasing
// (F, id) order.  Candidates go in decreasing degree order.  The first one,
// v0, is a full search that writes d0 = d(v0,.): its farness is the first
// cut threshold, d0 the landmark of the cut bound (with the tail table T0
// built from a histogram of d0), and its mean distance sets the bucket width
// (a sixteenth of it, so the bound is tested many times before the search
// passes the mean).  k = 1: one launch over the rest, each search cut against
// the best farness any search has finished with (a device atomic).  k > 1:
// launches of a few candidates per slot, each cut against the k-th best
// farness of the launches before.  A cut search's farness exceeds the
// threshold, so it is not among the k.
int run_wclosest(const gc_graph *g, const WWs &w, hipStream_t s, int32_t k,
                 std::vector<std::pair<int64_t, int32_t>> *top, int64_t *sources = nullptr) {
    const int32_t n = g->n;
    HIP_OK(hipMemcpyAsync(w.cand(), g->by_degree.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.flags()), 1, 0u, s));
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.d0()), (size_t)n, 0x7FFFFFFFu, s));
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.maxd0()), 1, 0u, s));
    int rc = wlaunch(g, w, W_WRITE, w.d0(), w.cand(), 1, w.res(), nullptr, nullptr, 0, nullptr, true, s);
    if (rc) return rc;
    HIP_OK(launch_wsum(w.d0(), n, w.best(), s));
    HIP_OK(launch_wmax(w.d0(), n, w.maxd0(), s));
    int64_t F0 = 0;
    int32_t maxd0 = 0;
    HIP_OK(hipMemcpyAsync(&F0, w.best(), sizeof(F0), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(&maxd0, w.maxd0(), sizeof(maxd0), hipMemcpyDeviceToHost, s));
    int32_t flag0 = 0;
    HIP_OK(hipMemcpyAsync(&flag0, w.flags(), sizeof(flag0), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (flag0 & 2) return fail(GC_EDEVICE, "a search passed the round cap (GC_ROUND_CAP = %u)", g->wround_cap);
    if (maxd0 == INT32_MAX) return fail(GC_EDISCONNECTED, "node %d does not reach every node", g->by_degree[0]);
    HIP_OK(launch_set_i64(w.out(), F0, s));
    WClose wc;
    wc.delta = g->wdelta_close_env ? g->wdelta_close
                                   : (int32_t)std::min<int64_t>(65535, std::max<int64_t>(1, F0 / std::max(1, n - 1) / 16));
    wc.d0 = w.d0();
    if ((int64_t)maxd0 + 2 <= w.L.t0_cap) {
        // T0[M] = sum_w max(0, d0(w) - M) = T0[M + 1] + #{w : d0(w) > M}
        const int32_t len = maxd0 + 2;
        std::vector<uint32_t> h((size_t)len);
        std::vector<int64_t> t((size_t)len, 0);
        HIP_OK(launch_fill_u32(w.hist(), (size_t)len, 0u, s));
        HIP_OK(launch_whist(w.d0(), n, w.hist(), s));
        HIP_OK(hipMemcpyAsync(h.data(), w.hist(), sizeof(uint32_t) * (size_t)len, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        int64_t above = 0;  // #{w : d0(w) > M}
        for (int32_t M = len - 2; M >= 0; --M) {
            above += h[(size_t)M + 1];
            t[(size_t)M] = t[(size_t)M + 1] + above;
        }
        HIP_OK(hipMemcpyAsync(w.t0(), t.data(), sizeof(int64_t) * (size_t)len, hipMemcpyHostToDevice, s));
        HIP_OK(hipStreamSynchronize(s));  // t lives on this stack frame
        wc.t0 = w.t0();
        wc.t0_len = len;
    }
    top->clear();
    int32_t flag = 0;
    if (k == 1) {
        // On an undirected graph a node v whose only neighbour is h (edge of
        // length e) reaches every other node through h, so F({v}) =
        // F({h}) + (n - 2) e > F({h}) for n >= 3: it cannot be the closest.
        // The degree order puts such nodes last.
        int32_t cnt = n;
        if (!g->directed && n >= 3)
            while (cnt > 1 && g->h_rp[(size_t)g->by_degree[(size_t)cnt - 1] + 1] -
                                      g->h_rp[(size_t)g->by_degree[(size_t)cnt - 1]] == 1)
                --cnt;
        rc = wlaunch(g, w, W_CLOSE, nullptr, w.cand() + 1, cnt - 1, w.out() + 1, nullptr, nullptr,
                     std::numeric_limits<int64_t>::max(), w.best(), false, s, &wc);
        if (rc) return rc;
        HIP_OK(launch_wargmin(w.out(), w.cand(), cnt, w.res(), s));
        if (sources) *sources = cnt;
        int64_t res[2] = {-1, -1};
        HIP_OK(hipMemcpyAsync(res, w.res(), sizeof(res), hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(&flag, w.flags(), sizeof(flag), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        if (flag & 2) return fail(GC_EDEVICE, "a search passed the round cap (GC_ROUND_CAP = %u)", g->wround_cap);
        if (flag || res[1] < 0) return fail(GC_EDISCONNECTED, "a closeness search did not reach every node");
        top->emplace_back(res[0], (int32_t)res[1]);
        return GC_OK;
    }
    top->emplace_back(F0, g->by_degree[0]);
    const int32_t chunk = std::max<int32_t>(1, 4 * g->wslots);
    std::vector<int64_t> hout((size_t)std::min<int32_t>(chunk, n));
    for (int32_t start = 1; start < n;) {
        const int32_t cnt = std::min<int32_t>(chunk, n - start);
        const int64_t thr = (int32_t)top->size() < k ? std::numeric_limits<int64_t>::max()
                                                     : (*top)[(size_t)k - 1].first;
        rc = wlaunch(g, w, W_CLOSE, nullptr, w.cand() + start, cnt, w.out() + start, nullptr, nullptr, thr,
                     nullptr, false, s, &wc);
        if (rc) return rc;
        HIP_OK(hipMemcpyAsync(hout.data(), w.out() + start, sizeof(int64_t) * (size_t)cnt, hipMemcpyDeviceToHost,
                              s));
        HIP_OK(hipStreamSynchronize(s));
        for (int32_t j = 0; j < cnt; ++j)
            if (hout[(size_t)j] >= 0) top->emplace_back(hout[(size_t)j], g->by_degree[(size_t)start + j]);
        std::sort(top->begin(), top->end());
        if ((int32_t)top->size() > k) top->resize((size_t)k);
        start += cnt;
    }
    HIP_OK(hipMemcpyAsync(&flag, w.flags(), sizeof(flag), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (flag & 2) return fail(GC_EDEVICE, "a search passed the round cap (GC_ROUND_CAP = %u)", g->wround_cap);
    if (flag || (int32_t)top->size() < k) return fail(GC_EDISCONNECTED, "a closeness search did not reach every node");
    if (sources) *sources = n;
    return GC_OK;
}

// add `node` to S: d(S,.) <- min(d(S,.), d(node,.)) by the pruned search,
// and F(S) in *d_far (S = {}: the sum of the new distances; else minus the
// gain, which the search leaves in w.res()[0])
int run_wupdate(const gc_graph *g, const WWs &w, int32_t node, int32_t *dS, int64_t *d_far, bool s_empty,
                hipStream_t s) {
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.one()), 1, (uint32_t)node, s));
    int rc = wlaunch(g, w, W_WRITE, dS, w.one(), 1, w.res(), nullptr, nullptr, 0, nullptr, true, s);
    if (rc) return rc;
    if (s_empty) HIP_OK(launch_wsum(dS, g->n, reinterpret_cast<unsigned long long *>(d_far), s));
    else HIP_OK(launch_wsub(d_far, w.res(), s));
    return GC_OK;
}

}  // namespace

extern "C" int gc_workspace_size(const gc_graph *g, int32_t bitset_width, size_t *bytes) {
    if (!g || !bytes) return fail(GC_EINVAL, "NULL argument");
    if (bitset_width != 0 && bitset_width != 64)
        return fail(GC_EINVAL, "bitset_width must be 64 or 0");
    if (g->weighted) {
        *bytes = wlayout(g).total;
        return GC_OK;
    }
    WsLayout L = ws_layout(g);
    *bytes = L.total + gc_mlp_ws_bytes(g->n);
    return GC_OK;
}

namespace {

// value of the workspace stamp for this graph
int64_t ws_stamp(const gc_graph *g) {
    return (int64_t)(0x4743575350414345ull ^ ((uint64_t)g->n << 1) ^ ((uint64_t)g->nnz << 29));
}

// search order and two-hop sums of the graph into the workspace, then the stamp
int write_graph_tables(const gc_graph *g, const Ws &w, hipStream_t s) {
    HIP_OK(hipMemcpyAsync(w.order(), g->search_order().data(), sizeof(int32_t) * (size_t)g->n,
                          hipMemcpyHostToDevice, s));
    HIP_OK(launch_twohop_i64(g->d_rp, g->d_ci, g->n, w.two(), s));
    HIP_OK(launch_set_i64(w.hdr(), ws_stamp(g), s));
    return GC_OK;
}

// the graph tables, rebuilt if the workspace lacks the stamp (synchronises)
int ensure_graph_tables(const gc_graph *g, const Ws &w, hipStream_t s) {
    int64_t stamp = 0;
    HIP_OK(hipMemcpyAsync(&stamp, w.hdr(), sizeof(stamp), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return stamp == ws_stamp(g) ? GC_OK : write_graph_tables(g, w, s);
}

}  // namespace

extern "C" int gc_workspace_init(const gc_graph *g, void *d_ws, size_t ws_bytes, hipStream_t stream) {
    if (g && g->weighted) {
        // every record of every slot starts at zero (untouched)
        WWs ww;
        int rc = get_wws(g, d_ws, ws_bytes, &ww);
        if (rc) return rc;
        HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(ww.base), ww.L.total / 4, 0u, stream));
        return GC_OK;
    }
    Ws w;
    int rc = get_ws(g, d_ws, ws_bytes, &w);
    if (rc) return rc;
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.base), w.L.total / 4, 0u, stream));
    return write_graph_tables(g, w, stream);
}

// ------------------------------------------------------------- operations

namespace {

// Set on the worker threads of the multi-job engines: their gain launches
// sum per-source results in LDS slots (WideArgs::pack == 2), which pays when
// several jobs' launches share the GPU's atomic units and costs a little when
// one launch has the chip to itself.
thread_local bool t_slot_sums = false;
struct SlotSums {  // on for the lifetime of a worker's loop (also when it runs on the caller's thread)
    bool prev;
    SlotSums() : prev(t_slot_sums) { t_slot_sums = true; }
    ~SlotSums() { t_slot_sums = prev; }
};

// Byte range [lo, hi) of a worker's workspace known to hold zeros between the
// jobs of gc_greedy_many / gc_greedy_batch: the wide engine's records of the
// last job (every call of the engine returns the records it touched to zero;
// an overflow clears them all).
struct ZeroRange {
    size_t lo = 0, hi = 0;
};

hipError_t fill_zero(char *base, size_t lo, size_t hi, hipStream_t s) {
    if (hi <= lo) return hipSuccess;
    return launch_fill_u32(reinterpret_cast<uint32_t *>(base + lo), (hi - lo) / 4, 0u, s);
}

// gc_workspace_init for the next job on a worker's workspace: zero everything
// but the frontier log and clean-up list (written before they are read) and
// the part of the record range already known to be zero.  `z` is cleared here
// and set to this job's record range by the caller once the job has ended
// without error.
int ws_init_reuse(const gc_graph *g, void *d_ws, size_t ws_bytes, hipStream_t s, ZeroRange &z) {
    const ZeroRange known = z;
    z = ZeroRange{};
    if (g->weighted) return gc_workspace_init(g, d_ws, ws_bytes, s);
    Ws w;
    int rc = get_ws(g, d_ws, ws_bytes, &w);
    if (rc) return rc;
    const size_t rlo = w.L.wvis, rhi = w.L.ly;  // records (all of [wvis, ly))
    HIP_OK(fill_zero(w.base, 0, rlo, s));
    if (known.hi <= rlo || known.lo >= rhi) {
        HIP_OK(fill_zero(w.base, rlo, rhi, s));
    } else {
        HIP_OK(fill_zero(w.base, rlo, known.lo, s));
        HIP_OK(fill_zero(w.base, known.hi, rhi, s));
    }
    HIP_OK(fill_zero(w.base, w.L.lvl, w.L.total, s));
    return write_graph_tables(g, w, s);
}

// the record range ws_init_reuse may take as zero after a job on g ended
ZeroRange ws_record_range(const gc_graph *g) {
    ZeroRange r;
    if (g->weighted) return r;
    const WsLayout L = ws_layout(g);
    r.lo = L.wvis;
    r.hi = L.ly;
    return r;
}

int bfs_grid(const gc_graph *g) {
    return std::max(1, std::min(4 * g->num_cu, (g->n + 3) / 4 + 1));
}

// Level-synchronous BFS from root over d_dist (pruned; full when S = {}).
// nlev >= 0: launch exactly nlev levels without synchronising (a pruned BFS
// needs at most max d(S,.) - 1); nlev < 0: launch chunks of levels until the
// frontier is empty (synchronises), reporting the deepest level in *last and
// the nodes reached in *claimed.
int run_update(const gc_graph *g, const Ws &w, int32_t root, void *d_dist, int dist_bytes,
               int64_t *d_far, hipStream_t s, int32_t *last, int32_t *claimed,
               int32_t nlev = -1) {
    BfsArgs a;
    a.rp = g->d_rp;
    a.ci = g->d_ci;
    a.n = g->n;
    a.dist = d_dist;
    a.q0 = reinterpret_cast<int32_t *>(w.base + w.L.q0);
    a.q1 = reinterpret_cast<int32_t *>(w.base + w.L.q1);
    a.claim = reinterpret_cast<uint32_t *>(w.base + w.L.claim);
    a.ctr = w.ctr();
    a.full = 0;
    HIP_OK(launch_bfs_init(a, dist_bytes, root, s));
    const int grid = bfs_grid(g);
    if (nlev >= 0) {
        if (int rc = level_cap_check(g, nlev)) return rc;
        for (int32_t L = 0; L < nlev; ++L) HIP_OK(launch_bfs_level(a, dist_bytes, L, grid, s));
        HIP_OK(launch_bfs_finish(a, d_far, s));
        return GC_OK;
    }
    int32_t level = 0;
    int chunk = 4;
    int32_t h[8];
    for (;;) {
        for (int i = 0; i < chunk; ++i) HIP_OK(launch_bfs_level(a, dist_bytes, level + i, grid, s));
        level += chunk;
        HIP_OK(hipMemcpyAsync(h, w.ctr(), sizeof(h), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        if (h[C_BFS_CNT0 + level % 3] == 0) break;
        if (int rc = level_cap_check(g, level)) return rc;
        chunk = std::min(chunk * 2, 64);
    }
    HIP_OK(launch_bfs_finish(a, d_far, s));
    if (last) *last = h[C_BFS_LAST];
    if (claimed) *claimed = h[C_BFS_CLAIMED];
    return GC_OK;
}

int wide_grid(const gc_graph *g) { return g->level_wgs_per_cu * g->num_cu; }

// Rows split by the distances a gain or update launch prunes against (see
// WideArgs::rinfo); valid while d(S,.) stays at or below those distances.
struct Split {
    const int32_t *ci = nullptr;
    const int4 *rinfo = nullptr;
    const void *dist1 = nullptr;
};

int build_split(const gc_graph *g, const Ws &w, const void *d_dist, int dist_bytes, hipStream_t s,
                Split *out) {
    int32_t *ci = reinterpret_cast<int32_t *>(w.base + w.L.cisplit);
    int4 *ri = reinterpret_cast<int4 *>(w.base + w.L.rinfo);
    void *d1 = w.base + w.L.dist1;
    // long rows by chunks when the layout holds their list (uploaded here, so
    // that any workspace of the graph works)
    int32_t *chunks = nullptr, *cnt = nullptr;
    int32_t nch = 0;
    if (w.L.nchunk > 0 && (int64_t)g->split_chunks.size() == 2 * w.L.nchunk) {
        chunks = reinterpret_cast<int32_t *>(w.base + w.L.lchunk);
        cnt = reinterpret_cast<int32_t *>(w.base + w.L.lcnt);
        nch = (int32_t)w.L.nchunk;
        HIP_OK(hipMemcpyAsync(chunks, g->split_chunks.data(), sizeof(int32_t) * g->split_chunks.size(),
                              hipMemcpyHostToDevice, s));
    }
    HIP_OK(launch_row_split(g->d_rp, g->d_ci, g->n, d_dist, dist_bytes, ci, ri, d1, chunks, nch, cnt, s));
    out->ci = ci;
    out->rinfo = ri;
    out->dist1 = d1;
    return GC_OK;
}

void apply_split(WideArgs &a, const Split *sp) {
    if (!sp || !sp->rinfo) return;
    a.ci = sp->ci;
    a.rinfo = sp->rinfo;
    a.dist1 = sp->dist1;
}

// Marginal gains of count candidates with the device-wide engine.
// nlev = number of BFS levels to expand (max d(S,.) - 1 suffices; < 0: measure
// it).  d_cand may be device memory or host-mapped pinned memory.  With
// host-mapped hm_gain/hm_edges/hm_flag (device pointers of pinned buffers) the
// final kernel writes the results there and no copy call is needed; h_gain/
// h_edges are their host views (or plain host buffers filled by copies).
// Synchronises the stream once to check for log overflow; an overflowed
// launch is redone with fewer batches (then fewer sources) per launch.
struct HostIO {
    int64_t *hm_gain = nullptr;   // device pointer of a pinned buffer
    int64_t *hm_edges = nullptr;
    int32_t *hm_flag = nullptr;
    volatile int32_t *h_flag = nullptr;  // host view of hm_flag
    // done word (device pointer and host view of one pinned int64): the last
    // launch of a call writes its sequence number there once its results are
    // in the mapped buffers, so the host can wait by polling
    int64_t *hm_done = nullptr;
    volatile int64_t *h_done = nullptr;
    int64_t seq = 0;
    // optional: max d(S,.) as last computed on the device (maxd_src), copied by
    // the last launch to the host-mapped hm_maxd
    const int32_t *maxd_src = nullptr;
    int32_t *hm_maxd = nullptr;
    // device copies of the lazy-loop state (learned order features)
    int64_t *ub = nullptr;
    int32_t *last_eval = nullptr;
    uint16_t *dist_at_eval = nullptr;
    int32_t round = 0;
    // optional: GPU time of each call from ev0 (start) to ev1 (all launches
    // done), added to *gpu_ms
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double *gpu_ms = nullptr;
    // launches of at most kFirstMaxSrc sources run their roots and level 0 as
    // one kernel (launch_wide_first) where its conditions hold
    bool first_level = false;
    // optional: candidate lists in pinned memory, seen by the device at
    // cand_dev and by the host at cand_host (cand_len ids); a launch whose
    // candidates lie there gets them as a kernel argument and a grid cut to
    // its level-0 adjacency entries.  Only for lists the host wrote: ids that
    // a kernel writes there are not in the host's view at enqueue time.
    const int32_t *cand_dev = nullptr;
    const int32_t *cand_host = nullptr;
    size_t cand_len = 0;
};

struct LaunchShape {
    int64_t kb = 0;   // batches per launch (0: as many as fit)
    int32_t spb = 64; // sources per batch
};

// Early exit inside the candidates' BFS (see k_gain_cut): the tail table of
// the bound for the current d(S,.), max d(S,.), and the threshold every source
// of the call is tested against.
struct CutSpec {
    const int64_t *T = nullptr;
    int32_t maxd = 0;
    int64_t thr = 0;
    int32_t thr_id = -1;
};

// phase: kGainsRun launches and waits; kGainsLaunch only enqueues (one
// launch over all candidates with host-mapped results: io->hm_done set and the
// candidates fit one chunk; *queued tells whether it did, else it ran the
// call through); kGainsWait then waits for that launch (redoing it on an
// overflow) with the same arguments.
enum GainsPhase { kGainsRun = 0, kGainsLaunch = 1, kGainsWait = 2 };

int run_gains(const gc_graph *g, const Ws &w, const void *d_dist, int dist_bytes,
              const int32_t *d_cand, int32_t count, int64_t *d_gain, int64_t *d_edges,
              int32_t *d_vis, hipStream_t s, int32_t nlev, int64_t *h_gain = nullptr,
              int64_t *h_edges = nullptr, const HostIO *io = nullptr,
              LaunchShape *shape = nullptr, const Split *split = nullptr,
              bool timing_started = false, int phase = kGainsRun, bool *queued = nullptr,
              const CutSpec *cut = nullptr) {
    if (queued) *queued = false;
    if (count <= 0) return GC_OK;
    if (cut && cut->thr_id < 0) cut = nullptr;  // no threshold yet: nothing to cut against
    if (phase == kGainsLaunch && (nlev < 0 || !io || !io->hm_flag || !io->hm_done)) phase = kGainsRun;
    if (nlev < 0) {
        int32_t maxd = 0;
        HIP_OK(launch_max_dist(d_dist, dist_bytes, g->n, w.maxd(), s));
        HIP_OK(hipMemcpyAsync(&maxd, w.maxd(), sizeof(maxd), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        nlev = std::max(maxd - 1, 0);
    }
    nlev = std::min(nlev, kMaxLevels - 1);
    if (int rc = level_cap_check(g, nlev)) return rc;
    const bool mapped = io && io->hm_flag;
    const int grid = wide_grid(g);
    const bool timed = io && io->ev0 && io->gpu_ms;
    if (phase != kGainsWait) {
        if (g_timing && !timing_started) HIP_OK(hipEventRecord(g_ev0, s));
        if (timed) HIP_OK(hipEventRecord(io->ev0, s));
    }
    // batches per launch and sources per batch; a caller-kept shape carries
    // what an earlier overflow taught across calls
    int64_t kb = (shape && shape->kb > 0) ? std::min<int64_t>(shape->kb, w.L.kmax) : w.L.kmax;
    int32_t spb = shape ? shape->spb : 64;
    if (phase == kGainsLaunch && count > kb * spb) phase = kGainsRun;
    int64_t done = 0;
    while (done < count) {
        // launch chunks of kb batches, then check the overflow flag once
        const int64_t per = kb * spb;
        int32_t tag = 0;
        int64_t off = phase == kGainsWait ? count : done;  // (already launched)
        while (off < count) {
            WideArgs a = w.wide();
            a.unroll = g->unroll;
            a.min_edges = g->min_edges;
            a.rp = g->d_rp;
            a.ci = g->d_ci;
            a.n = g->n;
            a.dist = d_dist;
            a.src = d_cand + off;
            a.nsrc = std::min<int64_t>(per, count - off);
            a.spb = spb;
            if (a.nsrc <= 1024) {
                // small launches: narrower steps keep more of each workgroup busy
                a.unroll = g->unroll_small;
                a.min_edges = g->min_edges_small;
            }
            a.gain = d_gain + off;
            a.edges = d_edges ? d_edges + off : nullptr;
            a.visited = d_vis ? d_vis + off : nullptr;
            a.tag = ++tag;
            a.dist_bytes = dist_bytes;
            a.words = w.words();
            apply_split(a, split);
            // one atomic per claim for gain and edge count when neither can
            // overflow its field: edges <= nnz, gain <= n * max d(S,.)
            a.pack = d_edges && g->nnz < (1ll << kPackShift) &&
                     (int64_t)g->n * (int64_t)(nlev + 1) < (1ll << (62 - kPackShift));
            if (a.pack && t_slot_sums) a.pack = 2;
            if (cut) {
                // the cut test reads each source's gain, reach and adjacency
                // between levels: separate counters, per-launch scratch
                a.pack = 0;
                if (!a.edges) a.edges = w.aux() + off;
                if (!a.visited) a.visited = w.aux2() + off;
                a.active = reinterpret_cast<unsigned long long *>(w.base + w.L.act);
                a.prev = reinterpret_cast<int64_t *>(w.base + w.L.cutprev);
                a.far_out = reinterpret_cast<int64_t *>(w.base + w.L.farout);
                a.cut_gain = 1;
                a.cut_T = cut->T;
                a.cut_maxd = cut->maxd;
                a.cut_thr = cut->thr;
                a.cut_id = cut->thr_id;
                a.cut_count = reinterpret_cast<unsigned long long *>(w.cuts());
            }
            if (mapped) {
                a.h_gain = io->hm_gain ? io->hm_gain + off : nullptr;
                a.h_edges = io->hm_edges ? io->hm_edges + off : nullptr;
                a.h_flag = io->hm_flag;
                if (io->hm_done && off + a.nsrc >= count) {
                    a.h_done = io->hm_done;
                    a.seq = ++const_cast<HostIO *>(io)->seq;
                    a.maxd_src = io->maxd_src;
                    a.h_maxd = io->maxd_src ? io->hm_maxd : nullptr;
                }
            }
            if (io && io->ub) {
                a.ub_out = io->ub;
                a.le_out = io->last_eval;
                a.dsat_out = io->dist_at_eval;
                a.round = io->round;
            }
            if (cut) {
                // roots, then the test after every level that a deeper level can follow
                HIP_OK(launch_wide_begin(a, dist_bytes, nlev, s));
                HIP_OK(launch_gain_cut(a, 0, s));
                for (int32_t L = 0; L < nlev; ++L) {
                    HIP_OK(launch_wide_levels(a, dist_bytes, L, L + 1, grid, s));
                    if (L + 1 < nlev) HIP_OK(launch_gain_cut(a, L + 1, s));
                }
                HIP_OK(launch_wide_end(a, nlev, grid, s));
            } else if (io && io->first_level && w.L.acc && a.pack && !a.visited && a.nsrc <= kFirstMaxSrc &&
                       nlev >= 1) {
                // roots and level 0 in one kernel (its sums in acc until the end)
                a.acc = reinterpret_cast<unsigned long long *>(w.base + w.L.acc);
                FirstIds ids;
                int32_t nids = 0;
                int gfirst = grid;
                const int32_t *src = a.src;
                if (io->cand_host && src >= io->cand_dev && src + a.nsrc <= io->cand_dev + io->cand_len) {
                    // the host's view of the same ids: their full rows bound
                    // level 0's adjacency entries, hence the workgroups it uses
                    const int32_t *hs = io->cand_host + (src - io->cand_dev);
                    const int32_t *hrp = g->h_rp.data();
                    int64_t ef = 0;
                    for (int64_t j = 0; j < a.nsrc; ++j) {
                        const int32_t v = hs[j];
                        if ((uint32_t)v < (uint32_t)g->n) ef += hrp[v + 1] - hrp[v];
                    }
                    const int64_t gw = (ef + a.min_edges - 1) / a.min_edges;
                    // (and one workgroup per 256 roots after them)
                    gfirst = (int)(std::max<int64_t>(1, std::min<int64_t>(grid, gw)) + (a.nsrc + kWG - 1) / kWG);
                    if (a.nsrc <= kFirstArgIds) {
                        nids = (int32_t)a.nsrc;
                        std::memcpy(ids.id, hs, sizeof(int32_t) * (size_t)nids);
                    }
                }
                HIP_OK(launch_wide_first(a, dist_bytes, gfirst, ids, nids, s));
                HIP_OK(launch_wide_levels(a, dist_bytes, 1, nlev, grid, s));
                HIP_OK(launch_wide_end(a, nlev, grid, s));
            } else {
                HIP_OK(launch_wide_begin(a, dist_bytes, nlev, s));
                HIP_OK(launch_wide_levels(a, dist_bytes, 0, nlev, grid, s));
                HIP_OK(launch_wide_end(a, nlev, grid, s));
            }
            off += a.nsrc;
        }
        int32_t flag = 0;
        if (phase != kGainsWait) {
            if (g_timing) HIP_OK(hipEventRecord(g_ev1, s));
            if (timed) HIP_OK(hipEventRecord(io->ev1, s));
        }
        if (phase == kGainsLaunch) {
            if (queued) *queued = true;
            return GC_OK;
        }
        phase = kGainsRun;  // an overflow below relaunches normally
        if (mapped) {
            // poll the done word (no wake-up latency of a blocking wait); an
            // overflow, a fault or a long launch ends up in the blocking wait
            bool done = false;
            if (io->hm_done) {
                const double t0 = now_ms();
                for (uint32_t spin = 0;; ++spin) {
                    if (*io->h_done == io->seq) {
                        done = true;
                        break;
                    }
                    if (*io->h_flag) break;
                    if ((spin & 255) == 255 && now_ms() - t0 > 2.0) break;
                }
            }
            if (!done) HIP_OK(hipStreamSynchronize(s));
            flag = *io->h_flag;
        } else {
            HIP_OK(hipMemcpyAsync(&flag, w.flags(), sizeof(flag), hipMemcpyDeviceToHost, s));
            // results go out with the same synchronisation (discarded on overflow)
            if (h_gain)
                HIP_OK(hipMemcpyAsync(h_gain, d_gain, sizeof(int64_t) * count, hipMemcpyDeviceToHost, s));
            if (h_edges && d_edges)
                HIP_OK(hipMemcpyAsync(h_edges, d_edges, sizeof(int64_t) * count, hipMemcpyDeviceToHost, s));
            HIP_OK(hipStreamSynchronize(s));
        }
        if (flag == 0) {
            // (after a polled wait the events behind the last kernel may still be pending)
            if (g_timing) {
                HIP_OK(hipEventSynchronize(g_ev1));
                HIP_OK(hipEventElapsedTime(&g_timing_ms, g_ev0, g_ev1));
            }
            if (timed) {
                float ms = 0.f;
                HIP_OK(hipEventSynchronize(io->ev1));
                HIP_OK(hipEventElapsedTime(&ms, io->ev0, io->ev1));
                *io->gpu_ms += ms;
            }
            if (shape) {
                shape->kb = kb;
                shape->spb = spb;
            }
            return GC_OK;
        }
        // chunk `flag` overflowed the frontier log: it and the chunks after it
        // are redone with fewer batches (then fewer sources per batch) per
        // launch, after clearing the visited words and level records.  One
        // source per launch claims each node at most once, so it always fits
        // (cap >= n).
        done += (int64_t)(flag - 1) * per;
        HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.base + w.L.wvis),
                               (size_t)w.L.kmax * w.L.vis_stride * 8, 0u, s));
        HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.base + w.L.lvl),
                               (size_t)(nlev + 2) * sizeof(WideLevel) / 4, 0u, s));
        HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.zcnt()), 2, 0u, s));
        HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.flags()), 1, 0u, s));
        if (w.L.acc)
            HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.base + w.L.acc), (size_t)kFirstMaxSrc * 2, 0u, s));
        if (kb > 1) kb = std::max<int64_t>(1, kb / 2);
        else if (spb > 1) spb = std::max(1, spb / 2);
        else
            return fail(GC_EWORKSPACE, "frontier log of %lld entries too small for one source",
                        (long long)w.L.cap);
    }
    return GC_OK;
}

// d(S,.) <- min(d(S,.), d(root,.)) and F(S) -= g(root, S) with the
// edge-balanced engine (S != {}); asynchronous.  nlev = max d(S,.) - 1.
int run_update_wide(const gc_graph *g, const Ws &w, int32_t root, void *d_dist, int dist_bytes,
                    int64_t *d_far, hipStream_t s, int32_t nlev, const Split *split = nullptr) {
    nlev = std::min(std::max(nlev, 0), kMaxLevels - 1);
    if (int rc = level_cap_check(g, nlev)) return rc;
    WideArgs a = w.wide();
    a.unroll = g->unroll_small;  // one source: a small launch
    a.min_edges = g->min_edges;
    a.rp = g->d_rp;
    a.ci = g->d_ci;
    a.n = g->n;
    a.dist = d_dist;
    a.src = nullptr;
    a.root = root;
    a.nsrc = 1;
    a.spb = 1;
    a.gain = w.far() + 1;
    a.tag = 1;
    a.write = true;
    a.far = d_far;
    a.dist_bytes = dist_bytes;
    apply_split(a, split);
    const int grid = wide_grid(g);
    HIP_OK(launch_wide_begin(a, dist_bytes, nlev, s));
    HIP_OK(launch_wide_levels(a, dist_bytes, 0, nlev, grid, s));
    HIP_OK(launch_wide_end(a, nlev, grid, s));
    return GC_OK;
}

// Full BFS from root into dist16 (uint16, INF = 65535 everywhere first) on the
// edge-balanced engine in write-back mode: every node's distance is written,
// *d_far = n*65535 - sum(65535 - d) = sum_w d(root,w) = F({root}), and
// *ecc_out = max distance (65535 if some node is farther: GC_ERANGE).
// Synchronises (the depth is not known in advance).
int run_full_bfs(const gc_graph *g, const Ws &w, int32_t root, uint16_t *dist16, int64_t *d_far,
                 hipStream_t s, int32_t *ecc_out) {
    const int32_t n = g->n;
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(dist16), ((size_t)n * 2 + 3) / 4, 0xFFFFFFFFu, s));
    HIP_OK(launch_set_i64(d_far, (int64_t)n * 65535, s));
    WideArgs a = w.wide();
    a.unroll = g->unroll;
    a.min_edges = g->min_edges;
    a.rp = g->d_rp;
    a.ci = g->d_ci;
    a.n = n;
    a.dist = dist16;
    a.src = nullptr;
    a.root = root;
    a.nsrc = 1;
    a.spb = 1;
    a.gain = w.far() + 1;
    a.tag = 1;
    a.write = true;
    a.far = d_far;
    a.dist_bytes = 2;
    const int grid = wide_grid(g);
    HIP_OK(launch_wide_begin(a, 2, 0, s));
    int32_t L = 0;
    for (;;) {
        const int32_t step = L < 16 ? 4 : 16;
        const int32_t L1 = std::min(L + step, kMaxLevels - 1);
        HIP_OK(launch_wide_levels(a, 2, L, L1, grid, s));
        L = L1;
        WideLevel rec;
        HIP_OK(hipMemcpyAsync(&rec, reinterpret_cast<WideLevel *>(w.base + w.L.lvl) + L, sizeof(rec),
                              hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        if ((rec.packed >> kCntShift) == 0 || L >= kMaxLevels - 1) break;
        if (int rc = level_cap_check(g, L)) return rc;
    }
    HIP_OK(launch_wide_end(a, L, grid, s));
    int32_t maxd = 0;
    HIP_OK(launch_max_dist(dist16, 2, n, w.maxd(), s));
    HIP_OK(hipMemcpyAsync(&maxd, w.maxd(), sizeof(maxd), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    *ecc_out = maxd;
    return GC_OK;
}

// s_1 = argmin (F({v}), v): the top-k closeness search of Section 3.1 with
// k = 1.  A full BFS from the highest-degree node gives a first bound F0.
// Every node's farness is at least its level-1 bound
//   deg(v) + 2*min(rem, two(v) - deg(v)) + 3*(rem - min(...)),  rem = n-1-deg(v),
// (nodes at distance 2 are at most the adjacency of v's neighbours minus one
// back-edge each; two(v) = sum of neighbour degrees), so nodes whose bound
// exceeds the best are dropped on the host.  The rest run 64 to a batch, in
// ball order (balls seeded by decreasing degree; the degree order of the
// paper's search with GC_BALLS=0), as full multi-source BFS on the device-wide engine
// (distances from an all-INF array), each source cut as soon as its BFScut
// bound exceeds the best farness found so far; the bound is re-applied on the
// host between chunks as the best improves.  Ties: smallest id.
// General k (top-k closeness): the cut threshold is the k-th best (F, id)
// found so far, raised on the host between chunks only (a source's own
// farness must not become the device's threshold), and no node is cut before
// k farness values are known.  `top` receives the k best (F, id), ascending.
// Largest graphs the closeness search has been run on (R-MAT scale 20,
// edge factor 16); a larger run of an earlier version of this search ended in
// a GPU memory fault whose cause was not found, so larger graphs are refused.
constexpr int64_t kSearchMaxN = (int64_t)1 << 20;
constexpr int64_t kSearchMaxNnz = (int64_t)1 << 25;

int search_size_ok(const gc_graph *g) {
    if (g->n > kSearchMaxN || g->nnz > kSearchMaxNnz)
        return fail(GC_ERANGE, "closeness search: graphs above %lld nodes or %lld adjacency entries "
                    "are not supported (n = %d, nnz = %lld)", (long long)kSearchMaxN,
                    (long long)kSearchMaxNnz, g->n, (long long)g->nnz);
    return GC_OK;
}

int run_closest(const gc_graph *g, const Ws &w, hipStream_t s, int32_t *node, int64_t *far,
                int64_t *sources, int32_t *ecc_out, int32_t *v0_out = nullptr, int32_t k = 1,
                std::vector<std::pair<int64_t, int32_t>> *top_out = nullptr) {
    if (int rc0 = search_size_ok(g)) return rc0;
    const int32_t n = g->n;
    const auto &rp = g->h_rp;
    const auto &order = g->search_order();
    const int32_t v0 = order[0];
    if (v0_out) *v0_out = v0;
    // full BFS from v0 in 16-bit distances (kept in dist16 for reuse)
    int32_t last = 0;
    int rc = run_full_bfs(g, w, v0, w.dist16(), w.far(), s, &last);
    if (rc) return rc;
    int64_t F0 = 0, stamp = 0;
    HIP_OK(hipMemcpyAsync(&F0, w.far(), sizeof(F0), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(&stamp, w.hdr(), sizeof(stamp), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (last >= 65535) return fail(GC_ERANGE, "a node is 65535 or more hops from node %d", v0);
    // the search order and two-hop sums come from gc_workspace_init; a
    // workspace without its stamp gets them now
    if (stamp != ws_stamp(g)) {
        int rc2 = write_graph_tables(g, w, s);
        if (rc2) return rc2;
    }
    // the k best (F, id) known, ascending; (bestF, best) is the k-th once k
    // are known, else no bound
    std::vector<std::pair<int64_t, int32_t>> top{{F0, v0}};
    int32_t best = INT32_MAX;
    int64_t bestF = INT64_MAX;
    auto set_threshold = [&]() {
        if ((int32_t)top.size() >= k) {
            bestF = top[(size_t)k - 1].first;
            best = top[(size_t)k - 1].second;
        }
    };
    set_threshold();
    // level-1 bound of every node against the threshold, on the device, in search order;
    // the bounds of the survivors come back to re-test them as the best improves
    uint8_t *keep_d = reinterpret_cast<uint8_t *>(w.base + w.L.q0);
    HIP_OK(launch_lb1_filter(w.order(), g->d_rp, w.two(), n, bestF, best, keep_d, w.aux(), g->directed, s));
    std::vector<uint8_t> keep((size_t)n);
    HIP_OK(hipMemcpyAsync(keep.data(), keep_d, (size_t)n, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    std::vector<int32_t> list, lpos;
    for (int32_t i = 1; i < n; ++i)
        if (keep[i]) {
            list.push_back(order[i]);
            lpos.push_back(i);
        }
    std::vector<int64_t> lbound(list.size());
    if (!list.empty()) {
        HIP_OK(hipMemcpyAsync(w.cand(), lpos.data(), sizeof(int32_t) * lpos.size(), hipMemcpyHostToDevice, s));
        HIP_OK(launch_gather_i64(w.aux(), w.cand(), (int32_t)lpos.size(), w.gain(), s));
        HIP_OK(hipMemcpyAsync(lbound.data(), w.gain(), sizeof(int64_t) * lbound.size(), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
    }
    auto may_win_at = [&](size_t j) {
        return lbound[j] < bestF || (lbound[j] == bestF && list[j] < best);
    };
    int64_t nsources = 1;
    const bool verbose = getenv("GC_VERBOSE") != nullptr;
    double t_print = now_ms();
    if (verbose) {
        fprintf(stderr, "[gc] closeness: F({%d}) = %lld, %zu of %d nodes pass the level-1 bound\n", v0,
                (long long)F0, list.size(), n - 1);
        fflush(stderr);
    }
    // INF distances for the full BFS: the second level-BFS queue is free here
    uint16_t *inf16 = reinterpret_cast<uint16_t *>(w.base + w.L.q1);
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(inf16), ((size_t)n * 2 + 3) / 4, 0xFFFFFFFFu, s));
    int64_t *dbest = reinterpret_cast<int64_t *>(w.ctr() + C_I64_BASE) + L_BEST_FAR;
    // a batch touches each record once (the clean-up list bounds the batches
    // of a launch); the log holds three levels at a time, and an overflow of
    // either halves the launch.
    // Chunks start at one batch and double up to kb_cap: the first sources
    // set a best that the bounds cut the later, larger chunks against.
    int64_t kb_cap = std::max<int64_t>(1, std::min<int64_t>(w.L.kmax, w.L.zcap / ((int64_t)n + 64)));
    int64_t kb = 1;
    int32_t spb = 64;
    std::vector<int64_t> fo;
    std::vector<int32_t> chunk;
    size_t pos = 0;
    const int grid = wide_grid(g);
    while (pos < list.size()) {
        chunk.clear();
        const size_t pos0 = pos;
        while (pos < list.size() && (int64_t)chunk.size() < kb * spb) {
            const size_t j = pos++;
            if (may_win_at(j)) chunk.push_back(list[j]);
        }
        if (chunk.empty()) break;
        const int64_t cnt = (int64_t)chunk.size();
        HIP_OK(hipMemcpyAsync(w.cand(), chunk.data(), sizeof(int32_t) * cnt, hipMemcpyHostToDevice, s));
        HIP_OK(launch_set_i64(dbest, bestF, s));
        WideArgs a = w.wide();
        a.unroll = g->unroll;
        a.min_edges = g->min_edges;
        a.rp = g->d_rp;
        a.ci = g->d_ci;
        a.n = n;
        a.dist = inf16;
        a.src = w.cand();
        a.nsrc = cnt;
        a.spb = spb;
        a.gain = w.gain();
        a.edges = w.aux();
        a.visited = w.aux2();
        a.tag = 1;
        a.dist_bytes = 2;
        a.active = reinterpret_cast<unsigned long long *>(w.base + w.L.act);
        a.prev = reinterpret_cast<int64_t *>(w.base + w.L.cutprev);
        a.far_out = reinterpret_cast<int64_t *>(w.base + w.L.farout);
        a.directed = g->directed ? 1 : 0;
        HIP_OK(launch_wide_begin(a, 2, 0, s));
        int32_t L = 0;
        bool overflow = false;
        // levels between host checks: 4, then doubling up to 32 (a deep
        // search waits less often; levels past the end find nothing to do)
        int32_t step = 4;
        for (;; step = std::min(step * 2, 32)) {
            for (int32_t i = 0; i < step && L + i < kMaxLevels - 1; ++i) {
                HIP_OK(launch_wide_levels(a, 2, L + i, L + i + 1, grid, s));
                HIP_OK(launch_wide_cut(a, L + i, dbest, k > 1, s));
            }
            L = std::min(L + step, kMaxLevels - 1);
            WideLevel rec;
            int32_t flag = 0;
            HIP_OK(hipMemcpyAsync(&rec, reinterpret_cast<WideLevel *>(w.base + w.L.lvl) + L,
                                  sizeof(rec), hipMemcpyDeviceToHost, s));
            HIP_OK(hipMemcpyAsync(&flag, w.flags(), sizeof(flag), hipMemcpyDeviceToHost, s));
            HIP_OK(hipStreamSynchronize(s));
            if (flag) {
                overflow = true;
                break;
            }
            if ((rec.packed >> kCntShift) == 0 || L >= kMaxLevels - 1) break;
            if (int rc = level_cap_check(g, L)) return rc;
        }
        if (overflow) {
            // too many frontier entries: clear and redo this chunk with fewer sources
            HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.base + w.L.wvis),
                                   (size_t)w.L.kmax * w.L.vis_stride * 8, 0u, s));
            HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.base + w.L.lvl),
                                   (size_t)(kMaxLevels + 2) * sizeof(WideLevel) / 4, 0u, s));
            HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.zcnt()), 2, 0u, s));
            HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.flags()), 1, 0u, s));
            if (kb > 1) kb_cap = kb = kb / 2;
            else if (spb > 1) spb = std::max(1, spb / 2);
            else return fail(GC_EWORKSPACE, "frontier log too small for one source");
            pos = pos0;  // the filtered-out nodes before the chunk's end are checked again
            continue;
        }
        HIP_OK(launch_wide_end(a, L, grid, s));
        fo.resize((size_t)cnt);
        HIP_OK(hipMemcpyAsync(fo.data(), a.far_out, sizeof(int64_t) * cnt, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        nsources += cnt;
        kb = std::min(kb * 2, kb_cap);
        for (int64_t i = 0; i < cnt; ++i) {
            if (fo[i] < 0) continue;
            if (fo[i] < bestF || (fo[i] == bestF && chunk[i] < best)) {
                const std::pair<int64_t, int32_t> e{fo[i], chunk[i]};
                top.insert(std::upper_bound(top.begin(), top.end(), e), e);
                if ((int32_t)top.size() > k) top.pop_back();
                set_threshold();
            }
        }
        if (verbose && now_ms() - t_print > 2000.0) {
            t_print = now_ms();
            fprintf(stderr, "[gc] closeness: %zu of %zu listed, %lld sources run, best %d (F %lld), "
                    "%lld batches x %d per launch\n", pos, list.size(), (long long)nsources, best,
                    (long long)bestF, (long long)kb, spb);
            fflush(stderr);
        }
    }
    if ((int32_t)top.size() < k) return fail(GC_EDEVICE, "closeness search ended with %zu of %d nodes",
                                             top.size(), k);
    *node = top[0].second;
    *far = top[0].first;
    if (top_out) *top_out = top;
    if (sources) *sources = nsources;
    if (ecc_out) *ecc_out = last;
    return GC_OK;
}

}  // namespace

extern "C" int gc_closest_node(const gc_graph *g, void *d_ws, size_t ws_bytes, hipStream_t stream,
                               int32_t *h_node, int64_t *h_farness) {
    if (!g) return fail(GC_EINVAL, "graph is NULL");
    if (g->weighted) {
        WWs ww;
        int rc = get_wws(g, d_ws, ws_bytes, &ww);
        if (rc) return rc;
        if (!h_node || !h_farness) return fail(GC_EINVAL, "NULL output");
        std::vector<std::pair<int64_t, int32_t>> top;
        rc = run_wclosest(g, ww, stream, 1, &top);
        if (rc) return rc;
        *h_node = top[0].second;
        *h_farness = top[0].first;
        return GC_OK;
    }
    if (int rc0 = search_size_ok(g)) return rc0;
    Ws w;
    int rc = get_ws(g, d_ws, ws_bytes, &w);
    if (rc) return rc;
    if (!h_node || !h_farness) return fail(GC_EINVAL, "NULL output");
    int32_t node;
    int64_t far;
    rc = run_closest(g, w, stream, &node, &far, nullptr, nullptr);
    if (rc) return rc;
    *h_node = node;
    *h_farness = far;
    return GC_OK;
}

extern "C" int gc_topk_closeness(const gc_graph *g, int32_t k, void *d_ws, size_t ws_bytes,
                                 hipStream_t stream, int32_t *h_nodes, int64_t *h_farness) {
    if (!g) return fail(GC_EINVAL, "graph is NULL");
    if (g->weighted) {
        WWs ww;
        int rc = get_wws(g, d_ws, ws_bytes, &ww);
        if (rc) return rc;
        if (!h_nodes || !h_farness) return fail(GC_EINVAL, "NULL output");
        if (k < 1 || k > g->n) return fail(GC_EINVAL, "k = %d out of range 1..%d", k, g->n);
        std::vector<std::pair<int64_t, int32_t>> top;
        rc = run_wclosest(g, ww, stream, k, &top);
        if (rc) return rc;
        for (int32_t i = 0; i < k; ++i) {
            h_nodes[i] = top[(size_t)i].second;
            h_farness[i] = top[(size_t)i].first;
        }
        return GC_OK;
    }
    if (int rc0 = search_size_ok(g)) return rc0;
    Ws w;
    int rc = get_ws(g, d_ws, ws_bytes, &w);
    if (rc) return rc;
    if (!h_nodes || !h_farness) return fail(GC_EINVAL, "NULL output");
    if (k < 1 || k > g->n) return fail(GC_EINVAL, "k = %d out of range 1..%d", k, g->n);
    int32_t node;
    int64_t far;
    std::vector<std::pair<int64_t, int32_t>> top;
    rc = run_closest(g, w, stream, &node, &far, nullptr, nullptr, nullptr, k, &top);
    if (rc) return rc;
    for (int32_t i = 0; i < k; ++i) {
        h_nodes[i] = top[(size_t)i].second;
        h_farness[i] = top[(size_t)i].first;
    }
    return GC_OK;
}

// ------------------------------------------------------------ bit vectors

namespace {
// bits buffer: `levels` stored levels of n rows of W words, then kBitsMaxS
// rows of b^i_S, then a counter block (change flag, max distance)
int64_t bits_words(const gc_graph *g) { return ((int64_t)g->n + 63) / 64; }
size_t bits_level_bytes(const gc_graph *g) { return (size_t)g->n * (size_t)bits_words(g) * 8; }
size_t bits_bytes(const gc_graph *g, int32_t levels) {
    return (size_t)levels * bits_level_bytes(g) + (size_t)kBitsMaxS * (size_t)bits_words(g) * 8 + 256;
}
}  // namespace

extern "C" int gc_bits_size(const gc_graph *g, int32_t levels, size_t *bytes) {
    if (!g || !bytes) return fail(GC_EINVAL, "NULL argument");
    if (levels < 2 || levels > kBitsMaxS) return fail(GC_EINVAL, "levels must be 2..%d", kBitsMaxS);
    *bytes = bits_bytes(g, levels);
    return GC_OK;
}

extern "C" int gc_bits_prepare(const gc_graph *g, void *d_bits, size_t bytes, hipStream_t s,
                               int32_t *h_levels) {
    if (!g || !d_bits || !h_levels) return fail(GC_EINVAL, "NULL argument");
    if (int rc0 = unweighted_only(g, "gc_bits_prepare")) return rc0;
    const size_t lb = bits_level_bytes(g);
    const size_t fixed = (size_t)kBitsMaxS * (size_t)bits_words(g) * 8 + 256;
    if (bytes < fixed + 2 * lb) return fail(GC_EWORKSPACE, "bits buffer too small for two levels");
    const int32_t cap = (int32_t)std::min<size_t>((bytes - fixed) / lb, (size_t)kBitsMaxS);
    char *base = reinterpret_cast<char *>(d_bits);
    auto level = [&](int32_t l) { return reinterpret_cast<uint64_t *>(base + (size_t)l * lb); };
    int32_t *flag = reinterpret_cast<int32_t *>(base + (size_t)cap * lb + (size_t)kBitsMaxS * bits_words(g) * 8);
    HIP_OK(launch_bits_identity(level(0), g->n, s));
    for (int32_t i = 1; i < cap; ++i) {
        HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(flag), 1, 0u, s));
        HIP_OK(launch_bits_level(g->d_rp, g->d_ci, g->n, level(i - 1), level(i), flag, s));
        int32_t changed = 0;
        HIP_OK(hipMemcpyAsync(&changed, flag, sizeof(changed), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        if (!changed) {
            *h_levels = i;  // levels 0 .. i-1; level i-1 is the fixed point
            return GC_OK;
        }
    }
    return fail(GC_EWORKSPACE, "bit vectors need more than %d levels", cap);
}

namespace {
// gains by the theorem's sum over the stored levels; b^i_S rebuilt from
// d(S,.) for i below max d(S,.) (every later term is zero)
int run_bits_gains(const gc_graph *g, const void *d_bits, size_t bytes, int32_t levels, const void *d_dist,
                   int dist_bytes, const int32_t *d_cand, int64_t count, int64_t *d_gain, hipStream_t s,
                   int32_t maxd = -1, bool count_words = false, bool build_bs = true) {
    const size_t lb = bits_level_bytes(g);
    const size_t fixed = (size_t)kBitsMaxS * (size_t)bits_words(g) * 8 + 256;
    if (bytes < fixed + (size_t)levels * lb) return fail(GC_EWORKSPACE, "bits buffer smaller than its levels");
    const int32_t cap = (int32_t)std::min<size_t>((bytes - fixed) / lb, (size_t)kBitsMaxS);
    const char *base = reinterpret_cast<const char *>(d_bits);
    uint64_t *bs = reinterpret_cast<uint64_t *>(const_cast<char *>(base) + (size_t)cap * lb);
    int32_t *ctr = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(bs) + (size_t)kBitsMaxS * bits_words(g) * 8);
    if (maxd < 0) {
        HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(ctr + 1), 1, 0u, s));
        HIP_OK(launch_max_dist(d_dist, dist_bytes, g->n, ctr + 1, s));
        HIP_OK(hipMemcpyAsync(&maxd, ctr + 1, sizeof(maxd), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
    }
    const int32_t levels_s = std::min(maxd, kBitsMaxS);
    if (build_bs) HIP_OK(launch_bits_group(d_dist, dist_bytes, g->n, levels_s, bs, s));
    // (the row words read go to the counter block's second int64)
    unsigned long long *words = count_words ? reinterpret_cast<unsigned long long *>(ctr) + 1 : nullptr;
    HIP_OK(launch_bits_gains(reinterpret_cast<const uint64_t *>(base), g->n, levels, bs, levels_s, d_cand, count,
                             d_gain, words, s));
    return GC_OK;
}

// the counter of row words read by the bit-vector gains of a greedy job
unsigned long long *bits_words_counter(const gc_graph *g, const void *d_bits, size_t bytes) {
    const size_t lb = bits_level_bytes(g);
    const size_t fixed = (size_t)kBitsMaxS * (size_t)bits_words(g) * 8 + 256;
    const int32_t cap = (int32_t)std::min<size_t>((bytes - fixed) / lb, (size_t)kBitsMaxS);
    char *base = reinterpret_cast<char *>(const_cast<void *>(d_bits));
    return reinterpret_cast<unsigned long long *>(base + (size_t)cap * lb + (size_t)kBitsMaxS * bits_words(g) * 8) + 1;
}
}  // namespace

extern "C" int gc_bits_gains(const gc_graph *g, const void *d_bits, size_t bytes, int32_t levels,
                             const void *d_dist, int32_t dist_bytes, const int32_t *d_cand, int64_t count,
                             int64_t *d_gain, hipStream_t stream) {
    if (int rc0 = unweighted_only(g, "gc_bits_gains")) return rc0;
    if (!g || !d_bits || !d_dist || (count > 0 && (!d_cand || !d_gain))) return fail(GC_EINVAL, "NULL argument");
    if (dist_bytes != 1) return fail(GC_EINVAL, "the bit-vector gains take uint8 distances");
    if (levels < 1 || levels > kBitsMaxS) return fail(GC_EINVAL, "levels out of range");
    if (count < 0) return fail(GC_EINVAL, "negative count");
    if (count == 0) return GC_OK;
    return run_bits_gains(g, d_bits, bytes, levels, d_dist, dist_bytes, d_cand, count, d_gain, stream);
}

extern "C" int gc_update_dist(const gc_graph *g, int32_t node, void *d_dist, int32_t dist_bytes,
                              void *d_ws, size_t ws_bytes, hipStream_t stream, int64_t *d_farness) {
    if (g && g->weighted) {
        WWs ww;
        int rc = get_wws(g, d_ws, ws_bytes, &ww);
        if (rc) return rc;
        if (node < 0 || node >= g->n) return fail(GC_EINVAL, "node %d out of range", node);
        if (dist_bytes != 4) return fail(GC_EINVAL, "weighted graphs: dist_bytes must be 4");
        if (!d_dist || !d_farness) return fail(GC_EINVAL, "NULL device pointer");
        int32_t dn = 0;
        HIP_OK(hipMemcpyAsync(&dn, reinterpret_cast<int32_t *>(d_dist) + node, sizeof(dn), hipMemcpyDeviceToHost,
                              stream));
        HIP_OK(hipStreamSynchronize(stream));
        // on a connected graph d(S, node) is finite unless S = {}
        return run_wupdate(g, ww, node, reinterpret_cast<int32_t *>(d_dist), d_farness, dn == INT32_MAX, stream);
    }
    Ws w;
    int rc = get_ws(g, d_ws, ws_bytes, &w);
    if (rc) return rc;
    if (node < 0 || node >= g->n) return fail(GC_EINVAL, "node %d out of range", node);
    if (dist_bytes != 1 && dist_bytes != 2) return fail(GC_EINVAL, "dist_bytes must be 1 or 2");
    if (!d_dist || !d_farness) return fail(GC_EINVAL, "NULL device pointer");
    return run_update(g, w, node, d_dist, dist_bytes, d_farness, stream, nullptr, nullptr);
}

extern "C" int gc_marginal_gains(const gc_graph *g, const void *d_dist, int32_t dist_bytes,
                                 const int32_t *d_cand, int32_t count, int64_t *d_gain,
                                 int64_t *d_edges, int32_t *d_visited, void *d_ws, size_t ws_bytes,
                                 hipStream_t stream) {
    if (g && g->weighted) {
        WWs ww;
        int rc = get_wws(g, d_ws, ws_bytes, &ww);
        if (rc) return rc;
        if (dist_bytes != 4) return fail(GC_EINVAL, "weighted graphs: dist_bytes must be 4");
        if (count < 0) return fail(GC_EINVAL, "count < 0");
        if (count > 0 && (!d_dist || !d_cand || !d_gain)) return fail(GC_EINVAL, "NULL device pointer");
        if (count == 0) return GC_OK;
        if (g_timing) HIP_OK(hipEventRecord(g_ev0, stream));
        // W_GAIN only reads d(S,.)
        rc = wlaunch(g, ww, W_GAIN, const_cast<int32_t *>(reinterpret_cast<const int32_t *>(d_dist)), d_cand, count,
                     d_gain, d_edges, d_visited, 0, nullptr, false, stream);
        if (rc) return rc;
        if (g_timing) {
            HIP_OK(hipEventRecord(g_ev1, stream));
            HIP_OK(hipEventSynchronize(g_ev1));
            HIP_OK(hipEventElapsedTime(&g_timing_ms, g_ev0, g_ev1));
        }
        return GC_OK;
    }
    Ws w;
    int rc = get_ws(g, d_ws, ws_bytes, &w);
    if (rc) return rc;
    if (dist_bytes != 1 && dist_bytes != 2) return fail(GC_EINVAL, "dist_bytes must be 1 or 2");
    if (count < 0) return fail(GC_EINVAL, "count < 0");
    if (count > 0 && (!d_dist || !d_cand || !d_gain)) return fail(GC_EINVAL, "NULL device pointer");
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.words()), 2 * kWordCounters, 0u, stream));
    if (count == 0) return GC_OK;
    // the row split is built from these distances for this call (its time
    // counts in the timed span)
    if (g_timing) HIP_OK(hipEventRecord(g_ev0, stream));
    Split sp;
    int rc2 = build_split(g, w, d_dist, dist_bytes, stream, &sp);
    if (rc2) return rc2;
    return run_gains(g, w, d_dist, dist_bytes, d_cand, count, d_gain, d_edges, d_visited, stream, -1,
                     nullptr, nullptr, nullptr, nullptr, &sp, true);
}

namespace {

// Layout of the marginal-gain path alone in a buffer of `bytes` bytes: the
// counter block, the level records, the row split, the frontier ring, the
// clean-up list and as many per-batch record blocks as fit, at most `kwant`
// (none of the closeness-search, level-BFS, graph-table or learned-order
// regions).  The ring and the clean-up list hold one source's BFS (n + 128
// entries, rounded up to a power of two); an overflow of a launch with more
// batches is redone with fewer.  False if not even one batch fits.
bool gains_layout(const gc_graph *g, size_t bytes, int64_t kwant, WsLayout *out) {
    WsLayout L{};
    const size_t n = (size_t)g->n;
    size_t o = 0;
    L.ctr = o; o += kCtrBytes;
    L.lvl = o; o += al256((size_t)(kMaxLevels + 2) * sizeof(WideLevel));
    L.cisplit = o; o += al256((size_t)g->nnz * 4 + 4);
    L.rinfo = o; o += al256(n * 16);
    L.dist1 = o; o += al256(n * 2 + 4);
    int64_t ring = 1;
    while (ring < (int64_t)n + 128) ring <<= 1;
    L.cap = ring;
    L.zcap = ring;
    L.ly = o; o += al256((size_t)ring * 4);
    L.lr = o; o += al256((size_t)ring * 4);
    L.lb = o; o += al256((size_t)ring * 4);
    L.lo = o; o += al256((size_t)ring * 8);
    L.lz = o; o += al256((size_t)ring * 8);
    L.vis_stride = (n + 31) & ~(size_t)31;
    const size_t per = L.vis_stride * 32;
    if (o > bytes || bytes - o < per) return false;
    int64_t kmax = (int64_t)((bytes - o) / per);
    kmax = std::max<int64_t>(1, std::min<int64_t>(kmax, std::max<int64_t>(kwant, 1)));
    L.kmax = kmax;
    L.wvis = o; o += (size_t)kmax * per;
    L.total = o;
    *out = L;
    return true;
}

}  // namespace

namespace gck {

int set_error(int code, const char *msg) { return fail(code, "%s", msg); }

size_t gains_buffer_min_bytes(const gc_graph *g) {
    // the layout with exactly one batch
    WsLayout L;
    gains_layout(g, (size_t)1 << 62, 1, &L);
    return L.total;
}

int gains_in_buffer(const gc_graph *g, const void *d_dist, int32_t dist_bytes, const int32_t *d_cand,
                    int32_t count, int64_t *d_gain, int64_t *d_edges, int32_t *d_visited, void *d_buf,
                    size_t buf_bytes, hipStream_t stream) {
    if (int rc0 = unweighted_only(g, "gc_marginal_gains_noalloc")) return rc0;
    if (!g) return fail(GC_EINVAL, "graph is NULL");
    if (dist_bytes != 1 && dist_bytes != 2) return fail(GC_EINVAL, "dist_bytes must be 1 or 2");
    if (count < 0) return fail(GC_EINVAL, "count < 0");
    if (count > 0 && (!d_dist || !d_cand || !d_gain)) return fail(GC_EINVAL, "NULL device pointer");
    Ws w;
    const int64_t kwant = ((int64_t)count + kSrc - 1) / kSrc;
    if (!gains_layout(g, buf_bytes, kwant, &w.L))
        return fail(GC_EWORKSPACE, "graph needs %zu bytes of scratch for one batch, %zu available",
                    gains_buffer_min_bytes(g), buf_bytes);
    w.base = reinterpret_cast<char *>(d_buf);
    w.bytes = buf_bytes;
    // the buffer holds whatever the last call left: zero the counters, the
    // level records and the batch records this call reads before writing
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.base + w.L.ctr), kCtrBytes / 4, 0u, stream));
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.base + w.L.lvl),
                           (size_t)(kMaxLevels + 2) * sizeof(WideLevel) / 4, 0u, stream));
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.base + w.L.wvis),
                           (size_t)w.L.kmax * w.L.vis_stride * 8, 0u, stream));
    if (count == 0) return GC_OK;
    if (g_timing) HIP_OK(hipEventRecord(g_ev0, stream));
    Split sp;
    int rc = build_split(g, w, d_dist, dist_bytes, stream, &sp);
    if (rc) return rc;
    return run_gains(g, w, d_dist, dist_bytes, d_cand, count, d_gain, d_edges, d_visited, stream, -1,
                     nullptr, nullptr, nullptr, nullptr, &sp, true);
}

}  // namespace gck

extern "C" int gc_gain_words(const gc_graph *g, const void *d_ws, size_t ws_bytes, hipStream_t stream,
                             int64_t *h_words) {
    if (int rc0 = unweighted_only(g, "gc_gain_words")) return rc0;
    Ws w;
    int rc = get_ws(g, const_cast<void *>(d_ws), ws_bytes, &w);
    if (rc) return rc;
    if (!h_words) return fail(GC_EINVAL, "NULL output");
    HIP_OK(hipMemcpyAsync(h_words, w.words(), sizeof(int64_t) * kWordCounters, hipMemcpyDeviceToHost,
                          stream));
    HIP_OK(hipStreamSynchronize(stream));
    return GC_OK;
}

// ------------------------------------------------------------- the greedy

namespace {

// Max tree over node ids holding the stale gains (ub; -1 for members of S).
// The plain scan's next candidate that can still beat the best is the leftmost
// id >= pos whose ub reaches the best gain, found in O(log n) instead of a walk
// over every remaining id.
struct MaxTree {
    int32_t leaves = 1;
    std::vector<int64_t> t;
    void build(const std::vector<int64_t> &ub, const std::vector<uint8_t> &inS) {
        const int32_t n = (int32_t)ub.size();
        leaves = 1;
        while (leaves < n) leaves <<= 1;
        t.assign((size_t)2 * leaves, -1);
        for (int32_t i = 0; i < n; ++i) t[(size_t)leaves + i] = inS[i] ? -1 : ub[i];
        for (int32_t i = leaves - 1; i >= 1; --i) t[i] = std::max(t[2 * i], t[2 * i + 1]);
    }
    void set(int32_t i, int64_t x) {
        size_t j = (size_t)leaves + i;
        t[j] = x;
        for (j >>= 1; j >= 1; j >>= 1) t[j] = std::max(t[2 * j], t[2 * j + 1]);
    }
    // leftmost id >= lo with value >= x, or -1
    int32_t first_at_least(int32_t lo, int64_t x) const { return first(1, 0, leaves, lo, x); }
    // the leftmost ids >= lo with value >= x, at most `want` of them, in one
    // walk of the tree (subtrees left of lo or below x are skipped)
    void collect(int32_t lo, int64_t x, int64_t want, std::vector<int32_t> &out) const {
        if (want > 0) collect_at(1, 0, leaves, lo, x, want, out);
    }
    void collect_at(size_t node, int32_t nl, int32_t nr, int32_t lo, int64_t x, int64_t want,
                    std::vector<int32_t> &out) const {
        if (nr <= lo || t[node] < x || (int64_t)out.size() >= want) return;
        if (nr - nl == 1) {
            out.push_back(nl);
            return;
        }
        const int32_t mid = nl + (nr - nl) / 2;
        collect_at(2 * node, nl, mid, lo, x, want, out);
        collect_at(2 * node + 1, mid, nr, lo, x, want, out);
    }
    int32_t first(size_t node, int32_t nl, int32_t nr, int32_t lo, int64_t x) const {
        if (nr <= lo || t[node] < x) return -1;
        if (nr - nl == 1) return nl;
        const int32_t mid = nl + (nr - nl) / 2;
        const int32_t r = first(2 * node, nl, mid, lo, x);
        return r >= 0 ? r : first(2 * node + 1, mid, nr, lo, x);
    }
};

// Tournament tree over candidate keys (value, -id): every node holds the
// leaf that wins its subtree and that leaf's value, so the best candidate is
// read at the root and a key changes in O(log n).  A value below zero means
// "not a candidate".
struct ArgTree {
    int32_t leaves = 1;
    std::vector<int32_t> t;   // winning leaf of each node (padding leaves hold their own index)
    std::vector<int64_t> tv;  // its value
    void pull(size_t j) {
        const int64_t va = tv[2 * j], vb = tv[2 * j + 1];
        const int32_t ia = t[2 * j], ib = t[2 * j + 1];
        const bool left = (va > vb) | ((va == vb) & (ia < ib));  // no branch on random keys
        t[j] = left ? ia : ib;
        tv[j] = left ? va : vb;
    }
    void build(const std::vector<int64_t> &ub, const std::vector<uint8_t> &inS, int32_t skip) {
        const int32_t n = (int32_t)ub.size();
        leaves = 1;
        while (leaves < n) leaves <<= 1;
        t.resize((size_t)2 * leaves);
        tv.resize((size_t)2 * leaves);
        for (int32_t i = 0; i < leaves; ++i) {
            t[(size_t)leaves + i] = i;
            tv[(size_t)leaves + i] = (i >= n || inS[i] || i == skip) ? -1 : ub[i];
        }
        for (size_t j = (size_t)leaves - 1; j >= 1; --j) pull(j);
    }
    // the best candidate, or -1 when none is left
    int32_t top() const { return tv[1] >= 0 ? t[1] : -1; }
    void set(int32_t i, int64_t x) {
        size_t j = (size_t)leaves + i;
        tv[j] = x;
        for (j >>= 1; j >= 1; j >>= 1) pull(j);
    }
};

// Failure injection for the error paths of the greedy's host allocations:
// GC_TEST_FAIL_ALLOC=<n> makes the n-th pinned allocation of each greedy call
// fail (1 = the first), as an exhausted pinned pool would.
int fail_alloc_at() {
    const char *e = getenv("GC_TEST_FAIL_ALLOC");
    return e ? atoi(e) : 0;
}

struct PinnedBuf {
    void *p = nullptr;
    size_t bytes = 0;
    int *counter = nullptr;  // allocations made by this call (failure injection)
    ~PinnedBuf() {
        if (p) (void)hipHostFree(p);
    }
    hipError_t ensure(size_t b) {
        if (b <= bytes) return hipSuccess;
        if (counter) {
            const int at = fail_alloc_at();
            if (at > 0 && ++*counter == at) return hipErrorOutOfMemory;
        }
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipHostMalloc(&p, b, hipHostMallocDefault);
        if (e == hipSuccess) bytes = b;
        return e;
    }
};

// Greedy++ on a weighted graph: the first pick by the closeness search, the
// first gain round over every other node in one launch, then the lazy loop
// of Section 4.2 (stale gains bound the new ones by supermodularity) in
// ascending-id or CELF order, batches growing as in the unweighted loop.
int greedy_weighted(const gc_graph *g, int32_t k, const gc_opts &o, void *d_ws, size_t ws_bytes, hipStream_t s,
                    int32_t *h_group, int64_t *h_farness, gc_stats *h_stats) {
    const double t_start = now_ms();
    WWs w;
    int rc = get_wws(g, d_ws, ws_bytes, &w);
    if (rc) return rc;
    const int32_t n = g->n;
    if (k < 1 || k > n) return fail(GC_EINVAL, "k = %d outside [1, n = %d]", k, n);
    if (!h_group || !h_farness) return fail(GC_EINVAL, "NULL output");
    if (o.order != GC_ORDER_PLAIN && o.order != GC_ORDER_CELF)
        return fail(GC_EINVAL, "weighted graphs: plain or CELF order");
    if (o.d_bits || o.early_exit || o.log_capacity > 0)
        return fail(GC_EINVAL, "weighted graphs: no bit-vector gains, early exit or evaluation log");
    if (o.bitset_width != 0 && o.bitset_width != 64) return fail(GC_EINVAL, "bitset_width must be 64");
    if (o.block < 0) return fail(GC_EINVAL, "block < 0");
    if (o.block_growth < 0 || o.block_growth > 8) return fail(GC_EINVAL, "block_growth outside [0, 8]");
    if (o.nprefix < 0 || o.nprefix > k || (o.nprefix > 0 && !o.h_prefix)) return fail(GC_EINVAL, "bad prefix");
    for (int32_t i = 0; i < o.nprefix; ++i)
        if (o.h_prefix[i] < 0 || o.h_prefix[i] >= n) return fail(GC_EINVAL, "prefix id out of range");
    if (o.nprefix > 1) {
        std::vector<int32_t> ids(o.h_prefix, o.h_prefix + o.nprefix);
        std::sort(ids.begin(), ids.end());
        if (std::adjacent_find(ids.begin(), ids.end()) != ids.end())
            return fail(GC_EINVAL, "prefix repeats a node id");
    }
    const int32_t block = o.block > 0 ? o.block : kSrc;
    const int32_t growth = o.block_growth > 0 ? o.block_growth : 2;
    const int64_t maxb = std::min<int64_t>(16LL * block, n);
    gc_stats st{};
    if (h_stats) st.h_evals_per_round = h_stats->h_evals_per_round;
    if (st.h_evals_per_round)
        for (int32_t i = 0; i < k; ++i) st.h_evals_per_round[i] = 0;
    st.dist_bytes = 4;
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.flags()), 1, 0u, s));
    int alloc_count = 0;
    PinnedBuf pin_cand, pin_out;
    pin_cand.counter = pin_out.counter = &alloc_count;
    if (pin_cand.ensure(sizeof(int32_t) * (size_t)n * 2) != hipSuccess ||
        pin_out.ensure(sizeof(int64_t) * (size_t)n * 2 + 64) != hipSuccess)
        return fail(GC_ENOMEM, "pinned host buffers");
    int32_t *hc = reinterpret_cast<int32_t *>(pin_cand.p);
    int32_t *hv = hc + n;
    int64_t *hg = reinterpret_cast<int64_t *>(pin_out.p);
    int64_t *he = hg + n;
    int64_t *hsmall = he + n;  // gain and F of an update, then the flags word
    int32_t *hflag = reinterpret_cast<int32_t *>(hsmall + 2);
    auto watchdog = [&]() -> int {
        return (*hflag & 2) ? fail(GC_EDEVICE, "a search passed the round cap (GC_ROUND_CAP = %u)", g->wround_cap)
                            : GC_OK;
    };

    // ---- s_1 and d(S,.) of S = {s_1}
    double t0 = now_ms();
    int32_t s1;
    if (o.nprefix > 0) {
        s1 = o.h_prefix[0];
    } else {
        std::vector<std::pair<int64_t, int32_t>> top;
        rc = run_wclosest(g, w, s, 1, &top, &st.closest_sources);
        if (rc) return rc;
        s1 = top[0].second;
    }
    st.ms_closest = now_ms() - t0;
    t0 = now_ms();
    int32_t *dS = w.dist();
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(dS), (size_t)n, 0x7FFFFFFFu, s));
    rc = run_wupdate(g, w, s1, dS, w.far(), true, s);
    if (rc) return rc;
    HIP_OK(hipMemcpyAsync(hsmall + 1, w.far(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(hflag, w.flags(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (int r0 = watchdog()) return r0;
    int64_t F = hsmall[1];
    std::vector<int32_t> group;
    std::vector<int64_t> Fs;
    std::vector<uint8_t> inS((size_t)n, 0);
    group.push_back(s1);
    Fs.push_back(F);
    inS[(size_t)s1] = 1;
    for (int32_t i = 1; i < o.nprefix; ++i) {
        const int32_t v = o.h_prefix[i];
        rc = run_wupdate(g, w, v, dS, w.far(), false, s);
        if (rc) return rc;
        HIP_OK(hipMemcpyAsync(hsmall + 1, w.far(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(hflag, w.flags(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        if (int r0 = watchdog()) return r0;
        F = hsmall[1];
        group.push_back(v);
        Fs.push_back(F);
        inS[(size_t)v] = 1;
    }
    st.ms_update += now_ms() - t0;

    auto evaluate = [&](int32_t cnt) -> int {
        HIP_OK(hipMemcpyAsync(w.cand(), hc, sizeof(int32_t) * (size_t)cnt, hipMemcpyHostToDevice, s));
        if (g_timing) HIP_OK(hipEventRecord(g_ev0, s));
        int r = wlaunch(g, w, W_GAIN, dS, w.cand(), cnt, w.out(), w.edges(), w.vis(), 0, nullptr, false, s);
        if (r) return r;
        if (g_timing) HIP_OK(hipEventRecord(g_ev1, s));
        HIP_OK(hipMemcpyAsync(hg, w.out(), sizeof(int64_t) * (size_t)cnt, hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(he, w.edges(), sizeof(int64_t) * (size_t)cnt, hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(hv, w.vis(), sizeof(int32_t) * (size_t)cnt, hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(hflag, w.flags(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        if (int r0 = watchdog()) return r0;
        if (g_timing) {
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, g_ev0, g_ev1));
            st.ms_gain_gpu += ms;
            g_timing_ms = ms;
        }
        for (int32_t j = 0; j < cnt; ++j) {
            st.edges_alg += he[j];
            st.visited += hv[j];
        }
        st.gain_launches += 1;
        return GC_OK;
    };

    std::vector<int64_t> ub((size_t)n, std::numeric_limits<int64_t>::max());
    const bool celf = o.order == GC_ORDER_CELF;
    MaxTree tree;
    ArgTree keys;
    const int32_t first_gain_round = (int32_t)group.size();
    for (int32_t r = first_gain_round; r < k; ++r) {
        const double tr = now_ms();
        int64_t bgain = -1;
        int32_t bid = -1;
        int64_t nev = 0;
        if (r == first_gain_round) {
            // every stale gain is +inf: all candidates in one launch, ascending id
            int32_t cnt = 0;
            for (int32_t v = 0; v < n; ++v)
                if (!inS[(size_t)v]) hc[cnt++] = v;
            rc = evaluate(cnt);
            if (rc) return rc;
            for (int32_t j = 0; j < cnt; ++j) {
                ub[(size_t)hc[j]] = hg[j];
                if (hg[j] > bgain) {
                    bgain = hg[j];
                    bid = hc[j];
                }
            }
            nev = cnt;
            if (celf) keys.build(ub, inS, -1);
            else tree.build(ub, inS);
        } else {
            int64_t cur = std::min<int64_t>(block, maxb);
            int32_t pos = 0;
            for (;;) {
                int32_t cnt = 0;
                if (celf) {
                    // largest (stale gain, -id) first, while it can still win
                    while (cnt < cur) {
                        const int32_t v = keys.top();
                        if (v < 0) break;
                        const int64_t u = ub[(size_t)v];
                        // stop unless (u, -v) beats (bgain, -bid); the best itself,
                        // back in the tree with its exact gain, does not
                        if (bid >= 0 && (u < bgain || (u == bgain && v >= bid))) break;
                        hc[cnt++] = v;
                        keys.set(v, -1);
                    }
                } else {
                    // ascending id: every id left is above bid, so it must beat bgain
                    while (cnt < cur) {
                        const int32_t v = tree.first_at_least(pos, bid < 0 ? 0 : bgain + 1);
                        if (v < 0) break;
                        hc[cnt++] = v;
                        pos = v + 1;
                    }
                }
                if (cnt == 0) break;
                rc = evaluate(cnt);
                if (rc) return rc;
                for (int32_t j = 0; j < cnt; ++j) {
                    const int32_t v = hc[j];
                    if (hg[j] > ub[(size_t)v]) return fail(GC_EDEVICE, "gain of node %d grew (supermodularity)", v);
                    ub[(size_t)v] = hg[j];
                    if (celf) keys.set(v, hg[j]);
                    else tree.set(v, hg[j]);
                    if (hg[j] > bgain || (hg[j] == bgain && v < bid)) {
                        bgain = hg[j];
                        bid = v;
                    }
                }
                nev += cnt;
                // a candidate is evaluated at most once per round
                if (nev > n) return fail(GC_EDEVICE, "round %d evaluated more than n candidates", r);
                cur = std::min<int64_t>(cur * growth, maxb);
            }
        }
        if (bid < 0) return fail(GC_EDEVICE, "no candidate left in round %d", r);
        const double tu = now_ms();
        if (r == first_gain_round) st.ms_round1 += tu - tr;
        else st.ms_later += tu - tr;
        rc = run_wupdate(g, w, bid, dS, w.far(), false, s);
        if (rc) return rc;
        HIP_OK(hipMemcpyAsync(hsmall, w.res(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(hsmall + 1, w.far(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(hflag, w.flags(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        if (int r0 = watchdog()) return r0;
        if (hsmall[0] != bgain || hsmall[1] != F - bgain)
            return fail(GC_EDEVICE, "update of node %d: gain %lld, expected %lld", bid, (long long)hsmall[0],
                        (long long)bgain);
        F -= bgain;
        if (o.debug_checks) {
            unsigned long long sum = 0;
            HIP_OK(launch_wsum(dS, n, w.sum(), s));
            HIP_OK(hipMemcpyAsync(&sum, w.sum(), sizeof(sum), hipMemcpyDeviceToHost, s));
            HIP_OK(hipStreamSynchronize(s));
            if ((int64_t)sum != F) return fail(GC_EDEVICE, "F(S) = %lld but d(S,.) sums to %llu", (long long)F, sum);
        }
        st.ms_update += now_ms() - tu;
        group.push_back(bid);
        Fs.push_back(F);
        inS[(size_t)bid] = 1;
        ub[(size_t)bid] = -1;
        if (celf) keys.set(bid, -1);
        else tree.set(bid, -1);
        st.evals_total += nev;
        if (r == first_gain_round) st.evals_round1 += nev;
        else st.evals_later += nev;
        if (st.h_evals_per_round) st.h_evals_per_round[r] = nev;
    }
    for (int32_t i = 0; i < k; ++i) {
        h_group[i] = group[(size_t)i];
        h_farness[i] = Fs[(size_t)i];
    }
    st.ms_total = now_ms() - t_start;
    if (h_stats) *h_stats = st;
    return GC_OK;
}

}  // namespace

extern "C" int gc_greedy_group(const gc_graph *g, int32_t k, const gc_opts *opts, void *d_ws,
                               size_t ws_bytes, hipStream_t s, int32_t *h_group,
                               int64_t *h_farness, gc_stats *h_stats) {
    const double t_start = now_ms();
    if (!g) return fail(GC_EINVAL, "graph is NULL");
    if (g->weighted) {
        gc_opts o{};
        if (opts) o = *opts;
        return greedy_weighted(g, k, o, d_ws, ws_bytes, s, h_group, h_farness, h_stats);
    }
    // without a prefix the first pick comes from the closeness search
    if (!opts || opts->nprefix == 0)
        if (int rc0 = search_size_ok(g)) return rc0;
    Ws w;
    int rc = get_ws(g, d_ws, ws_bytes, &w);
    if (rc) return rc;
    const int32_t n = g->n;
    if (k < 1 || k > n) return fail(GC_EINVAL, "k = %d outside [1, n = %d]", k, n);
    if (!h_group || !h_farness) return fail(GC_EINVAL, "NULL output");
    gc_opts o{};
    if (opts) o = *opts;
    if (o.bitset_width != 0 && o.bitset_width != 64) return fail(GC_EINVAL, "bitset_width must be 64");
    if (o.order < GC_ORDER_PLAIN || o.order > GC_ORDER_LEARNED) return fail(GC_EINVAL, "bad order");
    if (o.order == GC_ORDER_LEARNED && !o.d_mlp) return fail(GC_EINVAL, "learned order needs d_mlp");
    const bool bits = o.d_bits != nullptr;
    if (bits && o.order == GC_ORDER_LEARNED)
        return fail(GC_EINVAL, "bit-vector gains: plain or CELF order");
    if (bits && (o.bits_levels < 1 || o.bits_levels > kBitsMaxS))
        return fail(GC_EINVAL, "bits_levels out of range (gc_bits_prepare returns it)");
    if (bits && o.bits_bytes < bits_bytes(g, o.bits_levels))
        return fail(GC_EINVAL, "bits_bytes smaller than %d levels need", o.bits_levels);
    if (bits)
        HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(bits_words_counter(g, o.d_bits, o.bits_bytes)), 2, 0u,
                               s));
    const int32_t block = o.block > 0 ? o.block : kSrc;
    if (o.block_growth < 0 || o.block_growth > 8) return fail(GC_EINVAL, "block_growth outside [0, 8]");
    if (o.nprefix < 0 || o.nprefix > k || (o.nprefix > 0 && !o.h_prefix))
        return fail(GC_EINVAL, "bad prefix");
    for (int32_t i = 0; i < o.nprefix; ++i)
        if (o.h_prefix[i] < 0 || o.h_prefix[i] >= n) return fail(GC_EINVAL, "prefix id out of range");
    if (o.nprefix > 1) {
        // a group holds each node once: a repeated id is not a valid prefix
        std::vector<int32_t> ids(o.h_prefix, o.h_prefix + o.nprefix);
        std::sort(ids.begin(), ids.end());
        if (std::adjacent_find(ids.begin(), ids.end()) != ids.end())
            return fail(GC_EINVAL, "prefix repeats a node id");
    }

    if (o.early_exit < 0 || o.early_exit > 1 || o.early_exit_seed < 0)
        return fail(GC_EINVAL, "early_exit must be 0 or 1 and early_exit_seed >= 0");
    if (o.early_exit && bits) return fail(GC_EINVAL, "early exit: pruned-BFS gains only");

    gc_stats st{};
    if (h_stats) st.h_evals_per_round = h_stats->h_evals_per_round;
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.words()), 2 * kWordCounters, 0u, s));
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.cuts()), 2, 0u, s));
    std::vector<int32_t> group;
    std::vector<int64_t> Fs;
    group.reserve(k);
    Fs.reserve(k);
    std::vector<uint8_t> inS((size_t)n, 0);
    std::vector<int64_t> ub((size_t)n, std::numeric_limits<int64_t>::max());
    std::vector<int32_t> last_eval((size_t)n, -1);
    std::vector<uint8_t> ds_at_eval;  // d(S,v) when v was last evaluated (features)
    // pinned host buffers the kernels read and write directly (no copy calls)
    int alloc_count = 0;
    PinnedBuf pin_cand, pin_gain, pin_flag;
    pin_cand.counter = pin_gain.counter = pin_flag.counter = &alloc_count;
    // (two sets: a block's bookkeeping overlaps the next block's launch)
    if (pin_cand.ensure(sizeof(int32_t) * (size_t)n * 2) != hipSuccess ||
        pin_gain.ensure(sizeof(int64_t) * (size_t)n * 4) != hipSuccess ||
        pin_flag.ensure(256) != hipSuccess)
        return fail(GC_ENOMEM, "pinned host buffers");
    int32_t *hc = reinterpret_cast<int32_t *>(pin_cand.p);
    int64_t *hg = reinterpret_cast<int64_t *>(pin_gain.p);
    int64_t *he = hg + n;
    int32_t *hflag = reinterpret_cast<int32_t *>(pin_flag.p);
    *hflag = 0;
    int32_t *dc = nullptr;
    int64_t *dg = nullptr;
    int32_t *dflag = nullptr;
    HIP_OK(hipHostGetDevicePointer(reinterpret_cast<void **>(&dc), hc, 0));
    HIP_OK(hipHostGetDevicePointer(reinterpret_cast<void **>(&dg), hg, 0));
    HIP_OK(hipHostGetDevicePointer(reinterpret_cast<void **>(&dflag), hflag, 0));
    // with gc_timing_enable(1): events timing the gain launches (their GPU
    // time is reported in gc_stats)
    struct EvPair {
        hipEvent_t a = nullptr, b = nullptr, score = nullptr;
        ~EvPair() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
            if (score) (void)hipEventDestroy(score);
        }
    } ev;
    HostIO io;
    if (g_timing) {
        HIP_OK(hipEventCreate(&ev.a));
        HIP_OK(hipEventCreate(&ev.b));
        io.ev0 = ev.a;
        io.ev1 = ev.b;
        io.gpu_ms = &st.ms_gain_gpu;
    }
    io.hm_gain = dg;
    io.hm_edges = dg + n;
    io.hm_flag = dflag;
    io.h_flag = hflag;
    io.hm_done = reinterpret_cast<int64_t *>(reinterpret_cast<char *>(dflag) + 64);
    io.h_done = reinterpret_cast<volatile int64_t *>(reinterpret_cast<char *>(hflag) + 64);
    *io.h_done = 0;
    io.first_level = true;
    io.cand_dev = dc;
    io.cand_host = hc;
    io.cand_len = (size_t)n * 2;
    const bool want_edges = true;
    const bool learned = o.order == GC_ORDER_LEARNED;
    const bool logging = o.log_capacity > 0 && o.h_log_round && o.h_log_node && o.h_log_gain &&
                         o.h_log_feat && o.h_log_count;
    const bool need_state = learned || logging;
    if (need_state && ws_bytes < w.L.total + gc_mlp_ws_bytes(n))
        return fail(GC_EWORKSPACE, "learned order / logging needs the full gc_workspace_size()");
    PinnedBuf pin_score, pin_feat, pin_pool;
    pin_score.counter = pin_feat.counter = pin_pool.counter = &alloc_count;
    float *hscore = nullptr, *dscore = nullptr, *hfeat = nullptr, *dfeat = nullptr;
    int32_t *hpool = nullptr, *dpool = nullptr;
    if (need_state) {
        if (pin_score.ensure(sizeof(float) * (size_t)n) != hipSuccess ||
            pin_pool.ensure(sizeof(int32_t) * (size_t)n) != hipSuccess)
            return fail(GC_ENOMEM, "pinned score buffer");
        hscore = reinterpret_cast<float *>(pin_score.p);
        HIP_OK(hipHostGetDevicePointer(reinterpret_cast<void **>(&dscore), hscore, 0));
        hpool = reinterpret_cast<int32_t *>(pin_pool.p);
        HIP_OK(hipHostGetDevicePointer(reinterpret_cast<void **>(&dpool), hpool, 0));
        if (logging) {
            if (pin_feat.ensure(sizeof(float) * 8 * (size_t)n) != hipSuccess)
                return fail(GC_ENOMEM, "pinned feature buffer");
            hfeat = reinterpret_cast<float *>(pin_feat.p);
            HIP_OK(hipHostGetDevicePointer(reinterpret_cast<void **>(&dfeat), hfeat, 0));
            *o.h_log_count = 0;
        }
    }

    // ---- s_1 (Algorithm "mem-greedy", first line) and d(S,.) of S = {s_1}
    double t0 = now_ms();
    int32_t s1;
    int64_t F1;
    int32_t dist_bytes = 1;
    int32_t v0 = -1, ecc_v0 = 0;
    if (o.nprefix > 0) {
        s1 = o.h_prefix[0];
    } else {
        rc = run_closest(g, w, s, &s1, &F1, &st.closest_sources, &ecc_v0, &v0);
        if (rc) return rc;
    }
    st.ms_closest = now_ms() - t0;
    if (getenv("GC_VERBOSE")) {
        fprintf(stderr, "[gc] first pick %d after %.2f ms (%lld sources)\n", s1, st.ms_closest,
                (long long)st.closest_sources);
        fflush(stderr);
    }
    t0 = now_ms();
    int32_t ecc = 0, claimed = 0;
    if (s1 == v0) {
        // the closeness search already left d(v0,.) and F({v0}) in the workspace
        ecc = ecc_v0;
        claimed = n;
    } else {
        rc = run_full_bfs(g, w, s1, w.dist16(), w.far(), s, &ecc);
        if (rc) return rc;
        claimed = ecc < 65535 ? n : 0;
    }
    if (claimed != n) return fail(GC_ERANGE, "eccentricity of node %d exceeds 65534", s1);
    void *d_dist;
    if (ecc <= 254) {
        HIP_OK(launch_u16_to_u8(w.dist16(), w.dist8(), n, s));
        d_dist = w.dist8();
        dist_bytes = 1;
    } else {
        d_dist = w.dist16();
        dist_bytes = 2;
    }
    if (bits && dist_bytes != 1) return fail(GC_ERANGE, "bit-vector gains need eccentricity(s1) <= 254");
    int64_t F = 0;
    HIP_OK(hipMemcpyAsync(&F, w.far(), sizeof(F), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    st.ms_update += now_ms() - t0;
    st.ecc_s1 = ecc;
    st.dist_bytes = dist_bytes;
    const int32_t ecc_bound = ecc;  // max d(S,.) never grows as S grows
    group.push_back(s1);
    Fs.push_back(F);
    inS[s1] = 1;
    // resumed prefix: rebuild d(S,.) by pruned BFS, bounds restart at +inf
    for (int32_t i = 1; i < o.nprefix; ++i) {
        const int32_t v = o.h_prefix[i];
        t0 = now_ms();
        rc = run_update_wide(g, w, v, d_dist, dist_bytes, w.far(), s, ecc_bound - 1);
        if (rc) return rc;
        HIP_OK(hipMemcpyAsync(&F, w.far(), sizeof(F), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        st.ms_update += now_ms() - t0;
        group.push_back(v);
        Fs.push_back(F);
        inS[v] = 1;
    }
    // max d(S,.) bounds the levels a pruned BFS can claim (it never grows).
    // On graphs of large eccentricity it is computed on the device after
    // every update and copied to the host by the next gain launch, so later
    // launches run only the levels that can still claim a node.  On small
    // ones (R-MAT: 4) it rarely drops and the reduction would only add a
    // kernel to every round.
    constexpr int32_t kTrackMaxdFrom = 8;
    const bool track_maxd = ecc_bound >= kTrackMaxdFrom;
    volatile int32_t *h_maxd = hflag + 32;  // byte 128 of the flag page
    *h_maxd = ecc_bound;
    if (track_maxd) {
        io.hm_maxd = dflag + 32;
        io.maxd_src = w.maxd();
        HIP_OK(launch_max_dist(d_dist, dist_bytes, n, w.maxd(), s));
    }
    auto nlev_now = [&]() {
        const int32_t md = *h_maxd;
        return std::max(std::min(ecc_bound, md) - 1, 0);
    };
    if (st.h_evals_per_round)
        for (int32_t i = 0; i < k; ++i) st.h_evals_per_round[i] = 0;
    // rows split by d(S,.) of the first gain round: d(S,.) never grows, so the
    // split bounds every later round too
    Split split;
    rc = build_split(g, w, d_dist, dist_bytes, s, &split);
    if (rc) return rc;

    const bool verbose = getenv("GC_VERBOSE") != nullptr;
    LaunchShape shape_r1, shape_later;
    int32_t cur_round = 0, first_round_idx = (int32_t)group.size();
    // early exit in the first gain round: its candidates of largest degree
    // first, exactly; every other one then stops as soon as its bound cannot
    // beat their best (see k_gain_cut)
    const bool early = o.early_exit == 1;
    const int32_t early_seed = o.early_exit_seed > 0 ? o.early_exit_seed : 1024;
    CutSpec cutspec;
    const CutSpec *cur_cut = nullptr;
    std::vector<uint8_t> seeded;
    int r1_phase = 0;
    if (early) {
        int32_t md = 0;
        HIP_OK(launch_max_dist(d_dist, dist_bytes, n, w.maxd(), s));
        HIP_OK(hipMemcpyAsync(&md, w.maxd(), sizeof(md), hipMemcpyDeviceToHost, s));
        HIP_OK(launch_tail_table(d_dist, dist_bytes, n, ecc_bound, w.tail_hist(), w.tail_T(), s));
        HIP_OK(hipStreamSynchronize(s));
        cutspec.T = w.tail_T();
        cutspec.maxd = md;
        seeded.assign((size_t)n, 0);
    }
    // evaluate a list of candidates, returning gains (and edges) on the host
    int32_t bs_round = -1, bs_levels = 0;  // bitGreedy++: round and levels of the built b^i_S rows
    auto evaluate = [&](int32_t cnt) -> int {
        LaunchShape *shape = cur_round == first_round_idx ? &shape_r1 : &shape_later;
        int r;
        if (bits) {
            // bitGreedy++: the theorem's popcount sum over the stored levels;
            // max d(S,.) <= nlev_now() + 1 bounds the levels that can count
            const bool timed = io.ev0 && io.gpu_ms;
            if (timed) HIP_OK(hipEventRecord(io.ev0, s));
            // b^i_S changes only with d(S,.): once per round (again if more
            // levels are asked for than were built)
            const int32_t ls = nlev_now() + 1;
            const bool build = bs_round != cur_round || ls > bs_levels;
            // (the gains go straight to the host-mapped buffer)
            r = run_bits_gains(g, o.d_bits, o.bits_bytes, o.bits_levels, d_dist, dist_bytes, dc, cnt, dg, s,
                               ls, true, build);
            if (build) {
                bs_round = cur_round;
                bs_levels = ls;
            }
            if (r) return r;
            if (timed) HIP_OK(hipEventRecord(io.ev1, s));
            // poll (no wake-up latency of a blocking wait), then block after 2 ms
            HIP_OK(hipEventRecord(ev.score, s));
            {
                const double tw = now_ms();
                hipError_t q = hipErrorNotReady;
                for (uint32_t spin = 0; q == hipErrorNotReady; ++spin) {
                    q = hipEventQuery(ev.score);
                    if ((spin & 255) == 255 && now_ms() - tw > 2.0) break;
                }
                if (q != hipSuccess) HIP_OK(hipEventSynchronize(ev.score));
            }
            if (timed) {
                float ms = 0.f;
                HIP_OK(hipEventElapsedTime(&ms, io.ev0, io.ev1));
                *io.gpu_ms += ms;
            }
            if (want_edges)
                for (int32_t j = 0; j < cnt; ++j) he[j] = 0;  // no per-source edge counts here
            st.gain_launches += 1;
            return GC_OK;
        }
        r = run_gains(g, w, d_dist, dist_bytes, dc, cnt, w.gain(),
                      want_edges ? w.aux() : nullptr, nullptr, s,
                      nlev_now(), hg, want_edges ? he : nullptr, &io, shape,
                      &split, false, kGainsRun, nullptr, cur_cut);
        if (r) return r;
        st.gain_launches += 1;
        return GC_OK;
    };

    // Lazy selection (Section 4.2).  A candidate u is skipped while its gain
    // from an earlier round -- an upper bound by supermodularity -- cannot beat
    // the best (gain, -id) found so far in this round; the round ends when no
    // candidate is left that could.  With the key (ub, -id) compared
    // lexicographically the pick is the plain greedy's pick (smallest id among
    // equal gains) for every candidate order.
    //   plain: ascending id scan; CELF: the largest (ub, -id) first, from a
    //   tournament tree.
    const Ws::Mlp mw = w.mlp(n);
    if (need_state) {
        // two-hop sums come from the workspace table
        rc = ensure_graph_tables(g, w, s);
        if (rc) return rc;
        HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(mw.ub), (size_t)n * 2, 0u, s));
        HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(mw.last_eval), (size_t)n, 0xFFFFFFFFu, s));
        HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(mw.dist_at_eval), ((size_t)n + 1) / 2, 0u, s));
        io.ub = mw.ub;
        io.last_eval = mw.last_eval;
        io.dist_at_eval = mw.dist_at_eval;
    }
    // Features (and, asked, learned scores) of cnt nodes listed in a host-mapped
    // id buffer, in list order.  Within a round a node's features only change
    // when it is evaluated, so computing them on demand gives the round-start
    // values for every node not yet evaluated.
    auto features_of = [&](const int32_t *d_ids, int32_t cnt, int32_t r, bool want_scores,
                           bool wait = true) -> int {
        const double tm = now_ms();
        FeatArgs fa{};
        fa.rp = g->d_rp;
        fa.ci = g->d_ci;
        fa.dist = d_dist;
        fa.cand = d_ids;
        fa.count = cnt;
        fa.ub = mw.ub;
        fa.last_eval = mw.last_eval;
        fa.dist_at_eval = mw.dist_at_eval;
        fa.two64 = w.two();
        fa.round = r;
        fa.k = k;
        fa.ecc1 = ecc_bound;
        fa.feat = logging ? dfeat : mw.feat;
        HIP_OK(launch_features(fa, dist_bytes, s));
        ++st.mlp_launches;
        if (want_scores)
            HIP_OK(launch_mlp_forward(reinterpret_cast<const MlpBlock *>(o.d_mlp), fa.feat, cnt, nullptr,
                                      nullptr, nullptr, mw.ub, d_ids, dscore, s));
        if (wait) HIP_OK(hipStreamSynchronize(s));
        else HIP_OK(hipEventRecord(ev.score, s));
        st.ms_mlp += now_ms() - tm;
        return GC_OK;
    };
    std::vector<int32_t> pool, rank, fresh;
    // learned scores by node, valid in round sc_round[u]: an unevaluated
    // node's features do not change within a round, so a score is computed
    // once per round however many blocks the round takes
    std::vector<float> sc;
    std::vector<int32_t> sc_round;
    if (learned) {
        sc.assign((size_t)n, 0.0f);
        sc_round.assign((size_t)n, -1);
    }
    // learned order: the first pool of round r + 1 is scored right behind
    // the update of round r, on the stream, and waited for when the round
    // starts; later blocks score only the nodes the round has not scored
    std::vector<int32_t> pending;
    int32_t pending_round = -1;
    bool pending_scored = false;
    // the next round's first block, chosen on the device from the scored pool
    // and launched behind the update: 0 none, 1 queued, 2 already done
    int first_state = 0;
    int32_t first_cnt = 0, first_nlev = 0;
    std::vector<int32_t> chosen;  // round in which a pooled node went into that block
    if (learned) chosen.assign((size_t)n, -1);
    auto pool_of = [&](int64_t b) { return std::max<int64_t>(b + 1, b * g->learned_pool_pct / 100); };
    const int64_t pool_size = pool_of(block);
    if (learned || bits) HIP_OK(hipEventCreateWithFlags(&ev.score, hipEventDisableTiming));
    // CELF and learned: candidates keyed by (ub, -id); a candidate taken for
    // evaluation leaves the tree and comes back with its new gain
    ArgTree keys;
    const bool plain_scan = o.order != GC_ORDER_CELF && !learned;
    // Each later launch of a round may take a larger block than the one
    // before (up to kMaxBlockGrowth x block); default 2.  The first block of
    // a round sets a threshold, and what still passes it then goes in fewer,
    // larger launches, which pays on a GPU where a launch of a few hundred
    // candidates costs little more than one of 64 -- most on graphs whose
    // rounds need thousands of evaluations (grids).
    constexpr int64_t kMaxBlockGrowth = 16;
    const int32_t growth = o.block_growth > 0 ? o.block_growth : 2;
    MaxTree tree;
    const int32_t first_gain_round = (int32_t)group.size();
    for (int32_t r = first_gain_round; r < k; ++r) {
        const double tr = now_ms();
        int64_t best_gain = -1;
        int32_t best_id = -1;
        int64_t nev = 0;
        auto can_beat = [&](int32_t u) {
            return best_id < 0 || ub[u] > best_gain || (ub[u] == best_gain && u < best_id);
        };
        // no bounds exist yet in the first round: every candidate is evaluated at once
        const bool first_round = (r == first_gain_round);
        const bool use_keys = !first_round && (o.order == GC_ORDER_CELF || learned);
        int32_t blk = first_round ? n : block;
        int32_t pos = 0;
        io.round = r;
        cur_round = r;
        // Plain and CELF, rounds >= 2: a block's launch is enqueued before the
        // previous block's bookkeeping (stale gains, trees, counters) is done,
        // so the host work overlaps the GPU's.  The next selection needs only
        // the best gain, which is taken first; the deferred candidates are
        // behind the plain scan's position or out of CELF's tree until then.
        const bool overlap = !first_round && !learned && !logging && !bits;
        int dbuf = -1;        // buffer of the deferred block (-1: none)
        int32_t dcnt = 0;
        int cur = 0;          // buffer the next block goes to
        auto book = [&](int b, int32_t c) {
            const int32_t *ids = hc + (size_t)b * n;
            const int64_t *gs = hg + (size_t)b * 2 * n;
            const int64_t *es = gs + n;
            for (int32_t j = 0; j < c; ++j) {
                const int32_t u = ids[j];
                ub[u] = gs[j];
                if (plain_scan) tree.set(u, gs[j]);
                last_eval[u] = r;
                st.edges_alg += es[j];
                if (use_keys) keys.set(u, gs[j]);
            }
        };
        for (;;) {
            int32_t cnt = 0;
            bool prelaunched = false;
            cur_cut = nullptr;
            // the CELF and plain selections fill `sel`: the free buffer when
            // overlapping, else hc
            int32_t *const sel = overlap ? hc + (size_t)cur * n : hc;
            if (learned && !first_round) {
                // the pool_of(block) largest bounds that can still win,
                // best scored first; the rest go back into the tree unchanged
                pool.clear();
                if (pending_round == r && first_state != 0) {
                    // the round's first block is on the GPU already: wait for it,
                    // cache the pool's scores and return the nodes it did not
                    // take to the tree
                    if (first_state == 1) {
                        rc = run_gains(g, w, d_dist, dist_bytes, dc, first_cnt, w.gain(), w.aux(), nullptr, s,
                                       first_nlev, hg, he, &io, &shape_later, &split, false, kGainsWait);
                        if (rc) return rc;
                    }
                    for (size_t j = 0; pending_scored && j < pending.size(); ++j) {
                        sc[pending[j]] = hscore[j];
                        sc_round[pending[j]] = r;
                    }
                    for (int32_t j = 0; j < first_cnt; ++j) chosen[hc[j]] = r;
                    for (const int32_t u : pending)
                        if (chosen[u] != r) keys.set(u, ub[u]);
                    cnt = first_cnt;
                    prelaunched = true;
                    pending.clear();
                    pending_round = -1;
                    first_state = 0;
                } else if (pending_round == r) {
                    // the round's first pool, taken from the tree and scored
                    // behind the update that ended the last round
                    // (polled: a blocking wait adds its wake-up latency to every round)
                    const double tm = now_ms();
                    if (pending_scored) {
                        hipError_t q = hipErrorNotReady;
                        for (uint32_t spin = 0; q == hipErrorNotReady; ++spin) {
                            q = hipEventQuery(ev.score);
                            if ((spin & 255) == 255 && now_ms() - tm > 2.0) break;
                        }
                        if (q != hipSuccess) HIP_OK(hipEventSynchronize(ev.score));
                    }
                    st.ms_mlp += now_ms() - tm;
                    for (size_t j = 0; pending_scored && j < pending.size(); ++j) {
                        sc[pending[j]] = hscore[j];
                        sc_round[pending[j]] = r;
                    }
                    pool.swap(pending);
                    pending_round = -1;
                }
                // (the pool grows with the block)
                while (!prelaunched && pool.size() < (size_t)pool_of(blk)) {
                    const int32_t u = keys.top();
                    if (u < 0 || !can_beat(u)) break;
                    keys.set(u, -1);
                    pool.push_back(u);
                }
                if (prelaunched) {
                } else if (pool.size() <= (size_t)blk) {
                    // the whole pool fits in the block: its order cannot matter
                    for (size_t j = 0; j < pool.size(); ++j) hc[cnt++] = pool[j];
                } else {
                    // score only the nodes this round has not scored yet
                    fresh.clear();
                    for (size_t j = 0; j < pool.size(); ++j)
                        if (sc_round[pool[j]] != r) fresh.push_back(pool[j]);
                    if (!fresh.empty()) {
                        for (size_t j = 0; j < fresh.size(); ++j) hpool[j] = fresh[j];
                        rc = features_of(dpool, (int32_t)fresh.size(), r, true);
                        if (rc) return rc;
                        for (size_t j = 0; j < fresh.size(); ++j) {
                            sc[fresh[j]] = hscore[j];
                            sc_round[fresh[j]] = r;
                        }
                    }
                    rank.assign(pool.begin(), pool.end());
                    std::sort(rank.begin(), rank.end(), [&](int32_t x, int32_t y) {
                        return sc[x] > sc[y] || (sc[x] == sc[y] && x < y);
                    });
                    for (size_t j = 0; j < rank.size(); ++j) {
                        const int32_t u = rank[j];
                        if (cnt < blk)
                            hc[cnt++] = u;
                        else
                            keys.set(u, ub[u]);
                    }
                }
            } else if (use_keys) {
                while (cnt < blk) {
                    const int32_t u = keys.top();
                    if (u < 0 || !can_beat(u)) break;  // nothing below the top can either
                    keys.set(u, -1);
                    sel[cnt++] = u;
                }
            } else if (first_round && early && r1_phase == 0) {
                // the seed of the early exit: candidates of largest degree
                for (size_t i = 0; i < g->by_degree.size() && cnt < early_seed; ++i) {
                    const int32_t u = g->by_degree[i];
                    if (inS[u]) continue;
                    hc[cnt++] = u;
                    seeded[u] = 1;
                }
                r1_phase = 1;
            } else if (first_round) {
                // every candidate at once, packed into batches ball by ball
                // (with the early exit: the others, against the seed's best)
                const int32_t *r1 = g->balls ? g->by_ball.data() : nullptr;
                for (; pos < n && cnt < blk; ++pos) {
                    const int32_t u = r1 ? r1[pos] : pos;
                    if (!inS[u] && !(early && seeded[u])) hc[cnt++] = u;
                }
                if (early) {
                    cutspec.thr = best_gain;
                    cutspec.thr_id = best_id;
                    cur_cut = &cutspec;
                }
            } else {
                // ascending ids that can still beat the best: the tree skips
                // every id whose bound is below the best gain
                const int64_t thr = best_id < 0 ? 0 : best_gain;
                while (cnt < blk && pos < n) {
                    const int32_t u = tree.first_at_least(pos, thr);
                    if (u < 0) {
                        pos = n;
                        break;
                    }
                    pos = u + 1;
                    if (can_beat(u)) sel[cnt++] = u;  // an equal bound with a larger id cannot
                }
            }
            if (cnt == 0) break;
            if (g->balls && !first_round && !prelaunched && !logging && cnt > 64 && nlev_now() >= 32) {
                // deep launches (high diameter): batches of nearby candidates
                // share more frontier entries; results go back by position
                const int32_t *rk = g->ball_rank.data();
                std::sort(sel, sel + cnt, [rk](int32_t x, int32_t y) { return rk[x] < rk[y]; });
            }
            if (logging && !first_round) {
                rc = features_of(dc, cnt, r, false);  // rows of hfeat in block order
                if (rc) return rc;
            }
            if (overlap) {
                int32_t *const dcl = dc + (size_t)cur * n;
                io.hm_gain = dg + (size_t)cur * 2 * n;
                io.hm_edges = io.hm_gain + n;
                int64_t *const hgl = hg + (size_t)cur * 2 * n;
                bool queued = false;
                rc = run_gains(g, w, d_dist, dist_bytes, dcl, cnt, w.gain(), w.aux(), nullptr, s, nlev_now(),
                               hgl, hgl + n, &io, &shape_later, &split, false, kGainsLaunch, &queued);
                if (rc) return rc;
                st.gain_launches += 1;
                if (dbuf >= 0) book(dbuf, dcnt);
                if (queued) {
                    rc = run_gains(g, w, d_dist, dist_bytes, dcl, cnt, w.gain(), w.aux(), nullptr, s, nlev_now(),
                                   hgl, hgl + n, &io, &shape_later, &split, false, kGainsWait);
                    if (rc) return rc;
                }
                io.hm_gain = dg;
                io.hm_edges = dg + n;
                for (int32_t j = 0; j < cnt; ++j) {
                    const int32_t u = sel[j];
                    const int64_t gu = hgl[j];
                    if (best_id < 0 || gu > best_gain || (gu == best_gain && u < best_id)) {
                        best_gain = gu;
                        best_id = u;
                    }
                }
                nev += cnt;
                dbuf = cur;
                dcnt = cnt;
                cur ^= 1;
                if (growth > 1)
                    blk = (int32_t)std::min<int64_t>((int64_t)blk * growth,
                                                     std::min<int64_t>((int64_t)kMaxBlockGrowth * block, n));
                continue;
            }
            if (!prelaunched) {
                rc = evaluate(cnt);
                if (rc) return rc;
            }
            if (!first_round && growth > 1)
                blk = (int32_t)std::min<int64_t>((int64_t)blk * growth, std::min<int64_t>((int64_t)kMaxBlockGrowth * block, n));
            if (logging && !first_round) {
                for (int32_t j = 0; j < cnt; ++j) {
                    const int64_t at = (*o.h_log_count)++;
                    if (at >= o.log_capacity) continue;
                    o.h_log_round[at] = r;
                    o.h_log_node[at] = hc[j];
                    o.h_log_gain[at] = hg[j];
                    std::memcpy(o.h_log_feat + at * 8, hfeat + (size_t)j * 8, 8 * sizeof(float));
                }
            }
            for (int32_t j = 0; j < cnt; ++j) {
                const int32_t u = hc[j];
                const int64_t gu = hg[j];
                ub[u] = gu;
                if (plain_scan && !first_round) tree.set(u, gu);
                last_eval[u] = r;
                st.edges_alg += he[j];
                if (best_id < 0 || gu > best_gain || (gu == best_gain && u < best_id)) {
                    best_gain = gu;
                    best_id = u;
                }
                if (use_keys) keys.set(u, gu);
            }
            nev += cnt;
        }
        if (dbuf >= 0) book(dbuf, dcnt);
        if (first_round && plain_scan) tree.build(ub, inS);
        if (first_round && (o.order == GC_ORDER_CELF || learned)) {
            keys.build(ub, inS, best_id);
        }
        if (first_round) {
            st.evals_round1 += nev;
            st.ms_round1 += now_ms() - tr;
        } else {
            st.evals_later += nev;
            st.ms_later += now_ms() - tr;
        }
        if (st.h_evals_per_round) st.h_evals_per_round[r] = nev;
        st.evals_total += nev;
        if (verbose) {
            fprintf(stderr, "[gc] round %d: %lld evaluations, best %d gain %lld, %.2f ms since start\n", r,
                    (long long)nev, best_id, (long long)best_gain, now_ms() - t_start);
            fflush(stderr);
        }
        if (best_id < 0) return fail(GC_EINVAL, "no candidate left");
        // pick, then d(S,.) <- min(d(S,.), d(pick,.)) by pruned BFS
        t0 = now_ms();
        rc = run_update_wide(g, w, best_id, d_dist, dist_bytes, w.far(), s, nlev_now(), &split);
        if (rc) return rc;
        if (track_maxd && r + 1 < k) HIP_OK(launch_max_dist(d_dist, dist_bytes, n, w.maxd(), s));
        F -= best_gain;
        if (o.debug_checks || r == k - 1) {
            // the update BFS tracks F(S) on its own: it must agree with the gains
            int64_t Fdev = 0;
            HIP_OK(hipMemcpyAsync(&Fdev, w.far(), sizeof(Fdev), hipMemcpyDeviceToHost, s));
            HIP_OK(hipStreamSynchronize(s));
            if (Fdev != F)
                return fail(GC_EDEVICE, "farness mismatch after pick %d: update %lld vs gains %lld",
                            r, (long long)Fdev, (long long)F);
        }
        st.ms_update += now_ms() - t0;
        group.push_back(best_id);
        Fs.push_back(F);
        inS[best_id] = 1;
        if (plain_scan && !tree.t.empty()) tree.set(best_id, -1);
        if (!keys.t.empty()) keys.set(best_id, -1);
        if (learned && r + 1 < k) {
            // take the next round's first pool now and score it on the
            // stream behind the update (nothing is evaluated before it is
            // used, so every one of them can still win)
            pending.clear();
            while (pending.size() < (size_t)pool_size) {
                const int32_t u = keys.top();
                if (u < 0) break;
                keys.set(u, -1);
                pending.push_back(u);
            }
            // a pool that fits in one block is evaluated whole, unscored
            pending_scored = pending.size() > (size_t)block;
            if (pending_scored) {
                for (size_t j = 0; j < pending.size(); ++j) hpool[j] = pending[j];
                rc = features_of(dpool, (int32_t)pending.size(), r + 1, true, false);
                if (rc) return rc;
            }
            pending_round = r + 1;
            // ... and, without logging, its first block: the block best
            // scored, chosen on the device into the host-mapped candidate
            // list, and its gain launch, all on the stream behind the update
            if (!logging && !pending.empty() && pending.size() <= (size_t)kSelectMax) {
                if (pending_scored) {
                    first_cnt = block;
                    HIP_OK(launch_select_top(dscore, dpool, (int32_t)pending.size(), first_cnt, dc, s));
                } else {
                    first_cnt = (int32_t)pending.size();
                    for (int32_t j = 0; j < first_cnt; ++j) hc[j] = pending[(size_t)j];
                }
                io.round = r + 1;
                first_nlev = nlev_now();
                bool q = false;
                // (ids chosen on the device are not in the host's view until the stream gets there)
                const int32_t *const cand_host = io.cand_host;
                if (pending_scored) io.cand_host = nullptr;
                rc = run_gains(g, w, d_dist, dist_bytes, dc, first_cnt, w.gain(), w.aux(), nullptr, s,
                               first_nlev, hg, he, &io, &shape_later, &split, false, kGainsLaunch, &q);
                io.cand_host = cand_host;
                if (rc) return rc;
                st.gain_launches += 1;
                first_state = q ? 1 : 2;
            }
        }
    }
    for (int32_t i = 0; i < k; ++i) {
        h_group[i] = group[i];
        h_farness[i] = Fs[i];
    }
    st.ms_total = now_ms() - t_start;
    if (bits) {
        HIP_OK(hipMemcpyAsync(&st.bits_words, bits_words_counter(g, o.d_bits, o.bits_bytes), sizeof(int64_t),
                              hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
    }
    if (h_stats) {
        int64_t wc[kWordCounters];
        HIP_OK(hipMemcpyAsync(wc, w.words(), sizeof(wc), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        st.entries_word = wc[0];
        st.entries_root = wc[1];
        st.entries_last = wc[2];
        st.edges_word = wc[3];
        st.edges_last = wc[4];
        st.touched_word = wc[5];
        HIP_OK(hipMemcpyAsync(&st.cut_evals, w.cuts(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        *h_stats = st;
    }
    return GC_OK;
}

// ------------------------------------------------ candidate-ordering MLP

extern "C" size_t gc_mlp_block_bytes(void) { return sizeof(MlpBlock); }

extern "C" int gc_mlp_pack(const float *d_master, void *d_block, hipStream_t stream) {
    if (!d_master || !d_block) return fail(GC_EINVAL, "NULL device pointer");
    HIP_OK(launch_mlp_pack(d_master, reinterpret_cast<MlpBlock *>(d_block), stream));
    return GC_OK;
}

extern "C" int gc_mlp_forward(const void *d_block, const float *d_x, int32_t count, float *d_out,
                              float *d_h1, float *d_h2, hipStream_t stream) {
    if (count < 0) return fail(GC_EINVAL, "count < 0");
    if (count > 0 && (!d_block || !d_x || !d_out)) return fail(GC_EINVAL, "NULL device pointer");
    HIP_OK(launch_mlp_forward(reinterpret_cast<const MlpBlock *>(d_block), d_x, count, d_out, d_h1,
                              d_h2, nullptr, nullptr, nullptr, stream));
    return GC_OK;
}

extern "C" size_t gc_mlp_scratch_floats(int32_t count) {
    if (count < 0) return 0;
    return ((size_t)count + 63) / 64 * 64 + 2 * (size_t)count * GC_MLP_HIDDEN;
}

extern "C" int gc_mlp_backward(const void *d_block, const float *d_x, const float *d_h1,
                               const float *d_h2, const float *d_out, const float *d_y,
                               int32_t count, float *d_grad, float *d_scratch, hipStream_t stream) {
    if (count < 1) return fail(GC_EINVAL, "count must be >= 1");
    if (!d_block || !d_x || !d_h1 || !d_h2 || !d_out || !d_y || !d_grad || !d_scratch)
        return fail(GC_EINVAL, "NULL device pointer");
    HIP_OK(launch_mlp_backward(reinterpret_cast<const MlpBlock *>(d_block), d_x, d_h1, d_h2, d_out,
                               d_y, count, d_grad, d_scratch, stream));
    return GC_OK;
}

extern "C" int gc_mlp_adam(float *d_master, float *d_m, float *d_v, const float *d_grad,
                           int32_t step, float lr, float beta1, float beta2, float eps,
                           hipStream_t stream) {
    if (!d_master || !d_m || !d_v || !d_grad) return fail(GC_EINVAL, "NULL device pointer");
    if (step < 1) return fail(GC_EINVAL, "step counts from 1");
    HIP_OK(launch_mlp_adam(d_master, d_m, d_v, d_grad, step, lr, beta1, beta2, eps, stream));
    return GC_OK;
}

extern "C" int gc_greedy_many(int32_t count, const gc_graph *const *graphs, const int32_t *k,
                              const gc_opts *opts, int32_t nworkers, void *const *d_ws,
                              const size_t *ws_bytes, const hipStream_t *streams, int32_t *h_group,
                              int64_t *h_farness, gc_stats *h_stats) {
    if (count < 0) return fail(GC_EINVAL, "count < 0");
    if (count == 0) return GC_OK;
    if (!graphs || !k || !d_ws || !ws_bytes || !streams || !h_group || !h_farness)
        return fail(GC_EINVAL, "NULL argument");
    if (nworkers < 1 || nworkers > 64) return fail(GC_EINVAL, "nworkers = %d outside [1, 64]", nworkers);
    if (opts && (opts->nprefix != 0 || opts->log_capacity > 0))
        return fail(GC_EINVAL, "gc_greedy_many takes no prefix and no log");
    for (int32_t w = 0; w < nworkers; ++w) {
        if (!d_ws[w]) return fail(GC_EINVAL, "workspace %d is NULL", w);
        if (nworkers > 1 && !streams[w]) return fail(GC_EINVAL, "worker %d on the null stream", w);
    }
    std::vector<int64_t> off((size_t)count + 1, 0);
    for (int32_t i = 0; i < count; ++i) {
        if (!graphs[i]) return fail(GC_EINVAL, "graph %d is NULL", i);
        if (k[i] < 1 || k[i] > graphs[i]->n) return fail(GC_EINVAL, "job %d: k = %d outside [1, n]", i, k[i]);
        off[(size_t)i + 1] = off[(size_t)i] + k[i];
    }
    // largest graph first (ties by job index): the long jobs start early
    std::vector<int32_t> order((size_t)count);
    for (int32_t i = 0; i < count; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return graphs[a]->nnz + graphs[a]->n > graphs[b]->nnz + graphs[b]->n;
    });
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    std::atomic<int32_t> next{0};
    // a job no worker could take keeps this error
    std::vector<int> rc((size_t)count, GC_EDEVICE);
    std::vector<std::string> msg((size_t)count, std::string("not run: no worker could select the device"));
    auto work = [&](int32_t w) {
        if (hipSetDevice(dev) != hipSuccess) return;
        const SlotSums slot_sums;
        ZeroRange zero;  // nothing is known of the workspace before its first job
        for (;;) {
            const int32_t t = next.fetch_add(1);
            if (t >= count) break;
            const int32_t i = order[(size_t)t];
            if (h_stats) h_stats[i].h_evals_per_round = nullptr;
            int r = ws_init_reuse(graphs[i], d_ws[w], ws_bytes[w], streams[w], zero);
            if (r == GC_OK)
                r = gc_greedy_group(graphs[i], k[i], opts, d_ws[w], ws_bytes[w], streams[w],
                                    h_group + off[(size_t)i], h_farness + off[(size_t)i],
                                    h_stats ? &h_stats[i] : nullptr);
            if (r == GC_OK) zero = ws_record_range(graphs[i]);
            rc[(size_t)i] = r;
            if (r != GC_OK) msg[(size_t)i] = g_last_error;
        }
    };
    if (nworkers == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        th.reserve((size_t)nworkers);
        for (int32_t w = 0; w < nworkers; ++w) th.emplace_back(work, w);
        for (auto &t : th) t.join();
    }
    for (int32_t i = 0; i < count; ++i)
        if (rc[(size_t)i] != GC_OK) return fail(rc[(size_t)i], "job %d: %s", i, msg[(size_t)i].c_str());
    return GC_OK;
}

// ------------------------------------------------------------ batched jobs
//
// gc_greedy_batch: many independent jobs, their later rounds in lockstep.
// Phase 1 runs each job's first pick, first gain round (every candidate, one
// call) and second pick on the worker threads, as gc_greedy_many would, and
// leaves the job's d(S,.) in one array over the disjoint union of all the
// graphs and its first-round gains on the host.  Phase 2 then advances every
// job through its later rounds at once: in each step every job still
// selecting contributes its next batch of candidates (the same lazy rule and
// batch schedule as gc_greedy_group, so picks and evaluation counts are the
// same), and one gain call over the union evaluates all of them; the jobs
// whose round ended get their d(S,.) update in one write-mode call.  A batch
// holds sources of one job only and gets records for that job's nodes only
// (WideArgs::bbase), so a step's records scale with the jobs' sizes, not
// with the union's.

namespace {

struct BatchJob {
    const gc_graph *g = nullptr;
    int32_t k = 0;
    int32_t nb = 0;   // first node of the job in the union
    int64_t eb = 0;   // first adjacency entry of the job in the union
    int32_t ecc = 0;  // eccentricity of the first pick
    std::vector<int32_t> group;
    std::vector<int64_t> F;
    std::vector<int64_t> ub;     // stale gains (local ids); -1 for members of S
    std::vector<uint8_t> inS;
    std::vector<int64_t> evals;  // per round
    gc_stats st{};
    int rc = GC_OK;
    std::string msg;
    // phase 2
    MaxTree tree;
    ArgTree keys;
    bool in_round = false;
    int32_t pos = 0, bid = -1;
    int64_t bgain = -1, cur = 0, nev = 0;
    std::vector<int32_t> batch;  // local ids of the current step's batch
};

// union record budget: a step gives each job at most 16 blocks of candidates
int64_t batch_union_kmax(int32_t block) { return 16LL * std::max(block, 1) / 64 + 2; }

void batch_union_graph(const gc_graph *const *graphs, int32_t count, int32_t block, gc_graph *gu) {
    int64_t N = 0, NNZ = 0;
    int32_t md = 0;
    for (int32_t i = 0; i < count; ++i) {
        N += graphs[i]->n;
        NNZ += graphs[i]->nnz;
        md = std::max(md, graphs[i]->max_deg);
    }
    const gc_graph *g0 = graphs[0];
    gu->n = (int32_t)N;
    gu->nnz = NNZ;
    gu->max_deg = md;
    gu->num_cu = g0->num_cu;
    gu->level_wgs_per_cu = g0->level_wgs_per_cu;
    gu->unroll = g0->unroll;
    gu->min_edges = g0->min_edges;
    gu->unroll_small = g0->unroll_small;
    gu->min_edges_small = g0->min_edges_small;
    gu->learned_pool_pct = g0->learned_pool_pct;
    gu->balls = false;
    gu->directed = false;
    gu->level_cap = g0->level_cap;
    const int64_t stride = (N + 31) & ~(int64_t)31;
    gu->vis_budget = batch_union_kmax(block) * stride * 32;
    gu->log_entries = std::min<int64_t>((int64_t)256 << 20, std::max<int64_t>((int64_t)8 << 20, 16LL * N));
    gu->touch_entries = 0;
}

struct BatchUnionLayout {
    WsLayout L;
    size_t rp, ci, bbase, src, gout, total;
    int64_t max_batches;
};

BatchUnionLayout batch_union_layout(const gc_graph *gu, int32_t count) {
    BatchUnionLayout U;
    U.L = ws_layout(gu);
    size_t o = al256(U.L.total);
    U.rp = o; o += al256(((size_t)gu->n + 1) * 4);
    U.ci = o; o += al256((size_t)gu->nnz * 4 + 4);
    // a step's batches: at most one partial batch per job beyond n / 64
    U.max_batches = (int64_t)gu->n / 64 + 2LL * count + 64;
    U.bbase = o; o += al256((size_t)U.max_batches * 8);
    // sources of a launch (whole batches of 64, padded) and their gains and
    // adjacency counts: up to 64 per batch, which may exceed the node count
    U.src = o; o += al256((size_t)U.max_batches * 64 * 4);
    U.gout = o; o += al256((size_t)U.max_batches * 64 * 16);
    U.total = o;
    return U;
}

// Phase 1 of one job on a worker: s1, d(s1,.), every first-round gain, s2 and
// the update; d(S,.) goes to the union's uint16 array at the job's offset.
int batch_phase1(BatchJob &J, void *d_ws, size_t ws_bytes, hipStream_t s, uint16_t *u_dist16, ZeroRange &zero,
                 bool celf) {
    const gc_graph *g = J.g;
    const int32_t n = g->n;
    int rc = ws_init_reuse(g, d_ws, ws_bytes, s, zero);
    if (rc) return rc;
    Ws w;
    rc = get_ws(g, d_ws, ws_bytes, &w);
    if (rc) return rc;
    const double t0 = now_ms();
    int32_t s1 = -1, v0 = -1, ecc_v0 = 0;
    int64_t F1 = 0;
    rc = run_closest(g, w, s, &s1, &F1, &J.st.closest_sources, &ecc_v0, &v0);
    if (rc) return rc;
    J.st.ms_closest = now_ms() - t0;
    const double t1 = now_ms();
    int32_t ecc = 0;
    if (s1 == v0) {
        ecc = ecc_v0;  // the closeness search left d(v0,.) in dist16
    } else {
        rc = run_full_bfs(g, w, s1, w.dist16(), w.far(), s, &ecc);
        if (rc) return rc;
    }
    if (ecc >= 65535) return fail(GC_ERANGE, "eccentricity of node %d exceeds 65534", s1);
    HIP_OK(hipMemcpyAsync(&F1, w.far(), sizeof(F1), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    J.ecc = ecc;
    J.group.assign(1, s1);
    J.F.assign(1, F1);
    J.inS.assign((size_t)n, 0);
    J.inS[(size_t)s1] = 1;
    J.ub.assign((size_t)n, std::numeric_limits<int64_t>::max());
    J.ub[(size_t)s1] = -1;
    J.evals.assign((size_t)J.k, 0);
    J.st.ecc_s1 = ecc;
    J.st.ms_update += now_ms() - t1;
    if (J.k >= 2) {
        const double t2 = now_ms();
        void *d_dist = w.dist16();
        int dist_bytes = 2;
        if (ecc <= 254) {
            HIP_OK(launch_u16_to_u8(w.dist16(), w.dist8(), n, s));
            d_dist = w.dist8();
            dist_bytes = 1;
        }
        Split split;
        rc = build_split(g, w, d_dist, dist_bytes, s, &split);
        if (rc) return rc;
        // every other node, batched ball by ball as in gc_greedy_group's first round
        std::vector<int32_t> cand;
        cand.reserve((size_t)n);
        const auto &ord = g->balls ? g->by_ball : g->by_degree;
        for (int32_t i = 0; i < n; ++i) {
            const int32_t u = g->balls ? ord[(size_t)i] : i;
            if (u != s1) cand.push_back(u);
        }
        const int32_t cnt = (int32_t)cand.size();
        std::vector<int64_t> hg((size_t)cnt), he((size_t)cnt);
        if (cnt > 0) {
            HIP_OK(hipMemcpyAsync(w.cand(), cand.data(), sizeof(int32_t) * (size_t)cnt, hipMemcpyHostToDevice, s));
            rc = run_gains(g, w, d_dist, dist_bytes, w.cand(), cnt, w.gain(), w.aux(), nullptr, s,
                           std::max(ecc - 1, 0), hg.data(), he.data(), nullptr, nullptr, &split);
            if (rc) return rc;
        }
        int64_t bgain = -1;
        int32_t bid = -1;
        for (int32_t j = 0; j < cnt; ++j) {
            const int32_t u = cand[(size_t)j];
            J.ub[(size_t)u] = hg[(size_t)j];
            J.st.edges_alg += he[(size_t)j];
            if (hg[(size_t)j] > bgain || (hg[(size_t)j] == bgain && u < bid)) {
                bgain = hg[(size_t)j];
                bid = u;
            }
        }
        J.st.evals_round1 = cnt;
        J.evals[1] = cnt;
        J.st.gain_launches += 1;
        J.st.ms_round1 = now_ms() - t2;
        if (bid < 0) return fail(GC_EDEVICE, "no candidate in the first gain round");
        const double t3 = now_ms();
        rc = run_update_wide(g, w, bid, d_dist, dist_bytes, w.far(), s, std::max(ecc - 1, 0), &split);
        if (rc) return rc;
        int64_t F2 = 0;
        HIP_OK(hipMemcpyAsync(&F2, w.far(), sizeof(F2), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        if (F2 != F1 - bgain)
            return fail(GC_EDEVICE, "update of node %d: F %lld, expected %lld", bid, (long long)F2,
                        (long long)(F1 - bgain));
        J.group.push_back(bid);
        J.F.push_back(F2);
        J.inS[(size_t)bid] = 1;
        J.ub[(size_t)bid] = -1;
        if (dist_bytes == 1) HIP_OK(launch_u8_to_u16(w.dist8(), u_dist16 + J.nb, n, s));
        else HIP_OK(hipMemcpyAsync(u_dist16 + J.nb, w.dist16(), sizeof(uint16_t) * (size_t)n,
                                   hipMemcpyDeviceToDevice, s));
        J.st.ms_update += now_ms() - t3;
    } else {
        HIP_OK(hipMemcpyAsync(u_dist16 + J.nb, w.dist16(), sizeof(uint16_t) * (size_t)n, hipMemcpyDeviceToDevice,
                              s));
    }
    // the stale-gain tree of the later rounds, built while the copy runs
    if ((int32_t)J.group.size() < J.k) {
        if (celf) J.keys.build(J.ub, J.inS, -1);
        else J.tree.build(J.ub, J.inS);
    }
    // the worker's workspace is prepared again for its next job: wait for the copy
    HIP_OK(hipStreamSynchronize(s));
    return GC_OK;
}

// One gain (or, write = true, update) call over the union: `lists` holds, per
// job taking part, its sources as union ids; gains (and edges) come back in
// the same order.  Batches hold one job's sources each, padded with -1; a
// launch takes batches while their records fit.
struct UnionCall {
    const gc_graph *gu;
    const Ws *w;
    const std::vector<BatchJob> *jobs;
    int64_t *d_bbase;
    int32_t *d_src;      // max_batches * 64 sources
    int64_t *d_gain;     // max_batches * 64 gains, then as many adjacency counts
    int64_t max_batches;
    const void *d_dist;
    int dist_bytes;
    int32_t nlev;
    const Split *split;
    hipStream_t s;
    PinnedBuf *pin_src, *pin_base;
    std::vector<int64_t> hout;
    int64_t launches = 0;
};

int union_call(UnionCall &c, const std::vector<std::pair<int32_t, std::vector<int32_t>>> &lists, bool write,
               std::vector<int64_t> &gain, std::vector<int64_t> &edges) {
    const Ws &w = *c.w;
    const gc_graph *gu = c.gu;
    const int64_t R_all = w.L.kmax * (int64_t)w.L.vis_stride;  // records of the union workspace
    // flat layout: per list, its batches of 64 slots
    struct Bt {
        int32_t list, job;
        int64_t first;  // index of the batch's first source in the list
    };
    std::vector<Bt> bts;
    std::vector<int64_t> out_off(lists.size() + 1, 0);
    for (size_t l = 0; l < lists.size(); ++l) {
        const int64_t cnt = (int64_t)lists[l].second.size();
        for (int64_t f = 0; f < cnt; f += 64) bts.push_back({(int32_t)l, lists[l].first, f});
        out_off[l + 1] = out_off[l] + cnt;
    }
    gain.assign((size_t)out_off.back(), 0);
    edges.assign((size_t)out_off.back(), 0);
    if (bts.empty()) return GC_OK;
    const int64_t slots_cap = std::min<int64_t>(c.max_batches * 64, (int64_t)(c.pin_src->bytes / 4));
    int64_t R = R_all;
    const int grid = wide_grid(gu);
    size_t b0 = 0;
    while (b0 < bts.size()) {
        // the batches of this launch
        size_t b1 = b0;
        int64_t recs = 0;
        while (b1 < bts.size()) {
            const int64_t nj = (*c.jobs)[(size_t)bts[b1].job].g->n;
            if (b1 > b0 && (recs + nj > R || (int64_t)(b1 - b0 + 1) * 64 > slots_cap ||
                            (int64_t)(b1 - b0 + 1) > c.max_batches))
                break;
            recs += nj;
            ++b1;
        }
        if (recs > R_all) return fail(GC_EWORKSPACE, "union workspace too small for one batch");
        const int64_t nb = (int64_t)(b1 - b0);
        int32_t *hs = reinterpret_cast<int32_t *>(c.pin_src->p);
        int64_t *hb = reinterpret_cast<int64_t *>(c.pin_base->p);
        int64_t rec_at = 0;
        for (int64_t q = 0; q < nb; ++q) {
            const Bt &bt = bts[b0 + (size_t)q];
            const BatchJob &J = (*c.jobs)[(size_t)bt.job];
            hb[q] = rec_at - J.nb;
            rec_at += J.g->n;
            const auto &L = lists[(size_t)bt.list].second;
            for (int64_t j = 0; j < 64; ++j) {
                const int64_t x = bt.first + j;
                hs[q * 64 + j] = x < (int64_t)L.size() ? L[(size_t)x] : -1;
            }
        }
        const int64_t nsrc = nb * 64;
        HIP_OK(hipMemcpyAsync(c.d_src, hs, sizeof(int32_t) * (size_t)nsrc, hipMemcpyHostToDevice, c.s));
        HIP_OK(hipMemcpyAsync(c.d_bbase, hb, sizeof(int64_t) * (size_t)nb, hipMemcpyHostToDevice, c.s));
        WideArgs a = w.wide();
        a.unroll = nsrc <= 1024 ? gu->unroll_small : gu->unroll;
        a.min_edges = nsrc <= 1024 ? gu->min_edges_small : gu->min_edges;
        a.rp = gu->d_rp;
        a.ci = gu->d_ci;
        a.n = gu->n;
        a.dist = c.d_dist;
        a.src = c.d_src;
        a.nsrc = nsrc;
        a.spb = 64;
        a.gain = c.d_gain;
        a.edges = c.d_gain + nsrc;
        a.visited = nullptr;
        a.tag = 1;
        a.dist_bytes = c.dist_bytes;
        a.words = w.words();
        a.write = write;
        a.far = nullptr;
        a.bbase = c.d_bbase;
        apply_split(a, c.split);
        // (many jobs in one launch: window sums in LDS slots)
        a.pack = gu->nnz < (1ll << kPackShift) &&
                         (int64_t)gu->n * (int64_t)(c.nlev + 1) < (1ll << (62 - kPackShift))
                     ? 2
                     : 0;
        HIP_OK(launch_wide_begin(a, c.dist_bytes, c.nlev, c.s));
        HIP_OK(launch_wide_levels(a, c.dist_bytes, 0, c.nlev, grid, c.s));
        HIP_OK(launch_wide_end(a, c.nlev, grid, c.s));
        c.launches += 1;
        int32_t flag = 0;
        // results into ordinary (cached) host memory: the scatter below reads
        // every value, and reads of pinned memory bypass the CPU caches
        c.hout.resize(2 * (size_t)nsrc);
        int64_t *ho = c.hout.data();
        HIP_OK(hipMemcpyAsync(&flag, w.flags(), sizeof(flag), hipMemcpyDeviceToHost, c.s));
        HIP_OK(hipMemcpyAsync(ho, c.d_gain, sizeof(int64_t) * 2 * (size_t)nsrc, hipMemcpyDeviceToHost, c.s));
        HIP_OK(hipStreamSynchronize(c.s));
        if (flag) {
            // the frontier log overflowed: clear, and redo with fewer records per launch
            if (write) return fail(GC_EWORKSPACE, "frontier log too small for the batched update");
            HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.base + w.L.wvis),
                                   (size_t)w.L.kmax * w.L.vis_stride * 8, 0u, c.s));
            HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.base + w.L.lvl),
                                   (size_t)(c.nlev + 2) * sizeof(WideLevel) / 4, 0u, c.s));
            HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.zcnt()), 2, 0u, c.s));
            HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(w.flags()), 1, 0u, c.s));
            if (nb == 1) return fail(GC_EWORKSPACE, "frontier log too small for one batch");
            R = std::max<int64_t>(1, recs / 2);
            continue;
        }
        for (int64_t q = 0; q < nb; ++q) {
            const Bt &bt = bts[b0 + (size_t)q];
            const int64_t cnt = (int64_t)lists[(size_t)bt.list].second.size();
            for (int64_t j = 0; j < 64 && bt.first + j < cnt; ++j) {
                const size_t o = (size_t)(out_off[(size_t)bt.list] + bt.first + j);
                gain[o] = ho[q * 64 + j];
                edges[o] = ho[nsrc + q * 64 + j];
            }
        }
        b0 = b1;
    }
    return GC_OK;
}

}  // namespace

extern "C" int gc_batch_union_size(int32_t count, const gc_graph *const *graphs, int32_t block, size_t *bytes) {
    if (count < 1 || !graphs || !bytes) return fail(GC_EINVAL, "bad argument");
    int64_t N = 0, NNZ = 0;
    for (int32_t i = 0; i < count; ++i) {
        if (!graphs[i]) return fail(GC_EINVAL, "graph %d is NULL", i);
        if (graphs[i]->weighted) return fail(GC_EINVAL, "graph %d is weighted: batches take unweighted graphs", i);
        N += graphs[i]->n;
        NNZ += graphs[i]->nnz;
    }
    if (N >= INT32_MAX || NNZ >= INT32_MAX) return fail(GC_ERANGE, "the union of the graphs exceeds 2^31 nodes or entries");
    gc_graph gu;
    batch_union_graph(graphs, count, block > 0 ? block : kSrc, &gu);
    *bytes = batch_union_layout(&gu, count).total;
    return GC_OK;
}

extern "C" int gc_greedy_batch(int32_t count, const gc_graph *const *graphs, const int32_t *k,
                               const gc_opts *opts, int32_t nworkers, void *const *d_ws,
                               const size_t *ws_bytes, const hipStream_t *streams, void *d_union,
                               size_t union_bytes, int32_t *h_group, int64_t *h_farness, gc_stats *h_stats) {
    const double t_start = now_ms();
    if (count < 0) return fail(GC_EINVAL, "count < 0");
    if (count == 0) return GC_OK;
    if (!graphs || !k || !d_ws || !ws_bytes || !streams || !h_group || !h_farness || !d_union)
        return fail(GC_EINVAL, "NULL argument");
    if (nworkers < 1 || nworkers > 64) return fail(GC_EINVAL, "nworkers = %d outside [1, 64]", nworkers);
    gc_opts o{};
    if (opts) o = *opts;
    if (o.nprefix != 0 || o.log_capacity > 0 || o.d_bits || o.early_exit || o.d_mlp)
        return fail(GC_EINVAL, "gc_greedy_batch: plain or CELF order, no prefix, log, bit vectors or early exit");
    if (o.order != GC_ORDER_PLAIN && o.order != GC_ORDER_CELF)
        return fail(GC_EINVAL, "gc_greedy_batch: plain or CELF order");
    if (o.bitset_width != 0 && o.bitset_width != 64) return fail(GC_EINVAL, "bitset_width must be 64");
    if (o.block < 0) return fail(GC_EINVAL, "block < 0");
    if (o.block_growth < 0 || o.block_growth > 8) return fail(GC_EINVAL, "block_growth outside [0, 8]");
    const int32_t block = o.block > 0 ? o.block : kSrc;
    const int32_t growth = o.block_growth > 0 ? o.block_growth : 2;
    for (int32_t w = 0; w < nworkers; ++w) {
        if (!d_ws[w]) return fail(GC_EINVAL, "workspace %d is NULL", w);
        if (nworkers > 1 && !streams[w]) return fail(GC_EINVAL, "worker %d on the null stream", w);
    }
    size_t need = 0;
    int rc = gc_batch_union_size(count, graphs, block, &need);
    if (rc) return rc;
    if (((uintptr_t)d_union & 255) != 0) return fail(GC_EWORKSPACE, "union workspace must be 256-byte aligned");
    if (union_bytes < need)
        return fail(GC_EWORKSPACE, "union workspace has %zu bytes, needs %zu", union_bytes, need);
    std::vector<BatchJob> jobs((size_t)count);
    std::vector<int64_t> off((size_t)count + 1, 0);
    int64_t nb = 0, eb = 0;
    for (int32_t i = 0; i < count; ++i) {
        if (k[i] < 1 || k[i] > graphs[i]->n) return fail(GC_EINVAL, "job %d: k = %d outside [1, n]", i, k[i]);
        jobs[(size_t)i].g = graphs[i];
        jobs[(size_t)i].k = k[i];
        jobs[(size_t)i].nb = (int32_t)nb;
        jobs[(size_t)i].eb = eb;
        nb += graphs[i]->n;
        eb += graphs[i]->nnz;
        off[(size_t)i + 1] = off[(size_t)i] + k[i];
    }
    // the union graph over the caller's buffer
    gc_graph gu;
    batch_union_graph(graphs, count, block, &gu);
    const BatchUnionLayout U = batch_union_layout(&gu, count);
    char *ub = reinterpret_cast<char *>(d_union);
    int32_t *urp = reinterpret_cast<int32_t *>(ub + U.rp);
    int32_t *uci = reinterpret_cast<int32_t *>(ub + U.ci);
    gu.d_rp = urp;
    gu.d_ci = uci;
    Ws wu;
    wu.L = U.L;
    wu.base = ub;
    wu.bytes = U.L.total;
    const hipStream_t s0 = streams[0];
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(ub), U.L.total / 4, 0u, s0));
    for (const BatchJob &J : jobs) {
        HIP_OK(launch_copy_add_i32(J.g->d_rp, urp + J.nb, J.g->n, (int32_t)J.eb, s0));
        if (J.g->nnz > 0) HIP_OK(launch_copy_add_i32(J.g->d_ci, uci + J.eb, J.g->nnz, J.nb, s0));
    }
    HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(urp + gu.n), 1, (uint32_t)gu.nnz, s0));
    HIP_OK(hipStreamSynchronize(s0));
    uint16_t *u16 = wu.dist16();

    // ---- phase 1 on the workers, largest graph first
    const double t1 = now_ms();
    std::vector<int32_t> order((size_t)count);
    for (int32_t i = 0; i < count; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return graphs[a]->nnz + graphs[a]->n > graphs[b]->nnz + graphs[b]->n;
    });
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    std::atomic<int32_t> next{0};
    for (BatchJob &J : jobs) {
        J.rc = GC_EDEVICE;
        J.msg = "not run: no worker could select the device";
    }
    auto work = [&](int32_t wk) {
        if (hipSetDevice(dev) != hipSuccess) return;
        const SlotSums slot_sums;
        ZeroRange zero;
        for (;;) {
            const int32_t t = next.fetch_add(1);
            if (t >= count) break;
            BatchJob &J = jobs[(size_t)order[(size_t)t]];
            const int r = batch_phase1(J, d_ws[wk], ws_bytes[wk], streams[wk], u16, zero,
                                       o.order == GC_ORDER_CELF);
            if (r == GC_OK) zero = ws_record_range(J.g);
            J.rc = r;
            if (r != GC_OK) J.msg = g_last_error;
        }
    };
    if (nworkers == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        th.reserve((size_t)nworkers);
        for (int32_t w = 0; w < nworkers; ++w) th.emplace_back(work, w);
        for (auto &t : th) t.join();
    }
    for (int32_t i = 0; i < count; ++i)
        if (jobs[(size_t)i].rc != GC_OK) return fail(jobs[(size_t)i].rc, "job %d: %s", i, jobs[(size_t)i].msg.c_str());
    const double ms_phase1 = now_ms() - t1;

    // ---- phase 2: every job's later rounds in lockstep, on streams[0]
    const double t2 = now_ms();
    int32_t maxecc = 0;
    for (const BatchJob &J : jobs) maxecc = std::max(maxecc, J.ecc);
    const void *udist = u16;
    int dist_bytes = 2;
    if (maxecc <= 254) {
        HIP_OK(launch_u16_to_u8(u16, wu.dist8(), gu.n, s0));
        udist = wu.dist8();
        dist_bytes = 1;
    }
    const int32_t nlev = std::max(maxecc - 1, 0);
    Split usplit;
    rc = build_split(&gu, wu, udist, dist_bytes, s0, &usplit);
    if (rc) return rc;
    int alloc_count = 0;
    PinnedBuf pin_src, pin_base;
    pin_src.counter = pin_base.counter = &alloc_count;
    const int64_t max_slots = U.max_batches * 64;
    if (pin_src.ensure(sizeof(int32_t) * (size_t)max_slots) != hipSuccess ||
        pin_base.ensure(sizeof(int64_t) * (size_t)U.max_batches) != hipSuccess)
        return fail(GC_ENOMEM, "pinned host buffers");
    UnionCall c;
    c.gu = &gu;
    c.w = &wu;
    c.jobs = &jobs;
    c.d_bbase = reinterpret_cast<int64_t *>(ub + U.bbase);
    c.d_src = reinterpret_cast<int32_t *>(ub + U.src);
    c.d_gain = reinterpret_cast<int64_t *>(ub + U.gout);
    c.max_batches = U.max_batches;
    c.d_dist = udist;
    c.dist_bytes = dist_bytes;
    c.nlev = nlev;
    c.split = &usplit;
    c.s = s0;
    c.pin_src = &pin_src;
    c.pin_base = &pin_base;
    const bool celf = o.order == GC_ORDER_CELF;
    // The jobs' selection work (the lazy rule, the stale-gain trees) runs on
    // `nt` host threads, each owning the jobs i = tid (mod nt); thread 0 also
    // issues the shared gain and update calls.  Four barriers per step.
    const int32_t nt = std::max<int32_t>(1, std::min<int32_t>(nworkers, count));
    struct Barrier {
        std::atomic<int32_t> arrived{0}, gen{0};
        int32_t n = 1;
        void wait() {
            const int32_t g = gen.load(std::memory_order_acquire);
            if (arrived.fetch_add(1, std::memory_order_acq_rel) == n - 1) {
                arrived.store(0, std::memory_order_relaxed);
                gen.fetch_add(1, std::memory_order_acq_rel);
            } else {
                while (gen.load(std::memory_order_acquire) == g) std::this_thread::yield();
            }
        }
    } bar;
    bar.n = nt;
    std::vector<std::pair<int32_t, std::vector<int32_t>>> lists, picks;
    std::vector<int64_t> gain, edges, pgain, pedges;
    std::vector<int64_t> list_off((size_t)count, -1), pick_off((size_t)count, -1);
    std::vector<int32_t> job_rc((size_t)count, GC_OK);
    std::vector<std::string> job_msg((size_t)count);
    std::atomic<bool> stop{false};
    int call_rc = GC_OK;
    std::string call_msg;
    const bool verbose = getenv("GC_VERBOSE") != nullptr;
    const double t_loop = now_ms();
    double ms_gain_calls = 0, ms_update_calls = 0;
    int64_t steps = 0, gain_calls = 0, update_calls = 0, sources = 0;
    auto gather = [&](int32_t i) {
        BatchJob &J = jobs[(size_t)i];
        J.batch.clear();
        if ((int32_t)J.group.size() >= J.k || job_rc[(size_t)i] != GC_OK) return;
        const int32_t n = J.g->n;
        if (!J.in_round) {
            J.in_round = true;
            J.pos = 0;
            J.bid = -1;
            J.bgain = -1;
            J.nev = 0;
            J.cur = std::min<int64_t>(block, std::min<int64_t>(16LL * block, n));
        }
        if (celf) {
            while ((int64_t)J.batch.size() < J.cur) {
                const int32_t v = J.keys.top();
                if (v < 0) break;
                const int64_t u = J.ub[(size_t)v];
                // stop unless (u, -v) beats (bgain, -bid)
                if (J.bid >= 0 && (u < J.bgain || (u == J.bgain && v >= J.bid))) break;
                J.batch.push_back(v);
                J.keys.set(v, -1);
            }
        } else {
            J.tree.collect(J.pos, J.bid < 0 ? 0 : J.bgain + 1, J.cur, J.batch);
            if (!J.batch.empty()) J.pos = J.batch.back() + 1;
        }
        if (J.batch.empty() && J.bid < 0) {
            job_rc[(size_t)i] = GC_EDEVICE;
            job_msg[(size_t)i] = "no candidate left";
        }
    };
    auto distribute = [&](int32_t i) {
        BatchJob &J = jobs[(size_t)i];
        const int64_t o0 = list_off[(size_t)i];
        if (o0 < 0) return;
        for (size_t q = 0; q < J.batch.size(); ++q) {
            const int32_t v = J.batch[q];
            const int64_t gv = gain[(size_t)o0 + q];
            if (gv > J.ub[(size_t)v] && job_rc[(size_t)i] == GC_OK) {
                job_rc[(size_t)i] = GC_EDEVICE;
                job_msg[(size_t)i] = "a gain grew between rounds (supermodularity)";
            }
            J.ub[(size_t)v] = gv;
            if (celf) J.keys.set(v, gv);
            else J.tree.set(v, gv);
            J.st.edges_alg += edges[(size_t)o0 + q];
            if (gv > J.bgain || (gv == J.bgain && v < J.bid)) {
                J.bgain = gv;
                J.bid = v;
            }
        }
        J.nev += (int64_t)J.batch.size();
        J.st.gain_launches += 1;
        J.cur = std::min<int64_t>(J.cur * growth, std::min<int64_t>(16LL * block, J.g->n));
    };
    auto apply_pick = [&](int32_t i) {
        BatchJob &J = jobs[(size_t)i];
        const int64_t o0 = pick_off[(size_t)i];
        if (o0 < 0) return;
        if (pgain[(size_t)o0] != J.bgain && job_rc[(size_t)i] == GC_OK) {
            job_rc[(size_t)i] = GC_EDEVICE;
            job_msg[(size_t)i] = "the update's gain differs from the evaluated gain";
        }
        const int32_t r = (int32_t)J.group.size();
        J.group.push_back(J.bid);
        J.F.push_back(J.F.back() - J.bgain);
        J.inS[(size_t)J.bid] = 1;
        J.ub[(size_t)J.bid] = -1;
        if (celf) J.keys.set(J.bid, -1);
        else J.tree.set(J.bid, -1);
        J.evals[(size_t)r] = J.nev;
        J.st.evals_later += J.nev;
        J.in_round = false;
    };
    auto phase2 = [&](int32_t tid) {
        // (only thread 0 touches the device; the others work on host data)
        for (;;) {
            for (int32_t i = tid; i < count; i += nt) gather(i);
            bar.wait();
            if (tid == 0) {
                ++steps;
                lists.clear();
                picks.clear();
                std::fill(list_off.begin(), list_off.end(), -1);
                std::fill(pick_off.begin(), pick_off.end(), -1);
                int64_t lo = 0, po = 0;
                for (int32_t i = 0; i < count; ++i) {
                    BatchJob &J = jobs[(size_t)i];
                    if ((int32_t)J.group.size() >= J.k || job_rc[(size_t)i] != GC_OK) continue;
                    if (J.batch.empty()) {
                        pick_off[(size_t)i] = po++;
                        picks.push_back({i, std::vector<int32_t>{J.nb + J.bid}});
                    } else {
                        list_off[(size_t)i] = lo;
                        lo += (int64_t)J.batch.size();
                        std::vector<int32_t> ids(J.batch.size());
                        for (size_t q = 0; q < ids.size(); ++q) ids[q] = J.nb + J.batch[q];
                        lists.push_back({i, std::move(ids)});
                    }
                }
                if (lists.empty() && picks.empty()) {
                    stop = true;
                } else if (!lists.empty()) {
                    const double tc = now_ms();
                    const int r = union_call(c, lists, false, gain, edges);
                    ms_gain_calls += now_ms() - tc;
                    ++gain_calls;
                    sources += (int64_t)gain.size();
                    if (r) {
                        call_rc = r;
                        call_msg = g_last_error;
                        stop = true;
                    }
                }
            }
            bar.wait();
            if (stop) break;
            for (int32_t i = tid; i < count; i += nt) distribute(i);
            bar.wait();
            if (tid == 0 && !picks.empty()) {
                const double tc = now_ms();
                const int r = union_call(c, picks, true, pgain, pedges);
                ms_update_calls += now_ms() - tc;
                ++update_calls;
                if (r) {
                    call_rc = r;
                    call_msg = g_last_error;
                    stop = true;
                }
            }
            bar.wait();
            if (stop) break;
            for (int32_t i = tid; i < count; i += nt) apply_pick(i);
        }
    };
    {
        std::vector<std::thread> th;
        th.reserve((size_t)nt);
        for (int32_t tid = 1; tid < nt; ++tid) th.emplace_back(phase2, tid);
        phase2(0);
        for (auto &t : th) t.join();
    }
    if (call_rc) return fail(call_rc, "%s", call_msg.c_str());
    for (int32_t i = 0; i < count; ++i)
        if (job_rc[(size_t)i] != GC_OK) return fail(job_rc[(size_t)i], "job %d: %s", i, job_msg[(size_t)i].c_str());
    const double ms_phase2 = now_ms() - t2;
    if (verbose) {
        fprintf(stderr,
                "[gc] batch: phase 1 %.1f ms; phase 2 %.1f ms (setup %.1f, %lld steps: %lld gain calls %.1f ms "
                "over %lld sources, %lld update calls %.1f ms, %lld launches)\n",
                ms_phase1, ms_phase2, t_loop - t2, (long long)steps, (long long)gain_calls, ms_gain_calls,
                (long long)sources, (long long)update_calls, ms_update_calls, (long long)c.launches);
        fflush(stderr);
    }
    for (int32_t i = 0; i < count; ++i) {
        BatchJob &J = jobs[(size_t)i];
        for (int32_t q = 0; q < J.k; ++q) {
            h_group[off[(size_t)i] + q] = J.group[(size_t)q];
            h_farness[off[(size_t)i] + q] = J.F[(size_t)q];
        }
        if (h_stats) {
            gc_stats st = J.st;
            st.evals_total = st.evals_round1 + st.evals_later;
            st.dist_bytes = dist_bytes;
            st.ms_later = ms_phase2;           // shared by every job
            st.ms_total = now_ms() - t_start;  // the whole batch
            st.h_evals_per_round = nullptr;
            (void)ms_phase1;
            h_stats[i] = st;
        }
    }
    return GC_OK;
}

extern "C" int gc_node_features(const gc_graph *g, const void *d_dist, int32_t dist_bytes,
                                const int32_t *d_cand, int32_t count, const int64_t *d_ub,
                                const int32_t *d_last_eval, const uint16_t *d_dist_at_eval,
                                int32_t round, int32_t k, int32_t ecc1, float *d_feat,
                                hipStream_t stream) {
    if (int rc0 = unweighted_only(g, "gc_node_features")) return rc0;
    if (!g) return fail(GC_EINVAL, "graph is NULL");
    if (dist_bytes != 1 && dist_bytes != 2) return fail(GC_EINVAL, "dist_bytes must be 1 or 2");
    if (count < 0) return fail(GC_EINVAL, "count < 0");
    if (count > 0 && (!d_dist || !d_ub || !d_last_eval || !d_dist_at_eval || !d_feat))
        return fail(GC_EINVAL, "NULL device pointer");
    FeatArgs fa{};
    fa.rp = g->d_rp;
    fa.ci = g->d_ci;
    fa.dist = d_dist;
    fa.cand = d_cand;
    fa.count = count;
    fa.ub = d_ub;
    fa.last_eval = d_last_eval;
    fa.dist_at_eval = d_dist_at_eval;
    fa.round = round;
    fa.k = k;
    fa.ecc1 = ecc1;
    fa.feat = d_feat;
    HIP_OK(launch_features(fa, dist_bytes, stream));
    return GC_OK;
}
