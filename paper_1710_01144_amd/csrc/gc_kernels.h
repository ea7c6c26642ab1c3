// Internal interface between the host driver (gc_api.cpp) and the HIP
// kernels (gc_kernels.hip).  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gck {

constexpr int kWG = 256;      // threads per workgroup of the bit-parallel engine
constexpr int kSrc = 64;      // sources per bitset word

// Workspace counters (int32 slots of the counter block).
enum : int {
    C_BFS_CNT0 = 2,    // three rotating frontier counters of the level BFS
    C_BFS_LAST = 5,    // deepest level that claimed a node
    C_BFS_CLAIMED = 6, // nodes claimed by the current level BFS
    C_I64_BASE = 8,    // int64 area starts at int32 slot 8
};
// int64 slots (index into the int64 view starting at int32 slot 8)
enum : int {
    L_BFS_SUM = 0,     // sum of contributions of the level BFS
    L_BEST_FAR = 1,    // best farness found by the closeness search
    // word-level work of the device-wide engine, summed over gain launches:
    // frontier entries (all levels, root level, last level), adjacency entries
    // of expanded levels / of the last level, and (batch, node) records touched
    L_WORDS = 64,
    kWordCounters = 6,
    L_TOUCHED = 72,    // records touched by the current launch (clean-up list length)
    L_CUTS = 73,       // sources stopped by the early exit (k_gain_cut), summed over launches
    L_HDR = 80,        // stamp of gc_workspace_init: graph-derived tables are valid
};

struct BfsArgs {
    const int32_t *rp;
    const int32_t *ci;
    int32_t n;
    void *dist;              // uint8/uint16 (or int32 when dist_bytes == 4)
    int32_t *q0;
    int32_t *q1;
    uint32_t *claim;         // ceil(n/32) words
    int32_t *ctr;
    int32_t full;            // 1: S = {} (sum levels), 0: sum (old - level)
};
// init: clears claim bitmap and counters, claims the root (level 0).
hipError_t launch_bfs_init(const BfsArgs &a, int dist_bytes, int32_t root, hipStream_t s);
// one level: frontier at distance `level` -> distance level+1.
hipError_t launch_bfs_level(const BfsArgs &a, int dist_bytes, int32_t level, int grid,
                            hipStream_t s);
// F_out = full ? sum : F_in - sum
hipError_t launch_bfs_finish(const BfsArgs &a, int64_t *d_far, hipStream_t s);

// ------------------------------------------------ device-wide gain engine
// a level record packs its entry count above bit kCntShift and the adjacency
// entries its entries expand below it
constexpr int kCntShift = 36;
struct WideLevel {
    int64_t start;                 // first log index of this level's entries
    unsigned long long packed;     // (entry count << kCntShift) | adjacency entries to expand
};

struct WideArgs {
    const int32_t *rp;
    const int32_t *ci;
    int32_t n;
    const void *dist;              // uint8/uint16 d(S,.)
    const int32_t *src;            // candidates of this launch, spb per batch
    int64_t nsrc;
    int32_t spb;                   // sources per batch (bits used per word), 1..64
    int64_t *gain;                 // out [nsrc]
    int64_t *edges;                // out [nsrc] or null
    int32_t *visited;              // out [nsrc] or null
    uint64_t *vis;                 // batch b, node y: 4 words at (b*vis_stride + y)*4, zero between launches
    size_t vis_stride;
    // or, when set, at (bbase[b] + y)*4: a batch whose sources all lie in one
    // component of a disjoint union gets records for that component's nodes
    // only (bbase[b] = its first record minus the component's first node id)
    const int64_t *bbase;
    int32_t *ly;                   // frontier log: node
    int32_t *lr;                   //               row start of the node
    int32_t *lb;                   //               batch
    int64_t *lo;                   //               first adjacency position (per level)
    int64_t cap;                   // log capacity (entries, a power of two: a ring)
    // clean-up list: every (batch << 32 | node) record the launch touches, named
    // once by the claim that finds its visited word empty
    int64_t *lz;
    int64_t zcap;                  // capacity of lz (entries)
    unsigned long long *zcnt;      // entries in lz (zero between launches)
    WideLevel *lvl;                // per-level records, nlev + 2 of them
    int32_t *flags;                // [0]: nonzero after an overflow (value = tag)
    int32_t tag;
    int32_t min_edges;             // adjacency entries per workgroup before a level
                                   // uses more workgroups (small levels stay compact)
    // optional host-mapped destinations written by the final kernel
    int64_t *h_gain;
    int64_t *h_edges;
    int32_t *h_flag;
    int64_t *h_done;               // optional host-mapped word: = seq once everything is written
    int64_t seq;
    // optional: the reset copies *maxd_src (a device value written before the
    // launch) to the host-mapped *h_maxd ahead of the done word
    const int32_t *maxd_src;
    int32_t *h_maxd;
    // d(S,.) update mode: one source (the pick), distances written in place,
    // *far -= its gain at the end
    bool write;
    int64_t *far;
    int32_t root;                  // source when src is null (nsrc = 1)
    // optional scatter of the results into per-node lazy-loop state
    int64_t *ub_out;               // ub[src[i]] = gain[i]
    int32_t *le_out;               // last_eval[src[i]] = round
    uint16_t *dsat_out;            // dist_at_eval[src[i]] = d(S, src[i])
    int32_t round;
    int32_t dist_bytes;
    int32_t unroll;                // 4 or 8 edges per thread per step (large launches)
    // closeness search (first pick): per-batch masks of sources still expanding,
    // per-source previous (reached, adjacency) totals, farness or -1 (cut)
    unsigned long long *active;
    int64_t *prev;                 // 2 x nsrc
    int64_t *far_out;              // nsrc
    int64_t *words;                // optional: kWordCounters totals, added to at the end
    // optional row split by d1 = the d(S,.) it was built from, which bounds
    // d(S,.) from above for the rest of the run: ci rows ordered
    // [d1 > d1(y) | d1 == d1(y) | d1 < d1(y)] for the row's node y, and
    // rinfo[y] = {row start, degree, #first segment, #first two segments}
    const int4 *rinfo;
    const void *dist1;             // d1, same width as dist
    // gain and edge count of a source summed in one 64-bit word during the
    // launch, (gain << kPackShift) + edges, unpacked by the final kernel; the
    // host sets it only when edges < 2^kPackShift and the gain cannot reach
    // 2^(63 - kPackShift).  2: the same, and a launch of more than kLdsSrc
    // sources first sums each window's batches in LDS slots, which cuts the
    // global atomics when many launches share the chip (the multi-job engines)
    int32_t pack;
    // early exit inside the candidates' BFS (gain launches with `active`):
    // cut_gain selects it; the bound's tail table T (cut_maxd + 2 entries),
    // max d(S,.), and the launch's threshold (cut_thr, cut_id)
    int32_t cut_gain;
    int32_t cut_maxd;
    const int64_t *cut_T;
    int64_t cut_thr;
    int32_t cut_id;
    unsigned long long *cut_count; // sources stopped, added to
    int32_t directed;              // rows are out-neighbour lists of a directed graph
    // launches started by launch_wide_first: level 0's packed sums per source
    // (zero between launches; the final kernel adds them to gain and clears them)
    unsigned long long *acc;
};
constexpr int kPackShift = 30;
// most sources of a launch started by launch_wide_first
constexpr int64_t kFirstMaxSrc = 1024;
// the first kFirstArgIds candidates of such a launch may come as a kernel
// argument (read from the argument segment instead of WideArgs::src)
constexpr int kFirstArgIds = 256;
struct FirstIds {
    int32_t id[kFirstArgIds];
};
// Split every row of (rp, ci) by the distances dist (see WideArgs::rinfo);
// dist1 receives a copy of dist.  Rows of more than kSplitLongRow entries
// may be listed in `chunks` (nchunks pairs {row, index of the row's first
// pair}, one pair per kSplitChunk entries of the row, rows ascending): a
// workgroup then splits each chunk, with `cnt` (2 * nchunks ints) holding the
// chunks' part sizes between its two passes; without a list (chunks null)
// one wave splits each row, however long.
constexpr int32_t kSplitLongRow = 1024;
constexpr int32_t kSplitChunk = 2048;
hipError_t launch_row_split(const int32_t *rp, const int32_t *ci, int32_t n, const void *dist,
                            int dist_bytes, int32_t *ci_out, int4 *rinfo, void *dist1,
                            const int32_t *chunks, int32_t nchunks, int32_t *cnt, hipStream_t s);
// After level L: BFScut test for every live source of a closeness launch
// (distances from an all-INF 16-bit array, so F = reached*65535 - gain).
hipError_t launch_wide_cut(const WideArgs &a, int32_t L, int64_t *best, bool fixed, hipStream_t s);
// After level l of a gain launch with the early exit: test every live source
// (see k_gain_cut in gc_wide.hip).
hipError_t launch_gain_cut(const WideArgs &a, int32_t l, hipStream_t s);
// T[j] = sum_w max(0, d(S,w) - j - 1), j = 0..maxd (T[maxd + 1] = 0);
// hist: maxd + 2 scratch words.
hipError_t launch_tail_table(const void *dist, int dist_bytes, int64_t n, int32_t maxd,
                             unsigned long long *hist, int64_t *T, hipStream_t s);
hipError_t launch_twohop_i64(const int32_t *rp, const int32_t *ci, int32_t n, int64_t *out,
                             hipStream_t s);
// bound[i] = level-1 farness bound of node order[i]; keep[i] = 1 if it may
// beat (best_f, best_v) (i >= 1), else 0
hipError_t launch_lb1_filter(const int32_t *order, const int32_t *rp, const int64_t *two, int32_t n,
                             int64_t best_f, int32_t best_v, uint8_t *keep, int64_t *bound, bool directed,
                             hipStream_t s);
// out[j] = src[idx[j]]
hipError_t launch_gather_i64(const int64_t *src, const int32_t *idx, int32_t cnt, int64_t *out,
                             hipStream_t s);
hipError_t launch_wide_begin(const WideArgs &a, int dist_bytes, int32_t nlev, hipStream_t s);
// Roots and level 0 of a gain launch in one kernel, in place of
// launch_wide_begin and level 0 (the level kernels then start at level 1):
// at most kFirstMaxSrc sources, packed sums (pack != 0) with acc set, no
// per-source visited counts, active masks, early exit or write-back.  ids
// holds a.src[0 .. nids) (nids <= kFirstArgIds; 0: none); grid may be cut to
// the workgroups the level-0 adjacency entries can need plus one per 256
// sources (the roots are claimed from the last workgroup down).  A launch of
// more than kFirstMaxSrc sources raises the overflow flag and does nothing.
hipError_t launch_wide_first(const WideArgs &a, int dist_bytes, int grid, const FirstIds &ids, int32_t nids,
                             hipStream_t s);
hipError_t launch_wide_levels(const WideArgs &a, int dist_bytes, int32_t l0, int32_t l1, int grid,
                              hipStream_t s);
hipError_t launch_wide_end(const WideArgs &a, int32_t nlev, int grid, hipStream_t s);
// *out = max_i dist[i] (device int32), for the level bound of pruned BFS
hipError_t launch_max_dist(const void *dist, int dist_bytes, int64_t n, int32_t *out, hipStream_t s);

hipError_t launch_fill_u32(uint32_t *p, size_t count, uint32_t v, hipStream_t s);
hipError_t launch_u16_to_u8(const uint16_t *in, uint8_t *out, int64_t n, hipStream_t s);
// uint8 distances to uint16 (INF 255 -> 65535)
hipError_t launch_u8_to_u16(const uint8_t *in, uint16_t *out, int64_t n, hipStream_t s);
// out[i] = in[i] + add (building the disjoint union of several CSRs)
hipError_t launch_copy_add_i32(const int32_t *in, int32_t *out, int64_t n, int32_t add, hipStream_t s);
hipError_t launch_set_i64(int64_t *p, int64_t v, hipStream_t s);

}  // namespace gck
