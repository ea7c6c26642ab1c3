// Internal interface between the host driver (gc_api.cpp) and the weighted
// search kernels (gc_weighted.hip).  Not part of the public C ABI.
//
// On a graph with integer edge lengths 1..255 every distance query of the
// method is an SSSP (Section 2), and the pruning of Section 4.1 applies to it
// unchanged: a search from u enters a node y only while d(u,y) < d(S,y).
// Each search here runs inside one workgroup: a bucketed label-correcting
// search (delta-stepping) over the workgroup's own slot of per-node records
// and work lists, so thousands of candidates are searched at once with no
// grid-wide synchronisation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gck {

// Per-node state of one slot (zero = untouched), in two arrays: the word
// every relaxation reads, 4 bytes per node,
//   enc    0x7FFFFFFF - tentative distance (atomicMax lowers the distance),
// and the bookkeeping of the nodes whose distance dropped, 16 bytes:
//   mark   stamp of the last near-list iteration the node was queued for
//   far    1 once the node has been put on the far list
//   phase  stamp of the phase in which the node was settled (closeness mode)
struct WRec {
    uint32_t mark;
    uint32_t far;
    uint32_t phase;
    uint32_t pad;
};
// Work lists of one slot: near (current, next), far (current, next), the
// touched list (every node whose record the search changed, once) and the
// nodes settled in the current phase; each n entries.
constexpr int kWLists = 6;
constexpr size_t kWSlotBytesPerNode = 4 + sizeof(WRec) + kWLists * sizeof(int32_t);  // 44

enum WMode : int32_t {
    W_GAIN = 0,   // g(u,S) = sum over settled y of d(S,y) - d(u,y), search pruned by d(S,.)
    W_CLOSE = 1,  // F({u}) = sum_y d(u,y), no pruning, cut by the lower bound of the closeness search
    W_WRITE = 2,  // W_GAIN for one source, then d(S,y) <- d(u,y) for every settled y
};

struct WArgs {
    const int32_t *rp;
    const int32_t *ci;
    const uint8_t *w;
    int32_t n;
    int32_t mode;
    int32_t *dS;            // d(S,.) (int32, INT32_MAX = no member reaches it); W_CLOSE: unused
    const int32_t *cand;    // candidate ids (count entries; ids outside [0, n) get 0 / -1)
    int32_t count;
    uint32_t *next;         // work counter, zero at launch
    int64_t *out;           // W_GAIN / W_WRITE: gain; W_CLOSE: F({u}) or -1 when cut
    int64_t *edges;         // optional: sum of degrees over the settled nodes
    int32_t *visited;       // optional: settled nodes
    uint32_t *enc;          // slots x n distance words
    WRec *rec;              // slots x n records
    int32_t *lists;         // slots x kWLists x n entries
    int32_t delta;          // bucket width
    int64_t thr;            // W_CLOSE: cut once the bound exceeds min(thr, *best)
    unsigned long long *best;  // W_CLOSE: best F so far (atomicMin), or nullptr
    const int32_t *d0;      // W_CLOSE: distances from a landmark node, or nullptr
    const int64_t *t0;      // W_CLOSE: t0[M] = sum_w max(0, d0(w) - M), M < t0_len
    int32_t t0_len;         //          (t0[t0_len - 1] = 0), or nullptr
    int32_t *flags;         // bit 0: a closeness search did not reach every node;
                            // bit 1: a search passed max_rounds (and was abandoned)
    uint32_t max_rounds;    // watchdog: near-list rounds per search (0: no limit)
};

// count candidates over `slots` slots (at most `slots` workgroups of
// `threads` threads, 256 or 1024, each taking candidates from the work
// counter until none is left)
hipError_t launch_wsearch(const WArgs &a, int32_t slots, int32_t threads, hipStream_t s);
// one candidate on slot 0, with a workgroup of 1024 threads (updates, the
// first source of the closeness search)
hipError_t launch_wsearch_one(const WArgs &a, hipStream_t s);
// lexicographic minimum of (out[i], cand[i]) over entries with out[i] >= 0:
// res[0] = F, res[1] = id (-1, -1 if none)
hipError_t launch_wargmin(const int64_t *out, const int32_t *cand, int32_t count, int64_t *res, hipStream_t s);
// *sum = sum of d[0..n) (zeroed first)
hipError_t launch_wsum(const int32_t *d, int32_t n, unsigned long long *sum, hipStream_t s);
// *far -= *gain
hipError_t launch_wsub(int64_t *far, const int64_t *gain, hipStream_t s);
// *mx = max of d[0..n) (d >= 0); *mx must be 0 on entry
hipError_t launch_wmax(const int32_t *d, int32_t n, int32_t *mx, hipStream_t s);
// hist[d[i]] += 1 for every i (hist zeroed by the caller, entries > max(d))
hipError_t launch_whist(const int32_t *d, int32_t n, uint32_t *hist, hipStream_t s);

}  // namespace gck
