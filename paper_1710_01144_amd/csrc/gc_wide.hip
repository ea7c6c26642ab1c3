// Device-wide bit-parallel pruned BFS for marginal gains (gfx950).
//
// Candidates are grouped up to 64 to a batch (one bit per source).  Batch b
// owns one 32-byte record per node y: the visited word vis (bit j = source j
// has reached y) and three "frontier" words fr[0..2].  All batches of a launch
// advance one BFS level per kernel, so a level is one edge-balanced sweep over
// the whole device.  For a frontier entry (b, x) at distance L with source
// bits F = fr[L % 3] of (b, x), every neighbour y is handled as follows:
//
//   L+1 >= d(S,y)  -> pruned (Section 4.1): neither y nor anything behind it is
//                     closer to these sources than to S; nothing is written.
//   otherwise      -> nw = F & ~vis; one atomicOr on vis returns exactly the
//                     bits this claim adds, each source j in nw gains
//                     d(S,y) - (L+1) (the summand of the gain sum in the proof
//                     of the Section 4.3 theorem); then atomicOr(fr[(L+1)%3],
//                     nw), and the claim that finds that word empty appends
//                     (b, y) to the next frontier.
//
// So settlement is exact per claim, and every (batch, node) enters a level's
// frontier once, carrying the union of the bits that reached it: sources that
// share territory share the expansion (the point of the bit-parallel form).
// A node with nothing left to expand (see expand_len) gets no frontier entry;
// the claim that finds a record's visited word empty names the record in a
// clean-up list, from which the end of the launch zeroes every record touched.
// Level L+1 reads fr[(L+1)%3]; level L+2 writes fr[(L+3)%3] = fr[L%3], which
// level L+1 clears first -- no word is read and written in the same kernel.
//
// Load balance: one 64-bit atomic per workgroup step reserves both the slots
// of new entries and the adjacency positions they will expand
// ((count << kCntShift) | edges), so edge offsets are monotone in the entry index; the
// next level splits its total evenly over the workgroups (a hub's adjacency is
// spread over many of them), each finding its first entry with a 64-ary
// search and walking windows of 256 entries staged in LDS.
//
// A pruned BFS never goes deeper than max_y d(S,y) - 1, so the host launches
// that many levels without reading anything back.
#include "gc_kernels.h"

namespace gck {
namespace {

constexpr int kWin = 256;      // entries staged per window
constexpr int kLdsSrc = 1024;  // launches with at most this many sources sum gains in LDS
constexpr int kBatchSlots = 16; // larger launches: batches of a window summed in LDS
constexpr int64_t kReadFirstEdges = 1 << 20;  // levels beyond this read a visited word before its atomic
constexpr uint64_t kMEdges = (1ull << kCntShift) - 1;

__device__ __forceinline__ int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ int bits_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    const uint32_t lo = __shfl((uint32_t)v, src);
    const uint32_t hi = __shfl((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ void set_flag(int32_t *flag, int32_t v) { atomicCAS(flag, 0, v); }

// word k (0 = visited, 1..3 = frontier of level k-1 mod 3) of (batch b, node y)
// first record of batch b, counted from node 0
__device__ __forceinline__ int64_t batch_base(const WideArgs &a, int64_t b) {
    return a.bbase ? a.bbase[b] : b * (int64_t)a.vis_stride;
}

__device__ __forceinline__ unsigned long long *rec(const WideArgs &a, int64_t b, int64_t y, int k) {
    return reinterpret_cast<unsigned long long *>(a.vis) + (batch_base(a, b) + y) * 4 + k;
}

// The log is a ring of a.cap (a power of two) entries addressed by position
// mod a.cap: positions grow through a launch, and only three levels are live
// at a time (the one being cleared, the one being expanded, the one being
// appended).  An append may not reach a.cap positions past the oldest live
// entry, `live`.
__device__ __forceinline__ void log_entry(const WideArgs &a, int64_t live, int64_t pos, int32_t y,
                                          int32_t rs, int32_t b, int64_t off) {
    if (pos - live < a.cap) {
        const int64_t q = pos & (a.cap - 1);
        a.ly[q] = y;
        a.lr[q] = rs;
        a.lb[q] = b;
        a.lo[q] = off;
    } else {
        set_flag(a.flags, a.tag);
    }
}

// Adjacency entries of y worth expanding when y enters the frontier at level
// lvl.  A neighbour z can be claimed at lvl + 1 only if d(S,z) >= lvl + 2, and
// d(S,z) <= d1(z); along y's split row d1(z) is above, equal to, then below
// d1(y), so the candidates are a prefix of the row.  (A claimed y has
// lvl < d(S,y) <= d1(y), so lvl + 2 <= d1(y) + 1.)
__device__ __forceinline__ int32_t expand_len(const int4 &ri, uint32_t d1, uint32_t lvl) {
    const uint32_t need = lvl + 2;
    if (need < d1) return ri.y;   // any neighbour may qualify
    if (need == d1) return ri.w;  // neighbours with d1(z) >= d1(y)
    return ri.z;                  // neighbours with d1(z) > d1(y)
}

template <typename DistT>
__device__ __forceinline__ uint32_t load_d1(const WideArgs &a, int32_t y) {
    return reinterpret_cast<const DistT *>(a.dist1)[y];
}

// Wave-level append (every lane of a fully active wave calls it).
__device__ __forceinline__ void push_wave(const WideArgs &a, WideLevel *nl, int64_t nbase, int64_t live,
                                          bool p, int32_t y, int32_t rs, int32_t b, int32_t deg) {
    const uint64_t bal = __ballot(p);
    if (bal == 0) return;
    const int lane = lane_id();
    const int dp = p ? deg : 0;
    int incl = dp;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    const int total = __shfl(incl, 63);
    uint64_t old = 0;
    if (lane == 0) {
        old = atomicAdd(&nl->packed, ((unsigned long long)__popcll(bal) << kCntShift) + (unsigned long long)total);
        if ((old & kMEdges) + (uint64_t)total >= (1ull << (kCntShift - 1)) ||
            (old >> kCntShift) + 64 >= (1ull << (63 - kCntShift)))
            set_flag(a.flags, a.tag);
    }
    old = shfl64(old, 0);
    if (!p) return;
    log_entry(a, live, nbase + (int64_t)(old >> kCntShift) + bits_below(bal), y, rs, b,
              (int64_t)(old & kMEdges) + (incl - dp));
}

// Work-group append: thread t holds up to U new entries (p[r]); one 64-bit
// atomic reserves the slots and adjacency ranges of all of them.
template <int U>
__device__ __forceinline__ void push_block(const WideArgs &a, WideLevel *nl, int64_t nbase,
                                           int64_t live, const bool *p, const int32_t *y, const int32_t *rs,
                                           const int32_t *bb, const int32_t *deg, int64_t *s_wc,
                                           int64_t *s_wd, uint64_t *s_old) {
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    int64_t c = 0, dsum = 0;
#pragma unroll
    for (int r = 0; r < U; ++r)
        if (p[r]) {
            c += 1;
            dsum += deg[r];
        }
    int64_t ic = c, id = dsum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t tc = __shfl_up(ic, o);
        const int64_t td = __shfl_up(id, o);
        if (lane >= o) {
            ic += tc;
            id += td;
        }
    }
    if (lane == 63) {
        s_wc[w] = ic;
        s_wd[w] = id;
    }
    __syncthreads();
    int64_t pc = 0, pd = 0, tc = 0, td = 0;
#pragma unroll
    for (int k = 0; k < kWG / 64; ++k) {
        if (k < w) {
            pc += s_wc[k];
            pd += s_wd[k];
        }
        tc += s_wc[k];
        td += s_wd[k];
    }
    if (threadIdx.x == 0) {
        uint64_t old = 0;
        if (tc > 0) {
            old = atomicAdd(&nl->packed, ((unsigned long long)tc << kCntShift) + (unsigned long long)td);
            if ((old & kMEdges) + (uint64_t)td >= (1ull << (kCntShift - 1)) ||
                (old >> kCntShift) + (uint64_t)tc >= (1ull << (63 - kCntShift)))
                set_flag(a.flags, a.tag);
        }
        *s_old = old;
    }
    __syncthreads();
    if (tc == 0) return;
    const uint64_t old = *s_old;
    int64_t idx = (int64_t)(old >> kCntShift) + pc + (ic - c);
    int64_t off = (int64_t)(old & kMEdges) + pd + (id - dsum);
#pragma unroll
    for (int r = 0; r < U; ++r) {
        if (!p[r]) continue;
        log_entry(a, live, nbase + idx, y[r], rs[r], bb[r], off);
        idx += 1;
        off += deg[r];
    }
}

__device__ __forceinline__ void touch_entry(const WideArgs &a, int64_t pos, int32_t b, int32_t y) {
    if (pos < a.zcap) a.lz[pos] = ((int64_t)b << 32) | (uint32_t)y;
    else set_flag(a.flags, a.tag);
}

// Wave-level append of touched records: thread t names up to U of them (t[r]).
template <int U>
__device__ __forceinline__ void touch_wave(const WideArgs &a, const bool *t, const int32_t *bb,
                                           const int32_t *y) {
    int c = 0;
#pragma unroll
    for (int r = 0; r < U; ++r) c += t[r] ? 1 : 0;
    if (__ballot(c > 0) == 0) return;
    const int lane = lane_id();
    int incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    const int total = __shfl(incl, 63);
    unsigned long long old = 0;
    if (lane == 0) old = atomicAdd(a.zcnt, (unsigned long long)total);
    old = shfl64(old, 0);
    int64_t pos = (int64_t)old + (incl - c);
#pragma unroll
    for (int r = 0; r < U; ++r)
        if (t[r]) touch_entry(a, pos++, bb[r], y[r]);
}

// Level 0: every source claims its own node (weight d(S,v) - 0).
// WRITE: the d(S,.) update after a pick -- a claimed node also stores its new
// distance (in place: a later prune test against it fails, and the visited
// bit settles concurrent claims); the single source's gain is F(S) - F(S+s).
// Thread t of the launch (wave-uniform calls: the log append is a wave op).
template <typename DistT, bool WRITE>
__device__ __forceinline__ void roots_body(const WideArgs &a, int64_t t) {
    if (__hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    DistT *dist = reinterpret_cast<DistT *>(const_cast<void *>(a.dist));
    bool p = false, touched = false;
    int32_t v = 0, b = 0, deg = 0, rs = 0;
    if (t < a.nsrc) {
        v = a.src ? a.src[t] : a.root;
        b = (int32_t)(t / a.spb);
        const int64_t j = t - (int64_t)b * a.spb;
        a.gain[t] = 0;
        if (a.edges) a.edges[t] = 0;
        if (a.visited) a.visited[t] = 0;
        if (a.active) {
            a.far_out[t] = -1;
            // closeness: the root itself and its adjacency; gains with the
            // early exit: nothing yet (the test after level 0 counts the root)
            const bool base = !a.cut_gain && (uint32_t)v < (uint32_t)a.n;
            a.prev[2 * t] = base ? 1 : 0;
            a.prev[2 * t + 1] = base ? a.rp[v + 1] - a.rp[v] : 0;
            if (j == 0) {
                const int64_t left = a.nsrc - (int64_t)b * a.spb;
                const int64_t nb = left < a.spb ? left : a.spb;
                a.active[b] = nb >= 64 ? ~0ull : ((1ull << nb) - 1ull);
            }
        }
        // an id outside [0, n) touches nothing and gets gain 0
        const uint32_t d = (uint32_t)v < (uint32_t)a.n ? (uint32_t)dist[v] : 0u;
        if (d > 0u) {
            const uint64_t bit = 1ull << j;
            const uint64_t old = atomicOr(rec(a, b, v, 0), (unsigned long long)bit);
            touched = old == 0ull;
            if (bit & ~old) {
                if (WRITE) dist[v] = 0;
                int32_t full;
                if (a.rinfo) {
                    const int4 ri = a.rinfo[v];
                    rs = ri.x;
                    full = ri.y;
                    deg = expand_len(ri, load_d1<DistT>(a, v), 0u);
                } else {
                    rs = a.rp[v];
                    full = a.rp[v + 1] - rs;
                    deg = full;
                }
                if (a.pack) {
                    a.gain[t] = ((int64_t)d << kPackShift) + full;
                } else {
                    a.gain[t] = (int64_t)d;
                    if (a.edges) a.edges[t] = full;
                }
                if (a.visited) a.visited[t] = 1;
                // nothing to expand: no frontier word, no entry
                p = deg > 0 && atomicOr(rec(a, b, v, 1), (unsigned long long)bit) == 0ull;
            }
        }
    }
    touch_wave<1>(a, &touched, &b, &v);
    push_wave(a, &a.lvl[0], 0, 0, p, v, rs, b, deg);
}

template <typename DistT, bool WRITE>
__global__ __launch_bounds__(256) void k_wide_roots(WideArgs a) {
    roots_body<DistT, WRITE>(a, blockIdx.x * (int64_t)blockDim.x + threadIdx.x);
}

// One BFS level.  LDS: per-source sums in LDS (launches of <= kLdsSrc
// sources); large launches add to global memory, straight or (SLOTS) through
// per-window LDS slots of the window's batches.  U: edges per thread per step.
template <typename DistT, bool WRITE, bool LDS, int U, bool SLOTS>
__device__ __forceinline__ void level_body(const WideArgs &a, int32_t L) {
    constexpr int kStep = kWG * U;  // adjacency entries per workgroup step
    __shared__ int64_t s_off[kWin + 1];
    __shared__ int32_t s_rs[kWin];
    __shared__ int32_t s_b[kWin];
    __shared__ uint64_t s_m[kWin];
    __shared__ int64_t s_rb[kWin];  // first record of the entry's batch (from node 0)
    __shared__ int16_t s_idx[kStep];  // window entry of each adjacency entry of a step
    __shared__ int32_t s_wmax[kWG / 64];
    __shared__ int64_t s_first;
    __shared__ int64_t s_wc[kWG / 64], s_wd[kWG / 64];
    __shared__ uint64_t s_old;
    __shared__ unsigned long long s_g[LDS ? kLdsSrc : 1];
    __shared__ unsigned long long s_e[LDS ? kLdsSrc : 1];
    __shared__ unsigned int s_v[LDS ? kLdsSrc : 1];
    __shared__ int32_t s_flag;
    // large launches with packed sums in slots (pack == 2): the window's
    // batches get LDS slots of 64 per-source sums, added to global memory once
    // per window instead of once per claimed bit
    constexpr bool kSlotAcc = !LDS && SLOTS;
    __shared__ int32_t s_sb[kSlotAcc ? kBatchSlots : 1];                 // batch of each slot (-1: free)
    __shared__ unsigned long long s_sg[kSlotAcc ? kBatchSlots * 64 : 1];  // packed sums per slot and bit
    __shared__ int8_t s_es[kSlotAcc ? kWin : 1];                         // slot of each window entry (-1: none)

    // another workgroup may raise the overflow flag while this one starts:
    // read it once, so that every wave of the workgroup takes the same exit
    // (the barriers below need all of them)
    // (the level records were written by earlier kernels: load them while
    // the flag is read)
    const WideLevel me = a.lvl[L];
    const int64_t pstart = L >= 1 ? a.lvl[L - 1].start : 0;
    if (threadIdx.x == 0) s_flag = __hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (s_flag) return;
    const bool slot_acc = kSlotAcc && a.pack == 2;  // (uniform)
    const bool read_first = !LDS || (int64_t)(me.packed & kMEdges) > kReadFirstEdges;
    if (slot_acc) {
        for (int q = threadIdx.x; q < kBatchSlots * 64; q += kWG) s_sg[q] = 0ull;
        if (threadIdx.x < kBatchSlots) s_sb[threadIdx.x] = -1;
    }
    const int64_t N = (int64_t)(me.packed >> kCntShift);
    const int64_t E = (int64_t)(me.packed & kMEdges);
    const int64_t start = me.start;
    const int64_t nbase = start + N;
    const int64_t lmask = a.cap - 1;
    // oldest live log entry: the previous level's (cleared by this kernel)
    const int64_t live = L >= 1 ? pstart : start;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) a.lvl[L + 1].start = nbase;
    const int fr_cur = 1 + L % 3, fr_next = 1 + (L + 1) % 3;
    // small levels use few workgroups: each takes at least min_edges entries
    int64_t G = E == 0 ? 0 : (E + a.min_edges - 1) / a.min_edges;
    if (G > (int64_t)gridDim.x) G = gridDim.x;
    // Clear the frontier words of level L-1 (read by the previous kernel; the
    // next kernel writes this slot again).  The workgroups without expansion
    // work do it, off the others' path; if every workgroup expands, each
    // clears its share after its expansion.
    auto clear_prev = [&](int64_t w, int64_t nw) {
        const int fr_prev = 1 + (L + 2) % 3;
        for (int64_t q = pstart + w * kWG + tid; q < start; q += nw * kWG) {
            const int64_t m = q & lmask;
            *rec(a, a.lb[m], a.ly[m], fr_prev) = 0ull;
        }
    };
    if ((int64_t)blockIdx.x >= G) {
        if (L >= 1) clear_prev((int64_t)blockIdx.x - G, (int64_t)gridDim.x - G);
        return;
    }
    const int64_t eb = E * (int64_t)blockIdx.x / G;
    const int64_t ee = E * ((int64_t)blockIdx.x + 1) / G;
    if (eb >= ee) {
        if (L >= 1 && G == (int64_t)gridDim.x) clear_prev(blockIdx.x, gridDim.x);
        return;
    }

    DistT *dist = reinterpret_cast<DistT *>(const_cast<void *>(a.dist));
    const int32_t *__restrict__ rp = a.rp;
    const int32_t *__restrict__ ci = a.ci;
    const uint32_t nl = (uint32_t)L + 1u;
    WideLevel *next = &a.lvl[L + 1];
    constexpr bool lds_acc = LDS;
    if (lds_acc) {
        for (int q = tid; q < a.nsrc; q += kWG) {
            s_g[q] = 0;
            s_e[q] = 0;
            s_v[q] = 0;
        }
    }

    // largest entry index i with off[i] <= eb (64-ary search by wave 0);
    // the first workgroup starts at entry 0
    if (blockIdx.x == 0) {
        if (tid == 0) s_first = 0;
    } else if (tid < 64) {
        int64_t lo = 0, hi = N - 1;
        while (lo < hi) {
            const int64_t p = lo + ((hi - lo) * tid) / 63;
            const bool pr = a.lo[(start + p) & lmask] <= eb;
            const uint64_t bal = __ballot(pr);
            const int last = 63 - __clzll((long long)bal);  // lane 0 always true
            const int64_t plast = lo + ((hi - lo) * last) / 63;
            const int64_t pnext = (last == 63) ? hi + 1 : lo + ((hi - lo) * (last + 1)) / 63;
            lo = plast;
            hi = pnext - 1;
        }
        if (tid == 0) s_first = lo;
    }
    __syncthreads();
    int64_t i = s_first;

    for (;;) {
        const int64_t cnt64 = N - i < kWin ? N - i : kWin;
        const int cnt = (int)cnt64;
        if (tid < cnt) {
            const int64_t q = (start + i + tid) & lmask;
            const int32_t b = a.lb[q];
            const int64_t off = a.lo[q];
            s_off[tid] = off;
            s_rs[tid] = a.lr[q];
            s_b[tid] = b;
            s_rb[tid] = batch_base(a, b);
            if (slot_acc) {
                // the entry's batch: its slot, a free one, or none (table full)
                int slot = -1;
                for (int k = 0; k < kBatchSlots; ++k) {
                    int cur = s_sb[k];
                    if (cur == -1) cur = atomicCAS(&s_sb[k], -1, b);
                    if (cur == -1 || cur == b) {
                        slot = k;
                        break;
                    }
                }
                s_es[tid] = (int8_t)slot;
            }
            // an entry starting at or past this workgroup's last adjacency
            // entry is never expanded here: skip its frontier word (a random
            // line per entry)
            uint64_t f = 0;
            if (off < ee) {
                f = *rec(a, b, a.ly[q], fr_cur);
                if (a.active) f &= a.active[b];
            }
            s_m[tid] = f;
        }
        if (tid == 0) s_off[cnt] = (i + cnt < N) ? a.lo[(start + i + cnt) & lmask] : E;
        __syncthreads();
        const int64_t wlo = eb > s_off[0] ? eb : s_off[0];
        const int64_t whi = ee < s_off[cnt] ? ee : s_off[cnt];
        // the window's first adjacency entry to expand lies in entry 0
        int carry = 0;
        for (int64_t e0 = wlo; e0 < whi; e0 += kStep) {
            // Entry of every adjacency entry of the step: the entry holding
            // the first one marks position 0, every entry starting inside the
            // step marks its first position, and a max-scan fills the gaps.
#pragma unroll
            for (int r = 0; r < U; ++r) {
                const int q = tid + r * kWG;
                s_idx[q] = q == 0 ? (int16_t)carry : (int16_t)-1;
            }
            __syncthreads();
            if (tid < cnt) {
                const int64_t p = s_off[tid] - e0;
                if (p >= 0 && p < kStep) s_idx[p] = (int16_t)tid;
            }
            __syncthreads();
            {
                const int lane = lane_id();
                int run = -1;
                int16_t v[U];
#pragma unroll
                for (int r = 0; r < U; ++r) {
                    const int x = s_idx[tid * U + r];
                    run = x > run ? x : run;
                    v[r] = (int16_t)run;
                }
                int inc = run;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int t = __shfl_up(inc, o);
                    if (lane >= o) inc = t > inc ? t : inc;
                }
                int pre = __shfl_up(inc, 1);
                if (lane == 0) pre = -1;
                if (lane == 63) s_wmax[tid >> 6] = inc;
                __syncthreads();
                for (int k = 0; k < (tid >> 6); ++k) pre = s_wmax[k] > pre ? s_wmax[k] : pre;
#pragma unroll
                for (int r = 0; r < U; ++r) s_idx[tid * U + r] = v[r] > pre ? v[r] : (int16_t)pre;
            }
            __syncthreads();
            carry = s_idx[kStep - 1];
            int32_t y[U], own[U], bb[U], deg[U], rs[U];
            uint32_t d[U];
            bool p[U], tz[U];
#pragma unroll
            for (int r = 0; r < U; ++r) {
                const int64_t e = e0 + tid + (int64_t)r * kWG;
                own[r] = -1;
                y[r] = 0;
                if (e < whi) {
                    const int lo = s_idx[tid + r * kWG];
                    if (s_m[lo]) {
                        own[r] = lo;
                        y[r] = ci[s_rs[lo] + (int32_t)(e - s_off[lo])];
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < U; ++r) d[r] = own[r] >= 0 ? (uint32_t)dist[y[r]] : 0u;
#pragma unroll
            for (int r = 0; r < U; ++r) {
                p[r] = false;
                tz[r] = false;
                bb[r] = 0;
                deg[r] = 0;
                rs[r] = 0;
                if (own[r] >= 0 && nl < d[r]) {
                    bb[r] = s_b[own[r]];
                    unsigned long long *vw =
                        reinterpret_cast<unsigned long long *>(a.vis) + (s_rb[own[r]] + (int64_t)y[r]) * 4;
                    // row data is needed only for a claim: load it with the visited word
                    int4 ri;
                    uint32_t d1 = 0;
                    if (a.rinfo) {
                        ri = a.rinfo[y[r]];
                        d1 = load_d1<DistT>(a, y[r]);
                    } else {
                        const int32_t r0 = rp[y[r]];
                        ri = make_int4(r0, rp[y[r] + 1] - r0, 0, 0);
                    }
                    // small levels (latency-bound): claim with the atomic
                    // alone; large ones (many sources, or a level of a full
                    // BFS with many adjacency entries) first read the word, so
                    // that targets every source has reached cost no atomic
                    const uint64_t m = read_first ? s_m[own[r]] & ~(uint64_t)(*vw) : s_m[own[r]];
                    if (m) {
                        const uint64_t ov = atomicOr(vw, (unsigned long long)m);
                        tz[r] = ov == 0ull;
                        const uint64_t nw = m & ~ov;
                        if (nw) {
                            if (WRITE) dist[y[r]] = (DistT)nl;
                            const unsigned long long c = d[r] - nl;
                            const int32_t full = ri.y;
                            rs[r] = ri.x;
                            deg[r] = a.rinfo ? expand_len(ri, d1, nl) : full;
                            const int64_t gb = (int64_t)bb[r] * a.spb;
                            const unsigned long long cp =
                                a.pack ? (c << kPackShift) + (unsigned long long)full : c;
                            const int sl = slot_acc ? (int)s_es[own[r]] : -1;
                            for (uint64_t mm = nw; mm; mm &= mm - 1) {
                                const int bit = __ffsll((unsigned long long)mm) - 1;
                                const int64_t j = gb + bit;
                                if (a.pack) {
                                    if (lds_acc) atomicAdd(&s_g[j], cp);
                                    else if (sl >= 0) atomicAdd(&s_sg[sl * 64 + bit], cp);
                                    else atomicAdd(reinterpret_cast<unsigned long long *>(a.gain + j), cp);
                                    if (a.visited) {
                                        if (lds_acc) atomicAdd(&s_v[j], 1u);
                                        else atomicAdd(a.visited + j, 1);
                                    }
                                } else if (lds_acc) {
                                    atomicAdd(&s_g[j], c);
                                    if (a.edges) atomicAdd(&s_e[j], (unsigned long long)full);
                                    if (a.visited) atomicAdd(&s_v[j], 1u);
                                } else {
                                    atomicAdd(reinterpret_cast<unsigned long long *>(a.gain + j), c);
                                    if (a.edges)
                                        atomicAdd(reinterpret_cast<unsigned long long *>(a.edges + j),
                                                  (unsigned long long)full);
                                    if (a.visited) atomicAdd(a.visited + j, 1);
                                }
                            }
                            // first claim of (batch, node) at this level: one frontier
                            // entry, unless the node has nothing worth expanding
                            p[r] = deg[r] > 0 && atomicOr(vw + fr_next, (unsigned long long)nw) == 0ull;
                        }
                    }
                }
            }
            touch_wave<U>(a, tz, bb, y);
            push_block<U>(a, next, nbase, live, p, y, rs, bb, deg, s_wc, s_wd, &s_old);
        }
        __syncthreads();
        if (slot_acc) {
            // the window's sums to global memory; the slots free again
            for (int q = tid; q < kBatchSlots * 64; q += kWG) {
                const unsigned long long v = s_sg[q];
                if (v) {
                    const int32_t sb = s_sb[q >> 6];
                    atomicAdd(reinterpret_cast<unsigned long long *>(a.gain + (int64_t)sb * a.spb + (q & 63)), v);
                    s_sg[q] = 0ull;
                }
            }
            __syncthreads();
            if (tid < kBatchSlots) s_sb[tid] = -1;
            __syncthreads();
        }
        if (whi >= ee || i + cnt >= N) break;
        i += cnt;
    }
    if (lds_acc) {
        __syncthreads();
        for (int q = tid; q < a.nsrc; q += kWG) {
            if (s_g[q]) atomicAdd(reinterpret_cast<unsigned long long *>(a.gain + q), s_g[q]);
            if (a.edges && s_e[q]) atomicAdd(reinterpret_cast<unsigned long long *>(a.edges + q), s_e[q]);
            if (a.visited && s_v[q]) atomicAdd(a.visited + q, (int)s_v[q]);
        }
    }
    if (L >= 1 && G == (int64_t)gridDim.x) clear_prev(blockIdx.x, gridDim.x);
}

template <typename DistT, bool WRITE, bool LDS, int U, bool SLOTS = false>
__global__ __launch_bounds__(256) void k_wide_level(WideArgs a, int32_t L) {
    level_body<DistT, WRITE, LDS, U, SLOTS>(a, L);
}

// Adds a wave's entries (lanes with p, deg adjacency entries each) to a level
// record without log entries (every lane of a fully active wave calls it).
__device__ __forceinline__ void count_wave(const WideArgs &a, WideLevel *l, bool p, int32_t deg) {
    const uint64_t bal = __ballot(p);
    if (bal == 0) return;
    unsigned long long e = p ? (unsigned long long)deg : 0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
    if (lane_id() == 0) {
        const unsigned long long old =
            atomicAdd(&l->packed, ((unsigned long long)__popcll(bal) << kCntShift) + e);
        if ((old & kMEdges) + e >= (1ull << (kCntShift - 1)) ||
            (old >> kCntShift) + 64 >= (1ull << (63 - kCntShift)))
            set_flag(a.flags, a.tag);
    }
}

// Roots and level 0 of a gain launch in one kernel: the first two steps of
// every candidate's pruned BFS (Section 4.1), for launches of at most
// kFirstMaxSrc candidates with packed sums.  The candidates take the place of
// level 0's log: every workgroup reads all of them, forms the prefix sums of
// their expandable row prefixes in LDS and expands its share of those
// adjacency entries (edge-balanced, as a level kernel does), each candidate
// with its own bit.  A candidate's bit is set only by its own search, and no
// row holds its own node (a self-loop is skipped), so a root claimed by
// another workgroup later than its neighbours changes no result.  The
// workgroups also claim the roots (candidate t by thread t mod 256 of the
// (t / 256)-th workgroup from the last, grid-strided): they store the root
// terms in gain[] and count the roots into level 0's record as the roots
// kernel does, but write no log entries and no level-0 frontier words.  Level-0 sums therefore go to
// acc[] (zero between launches), which the final kernel adds to gain[].
// Level 0 and level 1 both start at log position nsrc: level 1 has nothing of
// level 0 to clear.  The first nids candidate ids come from the argument
// segment (every workgroup reads them all; src may be host memory).
template <typename DistT, int U>
__global__ __launch_bounds__(256) void k_wide_first(WideArgs a, FirstIds ids, int32_t nids) {
    constexpr int kStep = kWG * U;
    constexpr int kPer = (int)(kFirstMaxSrc / kWG);  // candidates per thread in the scan
    __shared__ int64_t c_off[kFirstMaxSrc + 1];       // first adjacency entry of each candidate
    __shared__ int32_t c_rs[kFirstMaxSrc];            // its row start
    __shared__ int32_t c_y[kFirstMaxSrc];             // its node
    __shared__ unsigned long long s_g[kFirstMaxSrc];  // packed level-0 sums
    __shared__ int64_t s_wc[kWG / 64], s_wd[kWG / 64];
    __shared__ uint64_t s_old;
    __shared__ int32_t s_flag;
    if (threadIdx.x == 0) s_flag = __hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (s_flag) return;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int64_t ns = a.nsrc;
    if (ns > kFirstMaxSrc) {
        // (the LDS tables hold kFirstMaxSrc candidates: flag the launch, which
        // the host then redoes with fewer batches)
        if (blockIdx.x == 0 && tid == 0) set_flag(a.flags, a.tag);
        return;
    }
    DistT *dist = reinterpret_cast<DistT *>(const_cast<void *>(a.dist));
    if (blockIdx.x == 0 && tid == 0) {
        a.lvl[0].start = ns;
        a.lvl[1].start = ns;
    }
    // the roots, from the last workgroup down (the host adds workgroups for
    // them beyond those level 0 can use, which keeps them off the
    // expansion's path; uniform trip count per workgroup: the appends are
    // wave ops)
    for (int64_t t0 = ((int64_t)gridDim.x - 1 - blockIdx.x) * kWG; t0 < ns; t0 += (int64_t)gridDim.x * kWG) {
        const int64_t t = t0 + tid;
        bool touched = false, p = false;
        int32_t v = 0, b = 0, deg = 0;
        if (t < ns) {
            v = t < nids ? ids.id[t] : a.src[t];
            b = (int32_t)(t / a.spb);
            const uint64_t bit = 1ull << (t - (int64_t)b * a.spb);
            const uint32_t d = (uint32_t)v < (uint32_t)a.n ? (uint32_t)dist[v] : 0u;
            int64_t gv = 0;
            if (d > 0u) {
                const uint64_t old = atomicOr(rec(a, b, v, 0), (unsigned long long)bit);
                touched = old == 0ull;
                if (bit & ~old) {
                    int32_t full;
                    if (a.rinfo) {
                        const int4 ri = a.rinfo[v];
                        full = ri.y;
                        deg = expand_len(ri, load_d1<DistT>(a, v), 0u);
                    } else {
                        full = a.rp[v + 1] - a.rp[v];
                        deg = full;
                    }
                    gv = ((int64_t)d << kPackShift) + full;
                    p = deg > 0;
                }
            }
            a.gain[t] = gv;
        }
        touch_wave<1>(a, &touched, &b, &v);
        count_wave(a, &a.lvl[0], p, deg);
    }
    // every candidate's expandable prefix (none for a node of S or an id
    // outside [0, n)); thread tid takes candidates kPer*tid .. kPer*tid+kPer-1
    int32_t dg[kPer];
    int64_t loc = 0;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int64_t q = (int64_t)kPer * tid + r;
        int32_t deg = 0;
        if (q < ns) {
            const int32_t v = q < nids ? ids.id[q] : a.src[q];
            int32_t rs = 0;
            const uint32_t d = (uint32_t)v < (uint32_t)a.n ? (uint32_t)dist[v] : 0u;
            if (d > 0u) {
                if (a.rinfo) {
                    const int4 ri = a.rinfo[v];
                    rs = ri.x;
                    deg = expand_len(ri, load_d1<DistT>(a, v), 0u);
                } else {
                    rs = a.rp[v];
                    deg = a.rp[v + 1] - rs;
                }
            }
            c_rs[q] = rs;
            c_y[q] = v;
            s_g[q] = 0ull;
        }
        dg[r] = deg;
        loc += deg;
    }
    int64_t inc = loc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == 63) s_wc[tid >> 6] = inc;
    __syncthreads();
    int64_t pre = inc - loc, E = 0;
#pragma unroll
    for (int k = 0; k < kWG / 64; ++k) {
        if (k < (tid >> 6)) pre += s_wc[k];
        E += s_wc[k];
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int64_t q = (int64_t)kPer * tid + r;
        if (q < ns) c_off[q] = pre;
        pre += dg[r];
    }
    if (tid == 0) c_off[ns] = E;
    __syncthreads();
    // this workgroup's adjacency entries [eb, ee), as a level kernel takes them
    int64_t G = E == 0 ? 0 : (E + a.min_edges - 1) / a.min_edges;
    if (G > (int64_t)gridDim.x) G = gridDim.x;
    if ((int64_t)blockIdx.x >= G) return;
    const int64_t eb = E * (int64_t)blockIdx.x / G;
    const int64_t ee = E * ((int64_t)blockIdx.x + 1) / G;
    if (eb >= ee) return;
    const uint32_t nl = 1u;
    const int32_t *__restrict__ ci = a.ci;
    for (int64_t e0 = eb; e0 < ee; e0 += kStep) {
        int32_t y[U], own[U], bb[U], deg[U], rs[U];
        uint32_t d[U];
        bool p[U], tz[U];
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const int64_t e = e0 + tid + (int64_t)r * kWG;
            own[r] = -1;
            y[r] = 0;
            if (e < ee) {
                // the last candidate whose first entry is at or before e (its prefix holds e)
                int lo = 0, hi = (int)ns - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (c_off[mid] <= e) lo = mid;
                    else hi = mid - 1;
                }
                own[r] = lo;
                y[r] = ci[c_rs[lo] + (int32_t)(e - c_off[lo])];
            }
        }
#pragma unroll
        for (int r = 0; r < U; ++r) d[r] = own[r] >= 0 ? (uint32_t)dist[y[r]] : 0u;
#pragma unroll
        for (int r = 0; r < U; ++r) {
            p[r] = false;
            tz[r] = false;
            bb[r] = 0;
            deg[r] = 0;
            rs[r] = 0;
            if (own[r] >= 0 && nl < d[r] && y[r] != c_y[own[r]]) {
                const int q = own[r];
                const int32_t b = (int32_t)(q / a.spb);
                bb[r] = b;
                const uint64_t bit = 1ull << (q - b * a.spb);
                unsigned long long *vw = rec(a, b, y[r], 0);
                int4 ri;
                uint32_t d1 = 0;
                if (a.rinfo) {
                    ri = a.rinfo[y[r]];
                    d1 = load_d1<DistT>(a, y[r]);
                } else {
                    const int32_t r0 = a.rp[y[r]];
                    ri = make_int4(r0, a.rp[y[r] + 1] - r0, 0, 0);
                }
                const uint64_t ov = atomicOr(vw, (unsigned long long)bit);
                tz[r] = ov == 0ull;
                if (!(ov & bit)) {
                    const int32_t full = ri.y;
                    rs[r] = ri.x;
                    deg[r] = a.rinfo ? expand_len(ri, d1, nl) : full;
                    atomicAdd(&s_g[q], ((unsigned long long)(d[r] - nl) << kPackShift) + (unsigned long long)full);
                    // level 1's frontier word is word 1 + (1 mod 3)
                    p[r] = deg[r] > 0 && atomicOr(vw + 2, (unsigned long long)bit) == 0ull;
                }
            }
        }
        touch_wave<U>(a, tz, bb, y);
        push_block<U>(a, &a.lvl[1], ns, ns, p, y, rs, bb, deg, s_wc, s_wd, &s_old);
    }
    __syncthreads();
    for (int q = tid; q < ns; q += kWG)
        if (s_g[q]) atomicAdd(a.acc + q, s_g[q]);
}

// End of a launch: return every touched record to zero, copy the results
// to the host-mapped buffers if given and scatter them into the lazy-loop
// state if asked.  After an overflow nothing is cleared here; the host clears
// and retries.
__device__ __forceinline__ void end_body(const WideArgs &a) {
    const int32_t flag = __hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    if (flag) {
        if (a.h_flag && blockIdx.x == 0 && threadIdx.x == 0) *a.h_flag = flag;
        // (the launch is redone: its level-0 sums go)
        if (a.acc)
            for (int64_t i = t0; i < a.nsrc; i += nt) a.acc[i] = 0ull;
        return;
    }
    int64_t tot = (int64_t)*a.zcnt;
    if (tot > a.zcap) tot = a.zcap;
    for (int64_t i = t0; i < tot; i += nt) {
        const int64_t z = a.lz[i];
        unsigned long long *r0 = rec(a, z >> 32, (int32_t)(uint32_t)z, 0);
        r0[0] = 0ull;
        r0[1] = 0ull;
        r0[2] = 0ull;
        r0[3] = 0ull;
    }
    if (a.pack)
        for (int64_t i = t0; i < a.nsrc; i += nt) {
            int64_t v = a.gain[i];
            if (a.acc) {
                v += (int64_t)a.acc[i];
                a.acc[i] = 0ull;
            }
            a.gain[i] = v >> kPackShift;
            if (a.edges) a.edges[i] = v & ((1ll << kPackShift) - 1);
        }
    if (a.h_gain)
        for (int64_t i = t0; i < a.nsrc; i += nt) a.h_gain[i] = a.gain[i];
    if (a.h_edges && a.edges)
        for (int64_t i = t0; i < a.nsrc; i += nt) a.h_edges[i] = a.edges[i];
    // host-mapped results written by this thread are visible before the done word
    if (a.h_done && t0 < a.nsrc && (a.h_gain || a.h_edges)) __threadfence_system();
    if (a.ub_out)
        for (int64_t i = t0; i < a.nsrc; i += nt) {
            const int32_t v = a.src[i];
            if ((uint32_t)v >= (uint32_t)a.n) continue;
            a.ub_out[v] = a.gain[i];
            a.le_out[v] = a.round;
            a.dsat_out[v] = a.dist_bytes == 1 ? (uint16_t)reinterpret_cast<const uint8_t *>(a.dist)[v]
                                              : reinterpret_cast<const uint16_t *>(a.dist)[v];
        }
}

__global__ void k_wide_end(WideArgs a, int32_t nlev) {
    (void)nlev;
    end_body(a);
}

// After k_wide_end (one workgroup): count the launch's word-level work, zero
// the level records so the next launch starts clean, clear the host-visible
// flag and (update mode) F(S + s) = F(S) - g(s, S).
__device__ __forceinline__ void reset_body(const WideArgs &a, int32_t nlev) {
    if (__hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    if (threadIdx.x == 0) {
        if (a.words) {
            int64_t nall = 0, eexp = 0;
            for (int32_t l = 0; l <= nlev; ++l) {
                const uint64_t pk = a.lvl[l].packed;
                nall += (int64_t)(pk >> kCntShift);
                if (l < nlev) eexp += (int64_t)(pk & kMEdges);
            }
            const uint64_t pl = a.lvl[nlev].packed;
            a.words[0] += nall;
            a.words[1] += (int64_t)(a.lvl[0].packed >> kCntShift);
            a.words[2] += (int64_t)(pl >> kCntShift);
            a.words[3] += eexp;
            a.words[4] += (int64_t)(pl & kMEdges);
            a.words[5] += (int64_t)*a.zcnt;
        }
        if (a.h_flag) *a.h_flag = 0;
        if (a.far) *a.far -= a.gain[0];  // update: F(S + s) = F(S) - g(s, S)
        *a.zcnt = 0ull;
        if (a.h_maxd) *a.h_maxd = *a.maxd_src;
        if (a.h_done) {
            __threadfence_system();
            *reinterpret_cast<volatile int64_t *>(a.h_done) = a.seq;
        }
    }
    __syncthreads();
    for (int32_t l = threadIdx.x; l <= nlev + 1; l += blockDim.x) {
        a.lvl[l].start = 0;
        a.lvl[l].packed = 0ull;
    }
}

__global__ void k_wide_reset(WideArgs a, int32_t nlev) { reset_body(a, nlev); }

// BFScut test (Section 3.1) after level L of a closeness launch: every node at
// distance <= L+1 from source v is known (r of them, distance sum `sum`); of
// the rem = n - r others at most ef (adjacency entries of the distance-(L+1)
// nodes, minus one back-edge each) are at distance L+2, the rest are farther.
// A source whose bound exceeds the best farness known is dropped.
// fixed: *best is a threshold set by the host (top-k with k > 1), not
// lowered by finished sources.
__global__ void k_wide_cut(WideArgs a, int32_t L, int64_t *best, int32_t fixed) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= a.nsrc) return;
    const int64_t b = t / a.spb;
    const uint64_t bit = 1ull << (t - b * a.spb);
    if (!(__hip_atomic_load(&a.active[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit)) return;
    const int64_t r = a.visited[t];
    const int64_t e = a.edges[t];
    const int64_t dr = r - a.prev[2 * t];
    const int64_t de = e - a.prev[2 * t + 1];
    a.prev[2 * t] = r;
    a.prev[2 * t + 1] = e;
    const int64_t sum = r * 65535 - a.gain[t];
    if (r == a.n) {
        a.far_out[t] = sum;
        if (!fixed) atomicMin(reinterpret_cast<unsigned long long *>(best), (unsigned long long)sum);
        atomicAnd(&a.active[b], ~bit);
        return;
    }
    if (dr == 0) {  // frontier empty before reaching every node (disconnected)
        atomicAnd(&a.active[b], ~bit);
        return;
    }
    const int64_t rem = (int64_t)a.n - r;
    // (undirected: one of each new node's adjacency entries leads back)
    const int64_t ef = a.directed ? de : de - dr;
    const int64_t near = ef < rem ? ef : rem;
    const int64_t lb = sum + (int64_t)(L + 2) * near + (int64_t)(L + 3) * (rem - near);
    const int64_t bv = (int64_t)__hip_atomic_load(reinterpret_cast<unsigned long long *>(best),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (lb > bv) atomicAnd(&a.active[b], ~bit);
}

// Early exit inside the candidates' pruned BFS (gain launches with an
// active mask): after the nodes at distance l from source v are claimed (gain
// so far g, de the adjacency entries of the nodes claimed at distance l),
// every node v can still claim is at distance >= l+1 with d(S,.) >= l+2 --
// at most de of them at distance l+1, each worth 1 + (d(S,.) - l - 2), the
// rest worth at most d(S,.) - l - 2 -- so g(v,S) <= g + de + T[l+1] with
// T[j] = sum_w max(0, d(S,w) - j - 1) (a BFScut-style bound, Section 3.1, on
// the pruned BFS of Section 4.1).  A source whose bound cannot beat the
// launch's threshold (bound < thr, or bound == thr and v > thr_id) stops: its
// bits leave the batch's active mask and its gain becomes the bound (an upper
// bound, kept as its stale gain); far_out marks it (1).  A source that claimed
// nothing at distance l has finished and keeps its exact gain.  The test is
// made only while a deeper level can still claim a node (l + 1 < max d(S,.)).
__global__ void k_gain_cut(WideArgs a, int32_t l) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= a.nsrc) return;
    const int64_t b = t / a.spb;
    const uint64_t bit = 1ull << (t - b * a.spb);
    if (!(__hip_atomic_load(&a.active[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit)) return;
    const int64_t r = a.visited[t];
    const int64_t e = a.edges[t];
    const int64_t dr = r - a.prev[2 * t];
    const int64_t de = e - a.prev[2 * t + 1];
    a.prev[2 * t] = r;
    a.prev[2 * t + 1] = e;
    if (dr == 0) {
        atomicAnd(&a.active[b], ~bit);
        return;
    }
    if (l + 1 >= a.cut_maxd) return;
    const int64_t bound = a.gain[t] + de + a.cut_T[l + 1];
    const int32_t v = a.src[t];
    if (bound < a.cut_thr || (bound == a.cut_thr && v > a.cut_id)) {
        a.gain[t] = bound;
        a.far_out[t] = 1;
        atomicAnd(&a.active[b], ~bit);
        atomicAdd(a.cut_count, 1ull);
    }
}

// hist[d] = #{w : d(S,w) = d} for d <= maxd (hist zeroed by the caller)
template <typename DistT>
__global__ void k_dist_hist(const DistT *dist, int64_t n, int32_t maxd, unsigned long long *hist) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t d = dist[i];
        if (d <= maxd) atomicAdd(&hist[d], 1ull);
    }
}

// T[j] = sum_{d >= j+2} (d - j - 1) hist[d] for j = 0..maxd, from suffix sums
// of the counts and of d times the counts (one thread: maxd is at most 65534)
__global__ void k_tail_table(const unsigned long long *hist, int32_t maxd, int64_t *T) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t cnt = 0, sum = 0;  // over d > j + 1
    for (int32_t j = maxd; j >= 0; --j) {
        if (j + 2 <= maxd) {
            cnt += (int64_t)hist[j + 2];
            sum += (int64_t)(j + 2) * (int64_t)hist[j + 2];
        }
        T[j] = sum - (int64_t)(j + 1) * cnt;
    }
    T[maxd + 1] = 0;
}

// sum of neighbour degrees, one wave per row (hub rows spread over the lanes)
__global__ __launch_bounds__(256) void k_twohop_i64(const int32_t *rp, const int32_t *ci, int32_t n,
                                                     int64_t *out) {
    const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int lane = lane_id();
    if (row >= n) return;
    const int32_t rs = rp[row], re = rp[row + 1];
    int64_t acc = 0;
    for (int32_t e = rs + lane; e < re; e += 64) {
        const int32_t u = ci[e];
        acc += rp[u + 1] - rp[u];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) out[row] = acc;
}

// One wave per row: order the row [d > d(y) | d == d(y) | d < d(y)] (stable
// within each part) and record the part sizes.
template <typename DistT>
__global__ __launch_bounds__(256) void k_row_split(const int32_t *rp, const int32_t *ci, int32_t n,
                                                    const DistT *dist, int32_t *ci_out, int4 *rinfo,
                                                    DistT *dist1, int32_t skip_long) {
    const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int lane = lane_id();
    if (row >= n) return;
    const int32_t rs = rp[row], re = rp[row + 1];
    if (skip_long && re - rs > kSplitLongRow) return;  // split chunk by chunk (below)
    const uint32_t dy = dist[row];
    if (re - rs <= 64) {
        // one chunk: classify and place in one pass
        const int32_t e = rs + lane;
        const bool ok = e < re;
        int32_t z = 0;
        uint32_t dz = dy;
        if (ok) {
            z = ci[e];
            dz = dist[z];
        }
        const bool down = ok && dz > dy, same = ok && dz == dy, up = ok && dz < dy;
        const uint64_t bd = __ballot(down), bs = __ballot(same), bu = __ballot(up);
        const int32_t nd1 = __popcll(bd), ns1 = __popcll(bs);
        if (down) ci_out[rs + bits_below(bd)] = z;
        if (same) ci_out[rs + nd1 + bits_below(bs)] = z;
        if (up) ci_out[rs + nd1 + ns1 + bits_below(bu)] = z;
        if (lane == 0) {
            rinfo[row] = make_int4(rs, re - rs, nd1, nd1 + ns1);
            dist1[row] = (DistT)dy;
        }
        return;
    }
    int32_t nd = 0, ns = 0;
    for (int32_t base = rs; base < re; base += 64) {
        const int32_t e = base + lane;
        uint32_t dz = dy;
        bool ok = e < re;
        if (ok) dz = dist[ci[e]];
        nd += __popcll(__ballot(ok && dz > dy));
        ns += __popcll(__ballot(ok && dz == dy));
    }
    int32_t pd = rs, ps = rs + nd, pu = rs + nd + ns;
    for (int32_t base = rs; base < re; base += 64) {
        const int32_t e = base + lane;
        const bool ok = e < re;
        int32_t z = 0;
        uint32_t dz = dy;
        if (ok) {
            z = ci[e];
            dz = dist[z];
        }
        const bool down = ok && dz > dy, same = ok && dz == dy, up = ok && dz < dy;
        const uint64_t bd = __ballot(down), bs = __ballot(same), bu = __ballot(up);
        if (down) ci_out[pd + bits_below(bd)] = z;
        if (same) ci_out[ps + bits_below(bs)] = z;
        if (up) ci_out[pu + bits_below(bu)] = z;
        pd += __popcll(bd);
        ps += __popcll(bs);
        pu += __popcll(bu);
    }
    if (lane == 0) {
        rinfo[row] = make_int4(rs, re - rs, nd, nd + ns);
        dist1[row] = (DistT)dy;
    }
}

// The rows of more than kSplitLongRow entries, a workgroup per chunk of
// kSplitChunk entries (a hub's row is split by many workgroups, not by one
// wave).  Pass 1 counts each chunk's entries of the first two parts.
template <typename DistT>
__global__ __launch_bounds__(256) void k_row_split_count(const int32_t *rp, const int32_t *ci, const DistT *dist,
                                                         const int32_t *chunks, int32_t *cnt) {
    __shared__ int32_t s_d[4], s_s[4];
    const int32_t i = blockIdx.x;
    const int32_t row = chunks[2 * i], first = chunks[2 * i + 1];
    const int32_t end = rp[row + 1];
    const int32_t rs = rp[row] + (i - first) * kSplitChunk;
    const int32_t re = end - rs < kSplitChunk ? end : rs + kSplitChunk;
    const uint32_t dy = dist[row];
    int32_t nd = 0, ns = 0;
    for (int32_t e = rs + (int32_t)threadIdx.x; e < re; e += 256) {
        const uint32_t dz = dist[ci[e]];
        nd += dz > dy ? 1 : 0;
        ns += dz == dy ? 1 : 0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        nd += __shfl_down(nd, o, 64);
        ns += __shfl_down(ns, o, 64);
    }
    if (lane_id() == 0) {
        s_d[threadIdx.x >> 6] = nd;
        s_s[threadIdx.x >> 6] = ns;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cnt[2 * i] = s_d[0] + s_d[1] + s_d[2] + s_d[3];
        cnt[2 * i + 1] = s_s[0] + s_s[1] + s_s[2] + s_s[3];
    }
}

// Pass 2: each chunk places its entries after the earlier chunks' entries of
// each part, in order; the row's first chunk writes the row's record.
template <typename DistT>
__global__ __launch_bounds__(256) void k_row_split_place(const int32_t *rp, const int32_t *ci, const DistT *dist,
                                                         const int32_t *chunks, const int32_t *cnt,
                                                         int32_t *ci_out, int4 *rinfo, DistT *dist1) {
    __shared__ int32_t s_pos[3];
    __shared__ int32_t s_w[3][4];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const int32_t i = blockIdx.x;
    const int32_t row = chunks[2 * i], first = chunks[2 * i + 1];
    const int32_t k = i - first;
    const int32_t RS = rp[row], RE = rp[row + 1];
    const uint32_t dy = dist[row];
    if (tid == 0) {
        const int32_t nch = (RE - RS + kSplitChunk - 1) / kSplitChunk;
        int32_t ND = 0, NS = 0, pd = 0, ps = 0;
        for (int32_t j = 0; j < nch; ++j) {
            const int32_t d = cnt[2 * (first + j)], sm = cnt[2 * (first + j) + 1];
            if (j < k) {
                pd += d;
                ps += sm;
            }
            ND += d;
            NS += sm;
        }
        s_pos[0] = RS + pd;
        s_pos[1] = RS + ND + ps;
        s_pos[2] = RS + ND + NS + (k * kSplitChunk - pd - ps);
        if (k == 0) {
            rinfo[row] = make_int4(RS, RE - RS, ND, ND + NS);
            dist1[row] = (DistT)dy;
        }
    }
    __syncthreads();
    const int32_t rs = RS + k * kSplitChunk;
    const int32_t re = RE - rs < kSplitChunk ? RE : rs + kSplitChunk;
    for (int32_t base = rs; base < re; base += 256) {
        const int32_t e = base + tid;
        const bool ok = e < re;
        int32_t z = 0;
        uint32_t dz = dy;
        if (ok) {
            z = ci[e];
            dz = dist[z];
        }
        const bool down = ok && dz > dy, same = ok && dz == dy, up = ok && dz < dy;
        const uint64_t bd = __ballot(down), bs = __ballot(same), bu = __ballot(up);
        if (lane == 0) {
            s_w[0][wave] = __popcll(bd);
            s_w[1][wave] = __popcll(bs);
            s_w[2][wave] = __popcll(bu);
        }
        __syncthreads();
        int32_t od = s_pos[0], os = s_pos[1], ou = s_pos[2];
        for (int w = 0; w < wave; ++w) {
            od += s_w[0][w];
            os += s_w[1][w];
            ou += s_w[2][w];
        }
        if (down) ci_out[od + bits_below(bd)] = z;
        if (same) ci_out[os + bits_below(bs)] = z;
        if (up) ci_out[ou + bits_below(bu)] = z;
        __syncthreads();  // every thread has read s_pos and s_w
        if (tid < 3) s_pos[tid] += s_w[tid][0] + s_w[tid][1] + s_w[tid][2] + s_w[tid][3];
        __syncthreads();
    }
}

// Level-1 bound of F({v}) (Section 3.1 with the BFS stopped after one level):
// deg(v) nodes at distance 1, at most two(v) - deg(v) at distance 2 (the
// adjacency of v's neighbours minus one back-edge each), the rest at 3 or more.
// Directed graphs: a neighbour's row need not hold the arc back to v, so
// nodes at distance 2 are bounded by two(v) itself.
__global__ void k_lb1_filter(const int32_t *order, const int32_t *rp, const int64_t *two, int32_t n,
                             int64_t best_f, int32_t best_v, uint8_t *keep, int64_t *bound,
                             int32_t directed) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i == 0) {
        keep[0] = 0;
        bound[0] = 0;
        return;
    }
    const int32_t v = order[i];
    const int64_t d = rp[v + 1] - rp[v];
    const int64_t rem = (int64_t)n - 1 - d;
    int64_t near = directed ? two[v] : two[v] - d;
    if (near > rem) near = rem;
    if (near < 0) near = 0;
    const int64_t b = d + 2 * near + 3 * (rem - near);
    bound[i] = b;
    keep[i] = (b < best_f || (b == best_f && v < best_v)) ? 1 : 0;
}

__global__ void k_gather_i64(const int64_t *src, const int32_t *idx, int32_t cnt, int64_t *out) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j < cnt) out[j] = src[idx[j]];
}

template <typename DistT>
__global__ void k_max_dist(const DistT *dist, int64_t n, int32_t *out) {
    uint32_t m = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = dist[i];
        m = v > m ? v : m;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t t = __shfl_xor(m, o);
        m = t > m ? t : m;
    }
    if (lane_id() == 0) atomicMax(out, (int32_t)m);
}

__global__ void k_fill_u64_tail(unsigned long long *p, int64_t count) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0ull;
}

__global__ void k_set_i32(int32_t *p, int32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

}  // namespace

hipError_t launch_wide_begin(const WideArgs &a, int dist_bytes, int32_t nlev, hipStream_t s) {
    (void)nlev;
    const int groots = (int)((a.nsrc + 255) / 256);
    if (dist_bytes == 1) {
        if (a.write) hipLaunchKernelGGL((k_wide_roots<uint8_t, true>), dim3(groots), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_wide_roots<uint8_t, false>), dim3(groots), dim3(256), 0, s, a);
    } else {
        if (a.write) hipLaunchKernelGGL((k_wide_roots<uint16_t, true>), dim3(groots), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_wide_roots<uint16_t, false>), dim3(groots), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_wide_first(const WideArgs &a, int dist_bytes, int grid, const FirstIds &ids, int32_t nids,
                             hipStream_t s) {
    const int g = grid < 1 ? 1 : grid;
    const int32_t k = nids < 0 ? 0 : (nids > kFirstArgIds ? kFirstArgIds : nids);
    if (dist_bytes == 1) {
        if (a.unroll >= 8) hipLaunchKernelGGL((k_wide_first<uint8_t, 8>), dim3(g), dim3(kWG), 0, s, a, ids, k);
        else hipLaunchKernelGGL((k_wide_first<uint8_t, 4>), dim3(g), dim3(kWG), 0, s, a, ids, k);
    } else {
        if (a.unroll >= 8) hipLaunchKernelGGL((k_wide_first<uint16_t, 8>), dim3(g), dim3(kWG), 0, s, a, ids, k);
        else hipLaunchKernelGGL((k_wide_first<uint16_t, 4>), dim3(g), dim3(kWG), 0, s, a, ids, k);
    }
    return hipGetLastError();
}

template <typename DistT, bool WRITE>
static void launch_level(const WideArgs &a, int32_t L, int grid, hipStream_t s) {
    const bool lds = a.nsrc <= kLdsSrc;
    if (lds) {
        if (a.unroll >= 8)
            hipLaunchKernelGGL((k_wide_level<DistT, WRITE, true, 8>), dim3(grid), dim3(kWG), 0, s, a, L);
        else
            hipLaunchKernelGGL((k_wide_level<DistT, WRITE, true, 4>), dim3(grid), dim3(kWG), 0, s, a, L);
    } else if (a.pack == 2) {
        // (a separate instantiation: the slots' LDS and code stay out of the others)
        if (a.unroll == 16)
            hipLaunchKernelGGL((k_wide_level<DistT, WRITE, false, 16, true>), dim3(grid), dim3(kWG), 0, s, a, L);
        else if (a.unroll == 8)
            hipLaunchKernelGGL((k_wide_level<DistT, WRITE, false, 8, true>), dim3(grid), dim3(kWG), 0, s, a, L);
        else
            hipLaunchKernelGGL((k_wide_level<DistT, WRITE, false, 4, true>), dim3(grid), dim3(kWG), 0, s, a, L);
    } else if (a.unroll == 16) {
        hipLaunchKernelGGL((k_wide_level<DistT, WRITE, false, 16>), dim3(grid), dim3(kWG), 0, s, a, L);
    } else if (a.unroll == 8) {
        hipLaunchKernelGGL((k_wide_level<DistT, WRITE, false, 8>), dim3(grid), dim3(kWG), 0, s, a, L);
    } else {
        hipLaunchKernelGGL((k_wide_level<DistT, WRITE, false, 4>), dim3(grid), dim3(kWG), 0, s, a, L);
    }
}

hipError_t launch_wide_levels(const WideArgs &a, int dist_bytes, int32_t l0, int32_t l1, int grid,
                              hipStream_t s) {
    for (int32_t L = l0; L < l1; ++L) {
        if (dist_bytes == 1) {
            if (a.write) launch_level<uint8_t, true>(a, L, grid, s);
            else launch_level<uint8_t, false>(a, L, grid, s);
        } else {
            if (a.write) launch_level<uint16_t, true>(a, L, grid, s);
            else launch_level<uint16_t, false>(a, L, grid, s);
        }
    }
    return hipGetLastError();
}

hipError_t launch_wide_end(const WideArgs &a, int32_t nlev, int grid, hipStream_t s) {
    // the record clean-up is a scatter of 32-byte stores, one per frontier
    // entry: it takes the whole grid even for a small batch (a hub's pruned
    // BFS can touch most of the graph); the level records are reset after it
    const int g = grid < 1 ? 1 : grid;
    hipLaunchKernelGGL(k_wide_end, dim3(g), dim3(256), 0, s, a, nlev);
    hipLaunchKernelGGL(k_wide_reset, dim3(1), dim3(256), 0, s, a, nlev);
    return hipGetLastError();
}

hipError_t launch_wide_cut(const WideArgs &a, int32_t L, int64_t *best, bool fixed, hipStream_t s) {
    const int g = (int)((a.nsrc + 255) / 256);
    hipLaunchKernelGGL(k_wide_cut, dim3(g < 1 ? 1 : g), dim3(256), 0, s, a, L, best, (int32_t)fixed);
    return hipGetLastError();
}

hipError_t launch_gain_cut(const WideArgs &a, int32_t l, hipStream_t s) {
    const int g = (int)((a.nsrc + 255) / 256);
    hipLaunchKernelGGL(k_gain_cut, dim3(g < 1 ? 1 : g), dim3(256), 0, s, a, l);
    return hipGetLastError();
}

hipError_t launch_tail_table(const void *dist, int dist_bytes, int64_t n, int32_t maxd,
                             unsigned long long *hist, int64_t *T, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64_tail, dim3(((int64_t)maxd + 2 + 255) / 256), dim3(256), 0, s, hist,
                       (int64_t)maxd + 2);
    int64_t g = (n + 255) / 256;
    const int grid = (int)(g > 2048 ? 2048 : (g < 1 ? 1 : g));
    if (dist_bytes == 1)
        hipLaunchKernelGGL((k_dist_hist<uint8_t>), dim3(grid), dim3(256), 0, s,
                           reinterpret_cast<const uint8_t *>(dist), n, maxd, hist);
    else
        hipLaunchKernelGGL((k_dist_hist<uint16_t>), dim3(grid), dim3(256), 0, s,
                           reinterpret_cast<const uint16_t *>(dist), n, maxd, hist);
    hipLaunchKernelGGL(k_tail_table, dim3(1), dim3(64), 0, s, hist, maxd, T);
    return hipGetLastError();
}

hipError_t launch_twohop_i64(const int32_t *rp, const int32_t *ci, int32_t n, int64_t *out,
                             hipStream_t s) {
    const int64_t g = ((int64_t)n * 64 + 255) / 256;
    hipLaunchKernelGGL(k_twohop_i64, dim3((int)(g < 1 ? 1 : g)), dim3(256), 0, s, rp, ci, n, out);
    return hipGetLastError();
}

template <typename DistT>
static void launch_split_t(const int32_t *rp, const int32_t *ci, int32_t n, const void *dist, int32_t *ci_out,
                           int4 *rinfo, void *dist1, const int32_t *chunks, int32_t nchunks, int32_t *cnt,
                           hipStream_t s) {
    const DistT *d = reinterpret_cast<const DistT *>(dist);
    DistT *d1 = reinterpret_cast<DistT *>(dist1);
    const bool chunked = chunks != nullptr && nchunks > 0;
    const int64_t g = ((int64_t)n * 64 + 255) / 256;
    hipLaunchKernelGGL((k_row_split<DistT>), dim3((unsigned)(g < 1 ? 1 : g)), dim3(256), 0, s, rp, ci, n, d,
                       ci_out, rinfo, d1, (int32_t)chunked);
    if (!chunked) return;
    hipLaunchKernelGGL((k_row_split_count<DistT>), dim3((unsigned)nchunks), dim3(256), 0, s, rp, ci, d, chunks,
                       cnt);
    hipLaunchKernelGGL((k_row_split_place<DistT>), dim3((unsigned)nchunks), dim3(256), 0, s, rp, ci, d, chunks,
                       cnt, ci_out, rinfo, d1);
}

hipError_t launch_row_split(const int32_t *rp, const int32_t *ci, int32_t n, const void *dist,
                            int dist_bytes, int32_t *ci_out, int4 *rinfo, void *dist1,
                            const int32_t *chunks, int32_t nchunks, int32_t *cnt, hipStream_t s) {
    if (dist_bytes == 1)
        launch_split_t<uint8_t>(rp, ci, n, dist, ci_out, rinfo, dist1, chunks, nchunks, cnt, s);
    else
        launch_split_t<uint16_t>(rp, ci, n, dist, ci_out, rinfo, dist1, chunks, nchunks, cnt, s);
    return hipGetLastError();
}

hipError_t launch_lb1_filter(const int32_t *order, const int32_t *rp, const int64_t *two, int32_t n,
                             int64_t best_f, int32_t best_v, uint8_t *keep, int64_t *bound, bool directed,
                             hipStream_t s) {
    const int64_t g = ((int64_t)n + 255) / 256;
    hipLaunchKernelGGL(k_lb1_filter, dim3((unsigned)(g < 1 ? 1 : g)), dim3(256), 0, s, order, rp, two, n,
                       best_f, best_v, keep, bound, (int32_t)directed);
    return hipGetLastError();
}

hipError_t launch_gather_i64(const int64_t *src, const int32_t *idx, int32_t cnt, int64_t *out,
                             hipStream_t s) {
    if (cnt <= 0) return hipSuccess;
    const int64_t g = ((int64_t)cnt + 255) / 256;
    hipLaunchKernelGGL(k_gather_i64, dim3((unsigned)g), dim3(256), 0, s, src, idx, cnt, out);
    return hipGetLastError();
}

hipError_t launch_max_dist(const void *dist, int dist_bytes, int64_t n, int32_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(64), 0, s, out, 0);
    int64_t g = (n + 255) / 256;
    int grid = (int)(g > 1024 ? 1024 : (g < 1 ? 1 : g));
    if (dist_bytes == 1)
        hipLaunchKernelGGL((k_max_dist<uint8_t>), dim3(grid), dim3(256), 0, s,
                           reinterpret_cast<const uint8_t *>(dist), n, out);
    else
        hipLaunchKernelGGL((k_max_dist<uint16_t>), dim3(grid), dim3(256), 0, s,
                           reinterpret_cast<const uint16_t *>(dist), n, out);
    return hipGetLastError();
}

}  // namespace gck
