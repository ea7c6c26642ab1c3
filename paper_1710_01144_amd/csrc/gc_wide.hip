// Device-wide bit-parallel pruned BFS for marginal gains (gfx950).
//
// Candidates are grouped 64 to a batch; batch b owns a dense word array
// vis_b[0..n) whose bit j marks nodes already reached by source j of the
// batch.  All batches of a launch advance one BFS level per kernel, so a
// level is one edge-balanced sweep over the whole device:
//
//   frontier entry (b, x, F) at distance L, F = bits of the sources that
//   reached x at distance L.  For each neighbour y of x:
//     L+1 >= d(S,y)        -> pruned (Section 4.1): neither y nor anything
//                             behind it can be closer to the source than to S;
//                             nothing is written;
//     otherwise claim nw = F & ~vis_b[y] with one atomicOr; every claimed
//     source j gains d(S,y) - (L+1) (the summand of the gain sum in the proof
//     of the Section 4.3 theorem) and (b, y, nw) joins the next frontier.
//
// Load balance: when entries are appended, one 64-bit atomic per wave
// reserves both their slots and the range of adjacency positions they will
// expand ((count << 40) | edges).  Edge offsets are therefore monotone in
// the entry index, and the next level splits its total edge count evenly over
// the workgroups (a hub's adjacency is spread over many of them); each
// workgroup finds its first entry with a 64-ary search and walks windows of
// 256 entries staged in LDS.
//
// No level count is needed from the host: a pruned BFS never goes deeper than
// max_y d(S,y) - 1, so the host launches that many levels.
#include "gc_kernels.h"

namespace gck {
namespace {

constexpr int kWin = 256;   // entries staged per window
constexpr int kUnroll = 4;  // edges per thread per step (independent loads in flight)
constexpr uint64_t kM40 = (1ull << 40) - 1;

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

__device__ __forceinline__ void set_flag(int32_t *flag, int32_t v) {
    atomicCAS(flag, 0, v);
}

// Append entries of lanes with p to the frontier of the next level.  Called
// by every lane of a fully active wave.
__device__ __forceinline__ void push_entries(const WideArgs &a, WideLevel *nl, int64_t nbase, bool p,
                                             int32_t y, int32_t b, uint64_t bits, int32_t deg) {
    const uint64_t bal = __ballot(p);
    if (bal == 0) return;
    const int lane = lane_id();
    int dp = p ? deg : 0;
    int incl = dp;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    const int total = __shfl(incl, 63);
    uint64_t old = 0;
    if (lane == 0) {
        old = atomicAdd(&nl->packed, ((unsigned long long)__popcll(bal) << 40) + (unsigned long long)total);
        if ((old & kM40) + (uint64_t)total >= (1ull << 39) || (old >> 40) + 64 >= (1ull << 24))
            set_flag(a.flags, a.tag);
    }
    old = shfl64(old, 0);
    if (!p) return;
    const int64_t idx = (int64_t)(old >> 40) + bits_below(bal);
    const int64_t pos = nbase + idx;
    if (pos >= a.cap) {
        set_flag(a.flags, a.tag);
        return;
    }
    a.ly[pos] = y;
    a.lb[pos] = b;
    a.lm[pos] = bits;
    a.lo[pos] = (int64_t)(old & kM40) + (incl - dp);
}

__global__ void k_wide_zero(WideArgs a, int32_t nlev) {
    const int64_t tot = (int64_t)a.nsrc > (int64_t)nlev + 2 ? (int64_t)a.nsrc : (int64_t)nlev + 2;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < a.nsrc) {
            a.gain[i] = 0;
            if (a.edges) a.edges[i] = 0;
            if (a.visited) a.visited[i] = 0;
        }
        if (i < nlev + 2) {
            a.lvl[i].start = 0;
            a.lvl[i].packed = 0ull;
        }
    }
}

// Level 0: every source claims its own node (weight d(S,v) - 0).
template <typename DistT>
__global__ __launch_bounds__(256) void k_wide_roots(WideArgs a) {
    if (__hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const DistT *dist = reinterpret_cast<const DistT *>(a.dist);
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool p = false;
    int32_t v = 0, b = 0, deg = 0;
    uint64_t nw = 0;
    if (t < a.nsrc) {
        v = a.src[t];
        b = (int32_t)(t / a.spb);
        const uint32_t d = dist[v];
        if (d > 0u) {
            const uint64_t bit = 1ull << (t - (int64_t)b * a.spb);
            unsigned long long *w = reinterpret_cast<unsigned long long *>(a.vis + (size_t)b * a.vis_stride + v);
            const uint64_t old = atomicOr(w, (unsigned long long)bit);
            nw = bit & ~old;
            if (nw) {
                deg = a.rp[v + 1] - a.rp[v];
                a.gain[t] = (int64_t)d;
                if (a.edges) a.edges[t] = deg;
                if (a.visited) a.visited[t] = 1;
                p = true;
            }
        }
    }
    push_entries(a, &a.lvl[0], 0, p, v, b, nw, deg);
}

template <typename DistT>
__global__ __launch_bounds__(256) void k_wide_level(WideArgs a, int32_t L) {
    __shared__ int64_t s_off[kWin + 1];
    __shared__ int32_t s_rs[kWin];
    __shared__ int32_t s_b[kWin];
    __shared__ uint64_t s_m[kWin];
    __shared__ int64_t s_first;

    if (__hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const WideLevel me = a.lvl[L];
    const int64_t N = (int64_t)(me.packed >> 40);
    const int64_t E = (int64_t)(me.packed & kM40);
    const int64_t start = me.start;
    const int64_t nbase = start + N;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) a.lvl[L + 1].start = nbase;
    if (E == 0) return;
    const int64_t G = gridDim.x;
    const int64_t eb = E * (int64_t)blockIdx.x / G;
    const int64_t ee = E * ((int64_t)blockIdx.x + 1) / G;
    if (eb >= ee) return;

    const DistT *dist = reinterpret_cast<const DistT *>(a.dist);
    const int32_t *__restrict__ rp = a.rp;
    const int32_t *__restrict__ ci = a.ci;
    const uint32_t nl = (uint32_t)L + 1u;
    WideLevel *next = &a.lvl[L + 1];

    // largest entry index i with off[i] <= eb (64-ary search by wave 0)
    if (tid < 64) {
        int64_t lo = 0, hi = N - 1;
        while (lo < hi) {
            const int64_t p = lo + ((hi - lo) * tid) / 63;
            const bool pr = a.lo[start + p] <= eb;
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
            const int64_t q = start + i + tid;
            s_off[tid] = a.lo[q];
            s_rs[tid] = rp[a.ly[q]];
            s_b[tid] = a.lb[q];
            s_m[tid] = a.lm[q];
        }
        if (tid == 0) s_off[cnt] = (i + cnt < N) ? a.lo[start + i + cnt] : E;
        __syncthreads();
        const int64_t wlo = eb > s_off[0] ? eb : s_off[0];
        const int64_t whi = ee < s_off[cnt] ? ee : s_off[cnt];
        for (int64_t e0 = wlo; e0 < whi; e0 += (int64_t)kWG * kUnroll) {
            int32_t y[kUnroll];
            int32_t own[kUnroll];
            uint32_t d[kUnroll];
#pragma unroll
            for (int r = 0; r < kUnroll; ++r) {
                const int64_t e = e0 + tid + (int64_t)r * kWG;
                own[r] = -1;
                y[r] = 0;
                if (e < whi) {
                    int lo = 0, hi = cnt - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_off[mid] <= e) lo = mid; else hi = mid - 1;
                    }
                    own[r] = lo;
                    y[r] = ci[s_rs[lo] + (int32_t)(e - s_off[lo])];
                }
            }
#pragma unroll
            for (int r = 0; r < kUnroll; ++r) d[r] = own[r] >= 0 ? (uint32_t)dist[y[r]] : 0u;
#pragma unroll
            for (int r = 0; r < kUnroll; ++r) {
                bool p = false;
                uint64_t nw = 0;
                int32_t bb = 0, deg = 0;
                if (own[r] >= 0 && nl < d[r]) {
                    bb = s_b[own[r]];
                    uint64_t *vw = a.vis + (size_t)bb * a.vis_stride + y[r];
                    const uint64_t m = s_m[own[r]] & ~(*vw);
                    if (m) {
                        const uint64_t old = atomicOr(reinterpret_cast<unsigned long long *>(vw),
                                                      (unsigned long long)m);
                        nw = m & ~old;
                        if (nw) {
                            const int64_t c = (int64_t)(d[r] - nl);
                            deg = rp[y[r] + 1] - rp[y[r]];
                            const int64_t gb = (int64_t)bb * a.spb;
                            for (uint64_t mm = nw; mm; mm &= mm - 1) {
                                const int j = __ffsll((unsigned long long)mm) - 1;
                                atomicAdd(reinterpret_cast<unsigned long long *>(a.gain + gb + j),
                                          (unsigned long long)c);
                                if (a.edges)
                                    atomicAdd(reinterpret_cast<unsigned long long *>(a.edges + gb + j),
                                              (unsigned long long)deg);
                                if (a.visited) atomicAdd(a.visited + gb + j, 1);
                            }
                            p = true;
                        }
                    }
                }
                push_entries(a, next, nbase, p, y[r], bb, nw, deg);
            }
        }
        __syncthreads();
        if (whi >= ee || i + cnt >= N) break;
        i += cnt;
    }
}

// Return every touched word of vis to zero (entries of all levels).
__global__ void k_wide_clear(WideArgs a, int32_t nlev) {
    if (__hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const WideLevel last = a.lvl[nlev];
    int64_t tot = last.start + (int64_t)(last.packed >> 40);
    if (tot > a.cap) tot = a.cap;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x)
        a.vis[(size_t)a.lb[i] * a.vis_stride + a.ly[i]] = 0;
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

__global__ void k_set_i32(int32_t *p, int32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

}  // namespace

hipError_t launch_wide_begin(const WideArgs &a, int dist_bytes, int32_t nlev, hipStream_t s) {
    const int64_t tot = a.nsrc > nlev + 2 ? a.nsrc : nlev + 2;
    int g = (int)((tot + 255) / 256);
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_wide_zero, dim3(g), dim3(256), 0, s, a, nlev);
    const int groots = (int)((a.nsrc + 255) / 256);
    if (dist_bytes == 1)
        hipLaunchKernelGGL((k_wide_roots<uint8_t>), dim3(groots), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_wide_roots<uint16_t>), dim3(groots), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_wide_levels(const WideArgs &a, int dist_bytes, int32_t l0, int32_t l1, int grid,
                              hipStream_t s) {
    for (int32_t L = l0; L < l1; ++L) {
        if (dist_bytes == 1)
            hipLaunchKernelGGL((k_wide_level<uint8_t>), dim3(grid), dim3(kWG), 0, s, a, L);
        else
            hipLaunchKernelGGL((k_wide_level<uint16_t>), dim3(grid), dim3(kWG), 0, s, a, L);
    }
    return hipGetLastError();
}

hipError_t launch_wide_end(const WideArgs &a, int32_t nlev, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_wide_clear, dim3(grid), dim3(256), 0, s, a, nlev);
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
