// HIP kernels (gfx950) for Greedy++ group-closeness maximisation.
//
//  * k_engine: bit-parallel multi-source BFS, one workgroup per batch of 64
//    sources (one bit per source in a uint64 word per node).
//      gain mode       -- pruned BFS of Section 4.1: a node y reached at
//                         level L by source v is entered only if L < d(S,y);
//                         it then adds d(S,y) - L to g(v,S) (the summand of
//                         the gain sum in the proof of the Section 4.3
//                         theorem).  Nodes failing the test are never marked,
//                         so the prune test costs one byte read per edge.
//      closeness mode  -- full BFS that keeps, per source, the distance sum,
//                         the reached count and the adjacency size of the
//                         last level, and drops a source once a lower bound
//                         on its farness exceeds the best farness known
//                         (BFScut of Section 3.1).
//  * k_bfs_*: level-synchronous single-source BFS over the whole device for
//    the d(S,.) update after a pick (pruned as in Section 4.1; full when
//    S = {}).
//
// Memory model: every per-batch array lives in a per-workgroup slot that only
// that workgroup touches during a launch, so __syncthreads() orders all its
// accesses; cross-workgroup state is limited to device-scope atomics on the
// counter block.
#include "gc_kernels.h"

namespace gck {

SlotLayout slot_layout(int64_t n) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    SlotLayout L;
    size_t o = 0;
    const size_t n8 = al((size_t)n * 8), n4 = al((size_t)n * 4);
    L.vis = o; o += n8;
    L.next = o; o += n8;
    L.tq = o; o += n4;
    L.uq = o; o += n4;
    L.qv0 = o; o += n4;
    L.qv1 = o; o += n4;
    L.qm0 = o; o += n8;
    L.qm1 = o; o += n8;
    L.bytes = o;
    return L;
}

namespace {

__device__ __forceinline__ int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ int bits_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Wave-aggregated append: every active lane calls it; lanes with p get
// consecutive slots after one atomic on the counter.  Returns -1 for !p.
__device__ __forceinline__ int wave_push(bool p, int *counter) {
    const uint64_t bal = __ballot(p);
    if (bal == 0) return -1;
    const int leader = __ffsll((unsigned long long)bal) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (int)__popcll(bal));
    base = __shfl(base, leader);
    return p ? base + bits_below(bal) : -1;
}

// Exclusive block scan over kWG threads; `total` receives the block sum.
__device__ __forceinline__ int block_excl_scan(int v, int *s_wave, int &total) {
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[w] = x;
    __syncthreads();
    int pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWG / 64; ++i) {
        int t = s_wave[i];
        pre += (i < w) ? t : 0;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

template <typename DistT>
struct DistInf;
template <>
struct DistInf<uint8_t> { static constexpr uint32_t v = 0xFFu; };
template <>
struct DistInf<uint16_t> { static constexpr uint32_t v = 0xFFFFu; };

__device__ __forceinline__ int64_t *ctr64(int32_t *ctr) {
    return reinterpret_cast<int64_t *>(ctr + C_I64_BASE);
}

// MODE 0: gains (pruned by dist); MODE 1: closeness with cut.
template <typename DistT, int MODE, bool STATS>
__global__ __launch_bounds__(kWG) void k_engine(EngineArgs a, SlotLayout lay) {
    __shared__ unsigned long long s_acc[kSrc];   // gain | distance sum
    __shared__ unsigned long long s_acc2[kSrc];  // edges | adjacency of last level
    __shared__ unsigned int s_acc3[kSrc];        // |V(v)| | reached
    __shared__ int s_off[kWG];
    __shared__ int s_rs[kWG];
    __shared__ unsigned long long s_m[kWG];
    __shared__ int s_wave[kWG / 64];
    __shared__ int s_cntT, s_cntQ, s_cntU, s_batch;
    __shared__ unsigned long long s_active;
    __shared__ unsigned long long s_done;

    const int tid = threadIdx.x;
    char *slot = a.slots.base + (size_t)blockIdx.x * a.slots.stride;
    uint64_t *vis = reinterpret_cast<uint64_t *>(slot + lay.vis);
    unsigned long long *nxt = reinterpret_cast<unsigned long long *>(slot + lay.next);
    int32_t *tq = reinterpret_cast<int32_t *>(slot + lay.tq);
    int32_t *uq = reinterpret_cast<int32_t *>(slot + lay.uq);
    int32_t *qv0 = reinterpret_cast<int32_t *>(slot + lay.qv0);
    int32_t *qv1 = reinterpret_cast<int32_t *>(slot + lay.qv1);
    uint64_t *qm0 = reinterpret_cast<uint64_t *>(slot + lay.qm0);
    uint64_t *qm1 = reinterpret_cast<uint64_t *>(slot + lay.qm1);
    const DistT *dist = reinterpret_cast<const DistT *>(a.dist);
    const int32_t *__restrict__ rp = a.rp;
    const int32_t *__restrict__ ci = a.ci;
    const int nbatch = (a.nsrc + kSrc - 1) / kSrc;
    int64_t *best_far = ctr64(a.ctr) + L_BEST_FAR;

    for (;;) {
        if (tid == 0) {
            s_batch = atomicAdd(&a.ctr[C_GAIN_NEXT], 1);
            s_cntT = 0;
            s_cntQ = 0;
            s_cntU = 0;
            s_done = 0;
        }
        if (tid < kSrc) {
            s_acc[tid] = 0;
            s_acc2[tid] = 0;
            s_acc3[tid] = 0;
        }
        __syncthreads();
        const int b = s_batch;
        if (b >= nbatch) break;
        const int base = b * kSrc;
        const int nb = min(kSrc, a.nsrc - base);
        if (tid == 0) s_active = (nb == 64) ? ~0ull : ((1ull << nb) - 1ull);

        // level 0: the roots.  In gain mode a root already in S (d = 0) is inert.
        {
            bool p = false;
            int v = 0;
            if (tid < nb) {
                v = a.src[base + tid];
                const bool alive = (MODE == 1) || ((uint32_t)dist[v] > 0u);
                if (alive) {
                    const unsigned long long old = atomicOr(&nxt[v], 1ull << tid);
                    p = (old == 0ull);
                }
            }
            const int pos = wave_push(p, &s_cntT);
            if (p) tq[pos] = v;
        }
        __syncthreads();

        int L = 0;
        int cur = 0;
        for (;;) {
            // ---- settle the nodes first reached at distance L
            int32_t *qv = cur ? qv1 : qv0;
            uint64_t *qm = cur ? qm1 : qm0;
            const int tn = s_cntT;
            for (int i0 = 0; i0 < tn; i0 += kWG) {
                const int i = i0 + tid;
                const bool valid = i < tn;
                int y = 0;
                uint64_t nw = 0, vs = 0;
                if (valid) {
                    y = tq[i];
                    nw = atomicExch(&nxt[y], 0ull);
                    vs = vis[y];
                    nw &= ~vs;
                    vis[y] = vs | nw;
                }
                const bool pu = valid && vs == 0 && nw != 0;
                const int pos = wave_push(pu, &s_cntU);
                if (pu) uq[pos] = y;
                if (valid && nw) {
                    if (MODE == 0) {
                        const unsigned long long c = (uint32_t)dist[y] - (uint32_t)L;
                        const unsigned long long dg = STATS ? (unsigned long long)(rp[y + 1] - rp[y]) : 0ull;
                        for (uint64_t m = nw; m; m &= m - 1) {
                            const int j = __ffsll((unsigned long long)m) - 1;
                            atomicAdd(&s_acc[j], c);
                            if (STATS) {
                                atomicAdd(&s_acc2[j], dg);
                                atomicAdd(&s_acc3[j], 1u);
                            }
                        }
                    } else {
                        const unsigned long long dg =
                            (unsigned long long)(rp[y + 1] - rp[y] - (L > 0 ? 1 : 0));
                        for (uint64_t m = nw; m; m &= m - 1) {
                            const int j = __ffsll((unsigned long long)m) - 1;
                            atomicAdd(&s_acc[j], (unsigned long long)L);
                            atomicAdd(&s_acc2[j], dg);
                            atomicAdd(&s_acc3[j], 1u);
                        }
                    }
                }
                const bool pq = valid && nw != 0;
                const int pos2 = wave_push(pq, &s_cntQ);
                if (pq) {
                    qv[pos2] = y;
                    qm[pos2] = nw;
                }
            }
            __syncthreads();

            if (MODE == 1) {
                // BFScut test per live source after completing level L:
                // all nodes at distance <= L are known; at most ef of the
                // remaining rem nodes are at distance L+1, the rest >= L+2.
                if (tid < nb && ((s_active >> tid) & 1ull)) {
                    const int64_t reached = (int64_t)s_acc3[tid];
                    const int64_t sum = (int64_t)s_acc[tid];
                    const int64_t ef = (int64_t)s_acc2[tid];
                    const int64_t rem = (int64_t)a.n - reached;
                    if (rem == 0) {
                        a.out_gain[base + tid] = sum;
                        atomicMin(reinterpret_cast<unsigned long long *>(best_far),
                                  (unsigned long long)sum);
                        atomicOr(&s_done, 1ull << tid);
                        atomicAnd(&s_active, ~(1ull << tid));
                    } else {
                        const int64_t near = ef < rem ? ef : rem;
                        const int64_t lb = sum + (int64_t)(L + 1) * near + (int64_t)(L + 2) * (rem - near);
                        const int64_t best = (int64_t)__hip_atomic_load(
                            reinterpret_cast<unsigned long long *>(best_far), __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
                        if (lb > best) atomicAnd(&s_active, ~(1ull << tid));
                    }
                }
                if (tid < kSrc) s_acc2[tid] = 0;
                __syncthreads();
            }

            const int qn = s_cntQ;
            const uint64_t act = (MODE == 1) ? s_active : ~0ull;
            __syncthreads();
            if (tid == 0) {
                s_cntT = 0;
                s_cntQ = 0;
            }
            if (qn == 0 || act == 0ull) break;
            __syncthreads();

            // ---- expand the frontier at distance L (edge-balanced in chunks)
            for (int c0 = 0; c0 < qn; c0 += kWG) {
                const int i = c0 + tid;
                int deg = 0, rs = 0;
                uint64_t m = 0;
                if (i < qn) {
                    const int x = qv[i];
                    m = qm[i] & act;
                    if (m) {
                        rs = rp[x];
                        deg = rp[x + 1] - rs;
                    }
                }
                int total;
                const int off = block_excl_scan(deg, s_wave, total);
                s_off[tid] = off;
                s_rs[tid] = rs;
                s_m[tid] = m;
                __syncthreads();
                const int cnt = min(kWG, qn - c0);
                for (int e0 = 0; e0 < total; e0 += kWG) {
                    const int e = e0 + tid;
                    bool p = false;
                    int y = 0;
                    if (e < total) {
                        int lo = 0, hi = cnt - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (s_off[mid] <= e) lo = mid; else hi = mid - 1;
                        }
                        y = ci[s_rs[lo] + (e - s_off[lo])];
                        uint64_t mm = s_m[lo];
                        bool ok = true;
                        if (MODE == 0) ok = (uint32_t)(L + 1) < (uint32_t)dist[y];
                        if (ok) {
                            mm &= ~vis[y];
                            if (mm) {
                                const unsigned long long old = atomicOr(&nxt[y], (unsigned long long)mm);
                                p = (old == 0ull);
                            }
                        }
                    }
                    const int pos = wave_push(p, &s_cntT);
                    if (p) tq[pos] = y;
                }
                __syncthreads();
            }
            ++L;
            cur ^= 1;
        }

        if (tid < nb) {
            if (MODE == 0) {
                a.out_gain[base + tid] = (int64_t)s_acc[tid];
                if (STATS) {
                    if (a.out_edges) a.out_edges[base + tid] = (int64_t)s_acc2[tid];
                    if (a.out_vis) a.out_vis[base + tid] = (int32_t)s_acc3[tid];
                }
            } else if (!((s_done >> tid) & 1ull)) {
                a.out_gain[base + tid] = -1;  // cut: cannot beat the best farness
            }
        }
        const int un = s_cntU;
        for (int i = tid; i < un; i += kWG) vis[uq[i]] = 0;
        __syncthreads();
    }

    if (tid == 0) {
        const int d = atomicAdd(&a.ctr[C_GAIN_DONE], 1);
        if (d == (int)gridDim.x - 1) {
            atomicExch(&a.ctr[C_GAIN_NEXT], 0);
            atomicExch(&a.ctr[C_GAIN_DONE], 0);
        }
    }
}

// ------------------------------------------------------- level BFS kernels

enum : int { C_BFS_FULL = 7 };

template <typename DistT>
__global__ void k_bfs_init(BfsArgs a, int32_t root) {
    const size_t words = ((size_t)a.n + 31) / 32;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words;
         i += (size_t)gridDim.x * blockDim.x)
        a.claim[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DistT *dist = reinterpret_cast<DistT *>(a.dist);
        const uint32_t d0 = dist[root];
        const int full = (d0 == DistInf<DistT>::v) ? 1 : 0;
        a.ctr[C_BFS_FULL] = full;
        a.ctr[C_BFS_CNT0 + 1] = 0;
        a.ctr[C_BFS_CNT0 + 2] = 0;
        a.ctr[C_BFS_LAST] = 0;
        int64_t *c64 = ctr64(a.ctr);
        if (d0 > 0u) {
            dist[root] = 0;
            a.q0[0] = root;
            a.ctr[C_BFS_CNT0 + 0] = 1;
            a.ctr[C_BFS_CLAIMED] = 1;
            c64[L_BFS_SUM] = full ? 0 : (int64_t)d0;
        } else {
            a.ctr[C_BFS_CNT0 + 0] = 0;
            a.ctr[C_BFS_CLAIMED] = 0;
            c64[L_BFS_SUM] = 0;
        }
    }
}

template <typename DistT>
__global__ __launch_bounds__(256) void k_bfs_level(BfsArgs a, int32_t level) {
    const int32_t *qin = (level & 1) ? a.q1 : a.q0;
    int32_t *qout = (level & 1) ? a.q0 : a.q1;
    int32_t *cin = &a.ctr[C_BFS_CNT0 + level % 3];
    int32_t *cout = &a.ctr[C_BFS_CNT0 + (level + 1) % 3];
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctr[C_BFS_CNT0 + (level + 2) % 3] = 0;
    const int nin = __hip_atomic_load(cin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (nin == 0) return;
    DistT *dist = reinterpret_cast<DistT *>(a.dist);
    const int full = a.ctr[C_BFS_FULL];
    const uint32_t nl = (uint32_t)level + 1u;
    const int lane = lane_id();
    const int wave = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
    const int nwaves = (int)((gridDim.x * (size_t)blockDim.x) >> 6);
    int64_t acc = 0;
    int claimed = 0;
    for (int i = wave; i < nin; i += nwaves) {
        const int x = qin[i];
        const int rs = a.rp[x], re = a.rp[x + 1];
        for (int e0 = rs; e0 < re; e0 += 64) {
            const int e = e0 + lane;
            bool p = false;
            int y = 0;
            if (e < re) {
                y = a.ci[e];
                const uint32_t dy = dist[y];
                if (nl < dy) {
                    const uint32_t bit = 1u << (y & 31);
                    const uint32_t old = atomicOr(&a.claim[y >> 5], bit);
                    if (!(old & bit)) {
                        p = true;
                        dist[y] = (DistT)nl;
                        acc += full ? (int64_t)nl : (int64_t)(dy - nl);
                        claimed += 1;
                    }
                }
            }
            const int pos = wave_push(p, cout);
            if (p) qout[pos] = y;
        }
    }
    // wave reduction of the contributions
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        acc += __shfl_xor(acc, o);
        claimed += __shfl_xor(claimed, o);
    }
    if (lane == 0 && claimed) {
        atomicAdd(reinterpret_cast<unsigned long long *>(ctr64(a.ctr) + L_BFS_SUM),
                  (unsigned long long)acc);
        atomicAdd(&a.ctr[C_BFS_CLAIMED], claimed);
        atomicMax(&a.ctr[C_BFS_LAST], (int)nl);
    }
}

__global__ void k_bfs_finish(BfsArgs a, int64_t *far) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t s = ctr64(a.ctr)[L_BFS_SUM];
        *far = a.ctr[C_BFS_FULL] ? s : (*far - s);
    }
}

__global__ void k_fill_u32(uint32_t *p, size_t count, uint32_t v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_u16_to_u8(const uint16_t *in, uint8_t *out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = in[i];
        out[i] = (uint8_t)(v >= 0xFFu ? 0xFFu : v);
    }
}

__global__ void k_set_i64(int64_t *p, int64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

}  // namespace

hipError_t launch_gain(const EngineArgs &a, int dist_bytes, int grid, hipStream_t s) {
    const SlotLayout lay = slot_layout(a.n);
    const bool stats = a.out_edges || a.out_vis;
    if (dist_bytes == 1) {
        if (stats) hipLaunchKernelGGL((k_engine<uint8_t, 0, true>), dim3(grid), dim3(kWG), 0, s, a, lay);
        else hipLaunchKernelGGL((k_engine<uint8_t, 0, false>), dim3(grid), dim3(kWG), 0, s, a, lay);
    } else {
        if (stats) hipLaunchKernelGGL((k_engine<uint16_t, 0, true>), dim3(grid), dim3(kWG), 0, s, a, lay);
        else hipLaunchKernelGGL((k_engine<uint16_t, 0, false>), dim3(grid), dim3(kWG), 0, s, a, lay);
    }
    return hipGetLastError();
}

hipError_t launch_closeness(const EngineArgs &a, int grid, hipStream_t s) {
    const SlotLayout lay = slot_layout(a.n);
    hipLaunchKernelGGL((k_engine<uint16_t, 1, false>), dim3(grid), dim3(kWG), 0, s, a, lay);
    return hipGetLastError();
}

hipError_t launch_bfs_init(const BfsArgs &a, int dist_bytes, int32_t root, hipStream_t s) {
    const size_t words = ((size_t)a.n + 31) / 32;
    int grid = (int)((words + 255) / 256);
    if (grid < 1) grid = 1;
    if (grid > 1024) grid = 1024;
    if (dist_bytes == 1) hipLaunchKernelGGL((k_bfs_init<uint8_t>), dim3(grid), dim3(256), 0, s, a, root);
    else hipLaunchKernelGGL((k_bfs_init<uint16_t>), dim3(grid), dim3(256), 0, s, a, root);
    return hipGetLastError();
}

hipError_t launch_bfs_level(const BfsArgs &a, int dist_bytes, int32_t level, int grid,
                            hipStream_t s) {
    if (dist_bytes == 1) hipLaunchKernelGGL((k_bfs_level<uint8_t>), dim3(grid), dim3(256), 0, s, a, level);
    else hipLaunchKernelGGL((k_bfs_level<uint16_t>), dim3(grid), dim3(256), 0, s, a, level);
    return hipGetLastError();
}

hipError_t launch_bfs_finish(const BfsArgs &a, int64_t *d_far, hipStream_t s) {
    hipLaunchKernelGGL(k_bfs_finish, dim3(1), dim3(64), 0, s, a, d_far);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, size_t count, uint32_t v, hipStream_t s) {
    if (count == 0) return hipSuccess;
    size_t g = (count + 255) / 256;
    int grid = (int)(g > 4096 ? 4096 : g);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

hipError_t launch_u16_to_u8(const uint16_t *in, uint8_t *out, int64_t n, hipStream_t s) {
    int64_t g = (n + 255) / 256;
    int grid = (int)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
    hipLaunchKernelGGL(k_u16_to_u8, dim3(grid), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_set_i64(int64_t *p, int64_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

}  // namespace gck
