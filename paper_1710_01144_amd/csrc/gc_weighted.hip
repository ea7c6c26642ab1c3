// Searches on graphs with integer edge lengths (Section 2: distances are SSSP
// distances, BFS being the unit-length case).
//
// One workgroup runs one search at a time on its own slot: n 16-byte records
// and six n-entry work lists that no other workgroup touches, so a launch
// needs no grid-wide synchronisation and every wait is a workgroup barrier.
// Workgroups take candidates from a counter until none is left.
//
// The search is bucketed label-correcting (delta-stepping): a phase with
// threshold theta relaxes, in rounds over a near list, every node whose
// tentative distance is below theta until no distance below theta changes;
// tentative distances of theta or more wait on the far list.  When a phase
// ends every node closer than theta is final (all lengths are >= 1 and every
// shorter path runs through nodes closer still), and every other node is at
// theta or more.  A round reads the near list in tiles of one node per
// thread, takes an exclusive scan of their degrees and spreads the tile's
// adjacency entries evenly over the threads (a binary search finds each
// entry's node), so a hub's row is relaxed by the whole workgroup.
//
// Modes (WMode):
//   W_GAIN   pruned search of Section 4.1: y is entered only while
//            d(u,y) < d(S,y); every node it reaches that way is exactly one
//            whose distance drops, so g(u,S) = sum over the touched nodes of
//            d(S,y) - d(u,y).
//   W_WRITE  the same search for the node just picked, then d(S,y) <- d(u,y)
//            on every touched node (the update after a pick).
//   W_CLOSE  full SSSP for the closeness search of Section 3.1: after each
//            phase, sum(settled) + theta * (n - settled) bounds F({u}) from
//            below, and the search stops once the bound exceeds the best
//            farness known (the weighted form of the BFScut bound).  With the
//            distances d0 from one landmark node, a node w the search has not
//            touched lies at least theta + d0(w) - M from u, M the largest d0
//            over the touched nodes (the triangle inequality through the
//            first touched node on a shortest path), which adds
//            T0[M] = sum_w max(0, d0(w) - M) to the bound.
#include "gc_weighted.h"

#include <stdint.h>

#include <algorithm>

namespace gck {
namespace {

constexpr uint32_t kEncZero = 0x7FFFFFFFu;  // enc of distance 0; enc 0 = unreached

__device__ __forceinline__ uint32_t ld_acq(const uint32_t *p) {
    // records change only through atomics, which the L2 performs: read them
    // there too, never from a vector L1 line that an atomic did not update
    return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t dist_of(uint32_t enc) { return (int32_t)(kEncZero - enc); }

// exclusive prefix sum of v over the workgroup; the total goes to *total
template <int BS>
__device__ __forceinline__ int32_t block_exscan(int32_t v, int32_t *s_wave, int32_t *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    int32_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) {
        const int32_t t = s_wave[i];
        base += i < wave ? t : 0;
        tot += t;
    }
    *total = tot;
    __syncthreads();  // s_wave is reused by the next call
    return base + x - v;
}

template <int BS>
__device__ __forceinline__ int64_t block_sum64(int64_t v, int64_t *s_red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) t += s_red[i];
    __syncthreads();
    return t;
}

template <int BS>
__global__ __launch_bounds__(BS) void k_wsearch(WArgs a) {
    __shared__ int32_t s_row[BS];
    __shared__ int32_t s_d[BS];
    __shared__ int32_t s_off[BS + 1];
    __shared__ int32_t s_wave[BS / 64];
    __shared__ int64_t s_red[BS / 64];
    __shared__ int32_t s_ci, s_ncur, s_nnext, s_nfar, s_nfar2, s_ntouch, s_nset, s_minfar, s_cut, s_maxd0;

    const int tid = threadIdx.x;
    const int32_t n = a.n;
    const bool close = a.mode == W_CLOSE;
    WRec *rec = a.rec + (size_t)blockIdx.x * (size_t)n;
    uint32_t *enc = a.enc + (size_t)blockIdx.x * (size_t)n;
    int32_t *lists = a.lists + (size_t)blockIdx.x * kWLists * (size_t)n;
    int32_t *const touch = lists + 4 * (size_t)n;
    int32_t *const setl = lists + 5 * (size_t)n;

    for (;;) {
        if (tid == 0) s_ci = (int32_t)atomicAdd(a.next, 1u);
        __syncthreads();
        const int32_t ci = s_ci;
        if (ci >= a.count) return;
        const int32_t u = a.cand[ci];
        if (u < 0 || u >= n || (!close && a.dS[u] <= 0)) {
            // not a node, or already in S: gain 0 (a closeness search: no value)
            if (tid == 0) {
                a.out[ci] = close ? -1 : 0;
                if (a.edges) a.edges[ci] = 0;
                if (a.visited) a.visited[ci] = 0;
            }
            __syncthreads();
            continue;
        }
        int32_t *cur = lists, *nxt = lists + n, *far = lists + 2 * (size_t)n, *far2 = lists + 3 * (size_t)n;
        if (tid == 0) {
            enc[u] = kEncZero;
            rec[u] = WRec{1u, 0u, 0u, 0u};
            cur[0] = u;
            touch[0] = u;
            s_ncur = 1;
            s_ntouch = 1;
            s_nfar = 0;
            s_nset = 0;
            s_cut = 0;
            s_maxd0 = a.d0 ? a.d0[u] : 0;
        }
        int32_t theta = a.delta;
        uint32_t it = 1, ph = 1;
        int64_t set_sum = 0, set_cnt = 0;  // closeness: settled nodes (uniform)
        // the source's record is written before any atomic on it; a slot is
        // private to its workgroup within a launch, so a workgroup-scope fence
        // is enough (a device-scope one would write back the L2 of the chip's
        // dies on every search)
        __threadfence_block();
        __syncthreads();
        for (;;) {
            // ---- rounds over the near list until nothing below theta changes
            for (;;) {
                const int32_t ncur = s_ncur;
                if (ncur == 0) break;
                if (a.max_rounds && it > a.max_rounds) {
                    // watchdog: give the search up (it is counted as cut) and
                    // let the host report it
                    if (tid == 0) {
                        s_cut = 1;
                        atomicOr(a.flags, 2);
                    }
                    __syncthreads();
                    break;
                }
                ++it;
                __syncthreads();  // every thread has read s_ncur
                if (tid == 0) s_nnext = 0;
                for (int32_t base = 0; base < ncur; base += BS) {
                    const int32_t i = base + tid;
                    int32_t x = 0, deg = 0, dx = 0, row = 0;
                    if (i < ncur) {
                        x = cur[i];
                        dx = dist_of(ld_acq(&enc[x]));
                        row = a.rp[x];
                        deg = a.rp[x + 1] - row;
                        if (close && atomicExch(&rec[x].phase, ph) != ph) {
                            const int32_t p = atomicAdd(&s_nset, 1);
                            setl[p] = x;
                        }
                    }
                    s_row[tid] = row;
                    s_d[tid] = dx;
                    int32_t tot;
                    const int32_t off = block_exscan<BS>(deg, s_wave, &tot);
                    s_off[tid] = off;
                    if (tid == 0) s_off[BS] = tot;
                    __syncthreads();
                    for (int32_t e = tid; e < tot; e += BS) {
                        // the tile entry whose adjacency range holds e: the
                        // largest j with s_off[j] <= e (s_off[0] = 0 <= e < s_off[BS])
                        int32_t lo = 0, hi = BS;
                        while (hi - lo > 1) {
                            const int32_t mid = (lo + hi) >> 1;
                            if (s_off[mid] <= e) lo = mid;
                            else hi = mid;
                        }
                        const int64_t idx = (int64_t)s_row[lo] + (e - s_off[lo]);
                        const int32_t y = a.ci[idx];
                        const int32_t nd = s_d[lo] + (int32_t)a.w[idx];
                        if (!close && nd >= a.dS[y]) continue;  // S is at least as close
                        const uint32_t e_new = kEncZero - (uint32_t)nd;
                        if (ld_acq(&enc[y]) >= e_new) continue;
                        const uint32_t old = atomicMax(&enc[y], e_new);
                        if (old >= e_new) continue;
                        if (old == 0u) {
                            const int32_t t = atomicAdd(&s_ntouch, 1);
                            touch[t] = y;
                            if (close && a.d0) atomicMax(&s_maxd0, a.d0[y]);
                        }
                        if (nd < theta) {
                            if (atomicExch(&rec[y].mark, it) != it) {
                                const int32_t q = atomicAdd(&s_nnext, 1);
                                nxt[q] = y;
                            }
                        } else if (atomicExch(&rec[y].far, 1u) == 0u) {
                            const int32_t q = atomicAdd(&s_nfar, 1);
                            far[q] = y;
                        }
                    }
                    __syncthreads();  // the tile's LDS is rewritten next
                }
                if (tid == 0) s_ncur = s_nnext;
                int32_t *t = cur;
                cur = nxt;
                nxt = t;
                __syncthreads();
            }
            // ---- phase end: every node closer than theta is settled
            if (close) {
                const int32_t ns = s_nset;
                int64_t part = 0;
                for (int32_t i = tid; i < ns; i += BS) part += dist_of(ld_acq(&enc[setl[i]]));
                set_sum += block_sum64<BS>(part, s_red);
                set_cnt += ns;
                if (tid == 0) {
                    s_nset = 0;
                    if (set_cnt < n) {
                        int64_t lim = a.thr;
                        if (a.best) {
                            const int64_t b = (int64_t)__hip_atomic_load(a.best, __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_AGENT);
                            lim = b < lim ? b : lim;
                        }
                        // every node not settled is at theta or more; one that is
                        // not even touched is reached through a touched node y, so
                        // it is also at theta + d0(w) - d0(y) >= theta + d0(w) - maxd0
                        int64_t lb = set_sum + (int64_t)theta * (int64_t)(n - set_cnt);
                        if (a.t0) lb += a.t0[s_maxd0 < a.t0_len ? s_maxd0 : a.t0_len - 1];
                        if (lb > lim) s_cut = 1;
                    }
                }
                __syncthreads();
            }
            if (s_cut || s_nfar == 0) break;
            // ---- the far list into the next phase
            const int32_t th_old = theta;
            theta += a.delta;
            const int32_t nf = s_nfar;
            __syncthreads();  // every thread has read s_nfar
            if (tid == 0) {
                s_nfar2 = 0;
                s_ncur = 0;
                s_minfar = 0x7FFFFFFF;
            }
            __syncthreads();
            for (int32_t i = tid; i < nf; i += BS) {
                const int32_t y = far[i];
                const int32_t d = dist_of(ld_acq(&enc[y]));
                if (d < th_old) continue;  // settled in an earlier phase
                if (d < theta) {
                    const int32_t q = atomicAdd(&s_ncur, 1);
                    cur[q] = y;
                } else {
                    const int32_t q = atomicAdd(&s_nfar2, 1);
                    far2[q] = y;
                    atomicMin(&s_minfar, d);
                }
            }
            __syncthreads();
            const int32_t nf2 = s_nfar2;
            if (s_ncur == 0 && nf2 > 0) {
                // nothing in [th_old, theta): move theta past the nearest waiting node
                theta = s_minfar + a.delta;
                __syncthreads();  // every thread has read s_minfar
                if (tid == 0) s_nfar = 0;
                __syncthreads();
                for (int32_t i = tid; i < nf2; i += BS) {
                    const int32_t y = far2[i];
                    const int32_t d = dist_of(ld_acq(&enc[y]));
                    if (d < theta) {
                        const int32_t q = atomicAdd(&s_ncur, 1);
                        cur[q] = y;
                    } else {
                        const int32_t q = atomicAdd(&s_nfar, 1);
                        far[q] = y;
                    }
                }
            } else {
                int32_t *t = far;
                far = far2;
                far2 = t;
                if (tid == 0) s_nfar = nf2;
            }
            ++ph;
            __syncthreads();
        }
        // ---- results, then every touched record back to zero
        const int32_t nt = s_ntouch;
        int64_t gsum = 0, esum = 0;
        for (int32_t i = tid; i < nt; i += BS) {
            const int32_t y = touch[i];
            const int32_t d = dist_of(ld_acq(&enc[y]));
            if (!close) {
                gsum += (int64_t)a.dS[y] - d;
                if (a.mode == W_WRITE) a.dS[y] = d;
            }
            esum += a.rp[y + 1] - a.rp[y];
            enc[y] = 0u;
            rec[y] = WRec{0u, 0u, 0u, 0u};
        }
        gsum = block_sum64<BS>(gsum, s_red);
        esum = block_sum64<BS>(esum, s_red);
        if (tid == 0) {
            if (close) {
                const bool done = !s_cut;
                a.out[ci] = done ? set_sum : -1;
                if (done && set_cnt != n) atomicOr(a.flags, 1);
                if (done && a.best) atomicMin(a.best, (unsigned long long)set_sum);
            } else {
                a.out[ci] = gsum;
            }
            if (a.edges) a.edges[ci] = esum;
            if (a.visited) a.visited[ci] = nt;
        }
        __threadfence_block();  // the zeroed records are written before the next search's atomics
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_wargmin(const int64_t *out, const int32_t *cand, int32_t count,
                                                  int64_t *res) {
    __shared__ int64_t s_f[1024];
    __shared__ int32_t s_i[1024];
    int64_t bf = INT64_MAX;
    int32_t bi = INT32_MAX;
    for (int32_t i = threadIdx.x; i < count; i += 1024) {
        const int64_t f = out[i];
        const int32_t id = cand[i];
        if (f >= 0 && (f < bf || (f == bf && id < bi))) {
            bf = f;
            bi = id;
        }
    }
    s_f[threadIdx.x] = bf;
    s_i[threadIdx.x] = bi;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const int64_t f = s_f[threadIdx.x + s];
            const int32_t id = s_i[threadIdx.x + s];
            if (f < s_f[threadIdx.x] || (f == s_f[threadIdx.x] && id < s_i[threadIdx.x])) {
                s_f[threadIdx.x] = f;
                s_i[threadIdx.x] = id;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool none = s_i[0] == INT32_MAX;
        res[0] = none ? -1 : s_f[0];
        res[1] = none ? -1 : s_i[0];
    }
}

__global__ __launch_bounds__(256) void k_wsum(const int32_t *d, int32_t n, unsigned long long *sum) {
    __shared__ int64_t s_red[4];
    int64_t v = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) v += d[i];
    v = block_sum64<256>(v, s_red);
    if (threadIdx.x == 0 && v != 0) atomicAdd(sum, (unsigned long long)v);
}

__global__ void k_wzero64(unsigned long long *p) { *p = 0ull; }

__global__ void k_wsub(int64_t *far, const int64_t *gain) { *far -= *gain; }

__global__ __launch_bounds__(256) void k_wmax(const int32_t *d, int32_t n, int32_t *mx) {
    int32_t v = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        v = d[i] > v ? d[i] : v;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t y = __shfl_down(v, o, 64);
        v = y > v ? y : v;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(mx, v);
}

__global__ __launch_bounds__(256) void k_whist(const int32_t *d, int32_t n, uint32_t *hist) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        atomicAdd(&hist[d[i]], 1u);
}

}  // namespace

hipError_t launch_wsearch(const WArgs &a, int32_t slots, int32_t threads, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    const int32_t grid = slots < a.count ? slots : a.count;
    if (threads == 1024) hipLaunchKernelGGL(k_wsearch<1024>, dim3(grid), dim3(1024), 0, s, a);
    else hipLaunchKernelGGL(k_wsearch<256>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_wsearch_one(const WArgs &a, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wsearch<1024>, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_wargmin(const int64_t *out, const int32_t *cand, int32_t count, int64_t *res, hipStream_t s) {
    hipLaunchKernelGGL(k_wargmin, dim3(1), dim3(1024), 0, s, out, cand, count, res);
    return hipGetLastError();
}

hipError_t launch_wsum(const int32_t *d, int32_t n, unsigned long long *sum, hipStream_t s) {
    hipLaunchKernelGGL(k_wzero64, dim3(1), dim3(1), 0, s, sum);
    const int32_t grid = (int32_t)std::min<int64_t>(1024, ((int64_t)n + 255) / 256);
    hipLaunchKernelGGL(k_wsum, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, d, n, sum);
    return hipGetLastError();
}

hipError_t launch_wsub(int64_t *far, const int64_t *gain, hipStream_t s) {
    hipLaunchKernelGGL(k_wsub, dim3(1), dim3(1), 0, s, far, gain);
    return hipGetLastError();
}

hipError_t launch_wmax(const int32_t *d, int32_t n, int32_t *mx, hipStream_t s) {
    const int32_t grid = (int32_t)std::min<int64_t>(1024, ((int64_t)n + 255) / 256);
    hipLaunchKernelGGL(k_wmax, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, d, n, mx);
    return hipGetLastError();
}

hipError_t launch_whist(const int32_t *d, int32_t n, uint32_t *hist, hipStream_t s) {
    const int32_t grid = (int32_t)std::min<int64_t>(1024, ((int64_t)n + 255) / 256);
    hipLaunchKernelGGL(k_whist, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, d, n, hist);
    return hipGetLastError();
}

}  // namespace gck
