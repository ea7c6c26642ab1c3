// HIP kernels (gfx950) for Greedy++ group-closeness maximisation: the
// level-synchronous single-source BFS of gc_update_dist (pruned as in Section
// 4.1; full when S = {}) and small fills.  The gain, closeness and update
// launches of the greedy run on the device-wide engine of gc_wide.hip.
#include "gc_kernels.h"

namespace gck {

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

template <typename DistT>
struct DistInf;
template <>
struct DistInf<uint8_t> { static constexpr uint32_t v = 0xFFu; };
template <>
struct DistInf<uint16_t> { static constexpr uint32_t v = 0xFFFFu; };

__device__ __forceinline__ int64_t *ctr64(int32_t *ctr) {
    return reinterpret_cast<int64_t *>(ctr + C_I64_BASE);
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

// 16-byte stores over the 16-byte aligned body, single words before and after
__global__ void k_fill_u32(uint32_t *p, size_t count, uint32_t v) {
    const size_t t0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t nt = (size_t)gridDim.x * blockDim.x;
    size_t head = ((16 - ((uintptr_t)p & 15)) & 15) / 4;
    if (head > count) head = count;
    const size_t nv = (count - head) / 4;
    uint4 *q = reinterpret_cast<uint4 *>(p + head);
    const uint4 vv = make_uint4(v, v, v, v);
    for (size_t i = t0; i < nv; i += nt) q[i] = vv;
    const size_t tail = head + nv * 4;
    if (t0 < head) p[t0] = v;
    if (t0 < count - tail) p[tail + t0] = v;
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

__global__ void k_u8_to_u16(const uint8_t *in, uint16_t *out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = in[i];
        out[i] = (uint16_t)(v == 0xFFu ? 0xFFFFu : v);
    }
}

__global__ void k_copy_add_i32(const int32_t *in, int32_t *out, int64_t n, int32_t add) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i] + add;
}

}  // namespace

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
    size_t g = (count / 4 + 255) / 256;
    int grid = (int)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

hipError_t launch_u16_to_u8(const uint16_t *in, uint8_t *out, int64_t n, hipStream_t s) {
    int64_t g = (n + 255) / 256;
    int grid = (int)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
    hipLaunchKernelGGL(k_u16_to_u8, dim3(grid), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_u8_to_u16(const uint8_t *in, uint16_t *out, int64_t n, hipStream_t s) {
    int64_t g = (n + 255) / 256;
    int grid = (int)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
    hipLaunchKernelGGL(k_u8_to_u16, dim3(grid), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_copy_add_i32(const int32_t *in, int32_t *out, int64_t n, int32_t add, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    int grid = (int)(g > 4096 ? 4096 : g);
    hipLaunchKernelGGL(k_copy_add_i32, dim3(grid), dim3(256), 0, s, in, out, n, add);
    return hipGetLastError();
}

hipError_t launch_set_i64(int64_t *p, int64_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

}  // namespace gck
