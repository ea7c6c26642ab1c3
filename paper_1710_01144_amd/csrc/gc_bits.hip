// Bit-vector form of the gain (Section 4.3, "bit-parallel group closeness"):
// b^i_u has bit w set iff d(u, w) <= i.  The levels are the fixed point of
// b^i_u = b^{i-1}_u OR (OR over neighbours v of b^{i-1}_v); b^i_S has bit w
// set iff d(S, w) <= i; and the gain of u is the sum over i of
// |b^i_u AND NOT b^i_S| (the theorem of Section 4.3).  A term that is zero
// stays zero at every later level, so a candidate stops there.
//
// Layout: level l, row u, word j at bits[(l * n + u) * W + j], W = ceil(n/64);
// the b^i_S rows for i = 0 .. kBitsMaxS-1 at bs[i * W + j].
#include <hip/hip_runtime.h>

#include "gc_bits.h"

namespace gck {
namespace {

__device__ __forceinline__ int lane() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// b^0: one bit per row, on the diagonal.  One thread per word of the level.
__global__ void k_bits_identity(uint64_t *b0, int32_t n, int64_t W) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * W) return;
    const int64_t u = t / W, j = t - u * W;
    b0[t] = (u >> 6) == j ? (1ull << (u & 63)) : 0ull;
}

// b^i from b^{i-1}: one wave per (row u, 64-word chunk c); every lane ORs one
// word over u's own row and its neighbours' rows (coalesced: a row's 64 words
// are contiguous).  *changed is raised if any word differs from b^{i-1}.
__global__ __launch_bounds__(256) void k_bits_level(const int32_t *rp, const int32_t *ci, int32_t n,
                                                     int64_t W, const uint64_t *prev, uint64_t *next,
                                                     int32_t *changed) {
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t chunks = (W + 63) >> 6;
    if (wave >= (int64_t)n * chunks) return;
    const int64_t u = wave / chunks;
    const int64_t j = (wave - u * chunks) * 64 + lane();
    const bool in = j < W;
    uint64_t acc = in ? prev[u * W + j] : 0ull;
    const uint64_t old = acc;
    const int32_t e1 = rp[u + 1];
    int32_t e = rp[u];
    // eight neighbours' rows in flight at a time
    for (; e + 8 <= e1; e += 8) {
        int64_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = ci[e + q];
        if (in) {
            uint64_t x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = prev[v[q] * W + j];
#pragma unroll
            for (int q = 0; q < 8; ++q) acc |= x[q];
        }
    }
    for (; e < e1; ++e) {
        const int64_t v = ci[e];
        if (in) acc |= prev[v * W + j];
    }
    if (in) next[u * W + j] = acc;
    // one flag write per wave that changed a word
    if (__ballot(in && acc != old) != 0ull && lane() == 0) atomicOr(changed, 1);
}

// b^i_S for i = 0 .. levels-1 from d(S,.): one thread per word, which reads
// its 64 distances once and writes the word of every level.
template <typename DistT>
__global__ void k_bits_group(const DistT *dist, int32_t n, int64_t W, int32_t levels, uint64_t *bs) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= W) return;
    const int64_t w0 = j * 64;
    uint32_t d[64];
    const DistT *src = dist + w0;
    if (sizeof(DistT) == 1 && w0 + 64 <= n && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
        // a whole word's 64 one-byte distances in four 16-byte loads
        const uint4 *p = reinterpret_cast<const uint4 *>(src);
        uint32_t x[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 v = p[q];
            x[4 * q] = v.x;
            x[4 * q + 1] = v.y;
            x[4 * q + 2] = v.z;
            x[4 * q + 3] = v.w;
        }
#pragma unroll
        for (int b = 0; b < 64; ++b) d[b] = (x[b >> 2] >> (8 * (b & 3))) & 0xFFu;
    } else {
#pragma unroll
        for (int b = 0; b < 64; ++b) d[b] = w0 + b < n ? (uint32_t)src[b] : 0xFFFFFFFFu;
    }
    for (int32_t i = 0; i < levels; ++i) {
        uint64_t word = 0;
#pragma unroll
        for (int b = 0; b < 64; ++b) word |= (uint64_t)(d[b] <= (uint32_t)i) << b;
        bs[(int64_t)i * W + j] = word;
    }
}

// Gains of the candidates: one wave per candidate, the sum over levels
// i < levels_s of popcount(b^i_u AND NOT b^i_S), level i read from stored
// level min(i, levels_b - 1) (the last stored level is the fixed point),
// stopping at the first zero term.  words (optional): += the row words read.
__global__ __launch_bounds__(256) void k_bits_gains(const uint64_t *bits, int32_t n, int64_t W,
                                                     int32_t levels_b, const uint64_t *bs, int32_t levels_s,
                                                     const int32_t *cand, int64_t count, int64_t *gain,
                                                     unsigned long long *words) {
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    if (wave >= count) return;
    const int64_t u = cand[wave];
    const int ln = lane();
    int64_t total = 0;
    int32_t read = 0;
    // two levels per step (their loads overlap); the second one's term
    // counts only if the first one's was not zero
    for (int32_t i = 0; i < levels_s; i += 2) {
        const bool two = i + 1 < levels_s;
        read += two ? 2 : 1;
        const int32_t l0 = i < levels_b ? i : levels_b - 1;
        const int32_t l1 = i + 1 < levels_b ? i + 1 : levels_b - 1;
        const uint64_t *r0 = bits + ((int64_t)l0 * n + u) * W;
        const uint64_t *r1 = bits + ((int64_t)l1 * n + u) * W;
        const uint64_t *s0 = bs + (int64_t)i * W;
        const uint64_t *s1 = bs + (int64_t)(two ? i + 1 : i) * W;
        int64_t c0 = 0, c1 = 0;
#pragma unroll 4
        for (int64_t j = ln; j < W; j += 64) {
            c0 += __popcll(r0[j] & ~s0[j]);
            if (two) c1 += __popcll(r1[j] & ~s1[j]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            c0 += __shfl_xor(c0, o);
            c1 += __shfl_xor(c1, o);
        }
        if (c0 == 0) break;
        total += c0;
        if (c1 == 0) break;
        total += c1;
    }
    if (ln == 0) {
        gain[wave] = total;
        if (words) atomicAdd(words, (unsigned long long)read * (unsigned long long)W);
    }
}

}  // namespace

hipError_t launch_bits_identity(uint64_t *b0, int32_t n, hipStream_t s) {
    const int64_t W = ((int64_t)n + 63) / 64;
    const int64_t g = ((int64_t)n * W + 255) / 256;
    hipLaunchKernelGGL(k_bits_identity, dim3((unsigned)g), dim3(256), 0, s, b0, n, W);
    return hipGetLastError();
}

hipError_t launch_bits_level(const int32_t *rp, const int32_t *ci, int32_t n, const uint64_t *prev,
                             uint64_t *next, int32_t *changed, hipStream_t s) {
    const int64_t W = ((int64_t)n + 63) / 64;
    const int64_t waves = (int64_t)n * ((W + 63) / 64);
    const int64_t g = (waves * 64 + 255) / 256;
    hipLaunchKernelGGL(k_bits_level, dim3((unsigned)g), dim3(256), 0, s, rp, ci, n, W, prev, next, changed);
    return hipGetLastError();
}

hipError_t launch_bits_group(const void *dist, int dist_bytes, int32_t n, int32_t levels, uint64_t *bs,
                             hipStream_t s) {
    const int64_t W = ((int64_t)n + 63) / 64;
    const int64_t g = (W + 255) / 256;
    if (levels <= 0 || g == 0) return hipSuccess;
    if (dist_bytes == 1)
        hipLaunchKernelGGL((k_bits_group<uint8_t>), dim3((unsigned)g), dim3(256), 0, s,
                           reinterpret_cast<const uint8_t *>(dist), n, W, levels, bs);
    else
        hipLaunchKernelGGL((k_bits_group<uint16_t>), dim3((unsigned)g), dim3(256), 0, s,
                           reinterpret_cast<const uint16_t *>(dist), n, W, levels, bs);
    return hipGetLastError();
}

hipError_t launch_bits_gains(const uint64_t *bits, int32_t n, int32_t levels_b, const uint64_t *bs,
                             int32_t levels_s, const int32_t *cand, int64_t count, int64_t *gain,
                             unsigned long long *words, hipStream_t s) {
    const int64_t W = ((int64_t)n + 63) / 64;
    const int64_t g = (count * 64 + 255) / 256;
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bits_gains, dim3((unsigned)g), dim3(256), 0, s, bits, n, W, levels_b, bs, levels_s,
                       cand, count, gain, words);
    return hipGetLastError();
}

}  // namespace gck
