// Candidate-ordering MLP for the lazy greedy loop (gfx950).
//
// 8 node features -> 64 -> 64 -> 1, ReLU.  Weights are bfloat16, biases and
// accumulation float32.  Rounding points (shared with the float64 reference):
//   x   = bf16(feature)
//   h1  = bf16(relu(W1 x + b1))        (dot products summed in index order)
//   h2  = bf16(relu(W2 h1 + b2))
//   out = W3 h2 + b3                   (float32, the predicted log2(1 + gain))
// Training minimises the mean squared error against log2(1 + exact gain) with
// Adam on float32 master weights; the bf16 copy is re-derived after each step.
// The network only orders exact evaluations: it never changes a pick.
#include <hip/hip_runtime.h>
#include <math.h>

#include "gc_kernels.h"
#include "gc_mlp.h"

namespace gck {
namespace {

constexpr int IN = kMlpIn, H = kMlpHidden;

__device__ __forceinline__ float bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return x;  // inf / nan unchanged
    u += 0x7fffu + ((u >> 16) & 1u);                   // round to nearest, ties to even
    return __uint_as_float(u & 0xffff0000u);
}
__device__ __forceinline__ uint16_t to_bf16(float x) {
    return (uint16_t)(__float_as_uint(bf16_round(x)) >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// The inference block (see gc_mlp.h for the byte layout) staged in LDS as floats.
struct SParams {
    float w1[H * IN];
    float w2[H * H];
    float w3[H];
    float b1[H];
    float b2[H];
    float b3;
};

__device__ void stage_params(const MlpBlock *p, SParams *sp) {
    for (int i = threadIdx.x; i < H * IN; i += blockDim.x) sp->w1[i] = from_bf16(p->w1[i]);
    for (int i = threadIdx.x; i < H * H; i += blockDim.x) sp->w2[i] = from_bf16(p->w2[i]);
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
        sp->w3[i] = from_bf16(p->w3[i]);
        sp->b1[i] = p->b1[i];
        sp->b2[i] = p->b2[i];
    }
    if (threadIdx.x == 0) sp->b3 = p->b3;
    __syncthreads();
}

// One thread per sample.  h1/h2 (count x 64) are stored when non-null.
// score: when non-null, score[s] = min(2^out - 1, ub[s]) (ub non-null) --
// the candidate key of the learned order.
__global__ __launch_bounds__(256) void k_mlp_forward(const MlpBlock *p, const float *x, int32_t count,
                                                     float *out, float *h1s, float *h2s,
                                                     const int64_t *ub, const int32_t *cand,
                                                     float *score) {
    __shared__ SParams sp;
    stage_params(p, &sp);
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    float xi[IN];
#pragma unroll
    for (int i = 0; i < IN; ++i) xi[i] = bf16_round(x[(size_t)s * IN + i]);
    float h1[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < IN; ++i) acc = fmaf(sp.w1[j * IN + i], xi[i], acc);
        acc += sp.b1[j];
        h1[j] = bf16_round(acc > 0.f ? acc : 0.f);
        if (h1s) h1s[(size_t)s * H + j] = h1[j];
    }
    float o = 0.f;
    for (int j = 0; j < H; ++j) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < H; ++i) acc = fmaf(sp.w2[j * H + i], h1[i], acc);
        acc += sp.b2[j];
        const float h2 = bf16_round(acc > 0.f ? acc : 0.f);
        if (h2s) h2s[(size_t)s * H + j] = h2;
        o = fmaf(sp.w3[j], h2, o);
    }
    o += sp.b3;
    if (out) out[s] = o;
    if (score) {
        float g = exp2f(fminf(o, 126.f)) - 1.f;
        if (ub) {
            const float u = (float)ub[cand ? cand[s] : s];
            g = fminf(g, u);
        }
        score[s] = g;
    }
}

// Per-sample backward: dh2 = dout * W3 * [h2 > 0], dh1 = (W2^T dh2) * [h1 > 0],
// dout = 2 (out - y) / count.  Writes dout (count), dh1, dh2 (count x 64).
__global__ __launch_bounds__(256) void k_mlp_backward_sample(const MlpBlock *p, const float *h1s,
                                                             const float *h2s, const float *out,
                                                             const float *y, int32_t count,
                                                             float *dout_s, float *dh1s, float *dh2s) {
    __shared__ SParams sp;
    stage_params(p, &sp);
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const float dout = 2.f * (out[s] - y[s]) / (float)count;
    dout_s[s] = dout;
    float dh2[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const float h2 = h2s[(size_t)s * H + i];
        dh2[i] = h2 > 0.f ? dout * sp.w3[i] : 0.f;
        dh2s[(size_t)s * H + i] = dh2[i];
    }
    for (int j = 0; j < H; ++j) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < H; ++i) acc = fmaf(sp.w2[i * H + j], dh2[i], acc);
        const float h1 = h1s[(size_t)s * H + j];
        dh1s[(size_t)s * H + j] = h1 > 0.f ? acc : 0.f;
    }
}

// Gradient of every master parameter: one thread per parameter, samples
// summed in order (deterministic).  Layout of grad = layout of the master
// vector: W1 (64x8), b1, W2 (64x64), b2, W3, b3.
__global__ __launch_bounds__(256) void k_mlp_grad_reduce(const float *x, const float *h1s,
                                                         const float *h2s, const float *dout_s,
                                                         const float *dh1s, const float *dh2s,
                                                         int32_t count, float *grad) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kMlpParams) return;
    float acc = 0.f;
    if (q < kOffB1) {  // W1[j][i]
        const int j = q / IN, i = q % IN;
        for (int s = 0; s < count; ++s) acc = fmaf(dh1s[(size_t)s * H + j], bf16_round(x[(size_t)s * IN + i]), acc);
    } else if (q < kOffW2) {  // b1[j]
        const int j = q - kOffB1;
        for (int s = 0; s < count; ++s) acc += dh1s[(size_t)s * H + j];
    } else if (q < kOffB2) {  // W2[j][i]
        const int t = q - kOffW2, j = t / H, i = t % H;
        for (int s = 0; s < count; ++s) acc = fmaf(dh2s[(size_t)s * H + j], h1s[(size_t)s * H + i], acc);
    } else if (q < kOffW3) {  // b2[j]
        const int j = q - kOffB2;
        for (int s = 0; s < count; ++s) acc += dh2s[(size_t)s * H + j];
    } else if (q < kOffB3) {  // W3[i]
        const int i = q - kOffW3;
        for (int s = 0; s < count; ++s) acc = fmaf(dout_s[s], h2s[(size_t)s * H + i], acc);
    } else {  // b3
        for (int s = 0; s < count; ++s) acc += dout_s[s];
    }
    grad[q] = acc;
}

// master float32 -> inference block (bf16 weights, float32 biases)
__global__ void k_mlp_pack(const float *m, MlpBlock *p) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < kMlpParams; q += gridDim.x * blockDim.x) {
        if (q < kOffB1) p->w1[q] = to_bf16(m[q]);
        else if (q < kOffW2) p->b1[q - kOffB1] = m[q];
        else if (q < kOffB2) p->w2[q - kOffW2] = to_bf16(m[q]);
        else if (q < kOffW3) p->b2[q - kOffB2] = m[q];
        else if (q < kOffB3) p->w3[q - kOffW3] = to_bf16(m[q]);
        else p->b3 = m[q];
    }
}

// Adam (Kingma and Ba, 2015) on the float32 master vector.
__global__ void k_mlp_adam(float *w, float *m, float *v, const float *g, int32_t step, float lr,
                           float b1, float b2, float eps) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kMlpParams) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    const float mh = mq / (1.f - powf(b1, (float)step));
    const float vh = vq / (1.f - powf(b2, (float)step));
    w[q] = w[q] - lr * mh / (sqrtf(vh) + eps);
}

// Node features for the learned order (8 floats per candidate), from the
// state of the lazy loop at the start of a round:
//   0 log2(1 + deg v)            1 d(S,v) / ecc(s_1)
//   2 log2(1 + stale gain)       3 log2(1 + sum_{u in N(v)} deg u)
//   4 log2(1 + rounds since v was last evaluated)
//   5 d(S,v) when last evaluated - d(S,v) now
//   6 round / k                  7 log2(1 + d(S,v))
template <typename DistT>
__global__ void k_features(FeatArgs a) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= a.count) return;
    const int32_t v = a.cand ? a.cand[t] : (int32_t)t;
    const DistT *dist = reinterpret_cast<const DistT *>(a.dist);
    const int32_t rs = a.rp[v], re = a.rp[v + 1];
    const float deg = (float)(re - rs);
    float two = 0.f;
    if (a.two64) {
        two = (float)a.two64[v];
    } else {
        int64_t acc = 0;
        for (int32_t e = rs; e < re; ++e) {
            const int32_t u = a.ci[e];
            acc += a.rp[u + 1] - a.rp[u];
        }
        two = (float)acc;
    }
    const float d = (float)(uint32_t)dist[v];
    const float ubv = a.ub[v] >= 0 ? (float)a.ub[v] : 0.f;
    const int32_t le = a.last_eval[v];
    const float since = le >= 0 ? (float)(a.round - le) : (float)a.round;
    const float dat = le >= 0 ? (float)a.dist_at_eval[v] : d;
    float *f = a.feat + (size_t)t * kMlpIn;
    f[0] = log2f(1.f + deg);
    f[1] = d / (float)(a.ecc1 > 0 ? a.ecc1 : 1);
    f[2] = log2f(1.f + ubv);
    f[3] = log2f(1.f + two);
    f[4] = log2f(1.f + since);
    f[5] = dat - d;
    f[6] = (float)a.round / (float)(a.k > 0 ? a.k : 1);
    f[7] = log2f(1.f + d);
}

// Top `take` of count (score, id) pairs by score descending, id ascending:
// a bitonic sort of 64-bit keys in LDS.  The key puts the score's bits in an
// order-preserving form in the high word (inverted, so that ascending keys
// are descending scores) and the id in the low word.
__global__ __launch_bounds__(1024) void k_select_top(const float *score, const int32_t *ids,
                                                     int32_t count, int32_t take, int32_t *out) {
    __shared__ unsigned long long key[kSelectMax];
    int m = 1;
    while (m < count) m <<= 1;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        unsigned long long k = ~0ull;
        if (i < count) {
            uint32_t u = __float_as_uint(score[i]);
            u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);  // ascending as the float
            k = ((unsigned long long)(~u) << 32) | (uint32_t)ids[i];
        }
        key[i] = k;
    }
    __syncthreads();
    for (int size = 2; size <= m; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < m; i += blockDim.x) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const unsigned long long a = key[i], b = key[j];
                    if ((a > b) == up) {
                        key[i] = b;
                        key[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < take; i += blockDim.x) out[i] = (int32_t)(uint32_t)key[i];
}

int grid_for(int64_t n, int bs) {
    int64_t g = (n + bs - 1) / bs;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t launch_mlp_forward(const MlpBlock *p, const float *x, int32_t count, float *out,
                              float *h1, float *h2, const int64_t *ub, const int32_t *cand,
                              float *score, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid_for(count, 256)), dim3(256), 0, s, p, x, count, out,
                       h1, h2, ub, cand, score);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const MlpBlock *p, const float *x, const float *h1, const float *h2,
                               const float *out, const float *y, int32_t count, float *grad,
                               float *scratch, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    float *dout = scratch;
    float *dh1 = scratch + ((count + 63) / 64) * 64;
    float *dh2 = dh1 + (size_t)count * kMlpHidden;
    hipLaunchKernelGGL(k_mlp_backward_sample, dim3(grid_for(count, 256)), dim3(256), 0, s, p, h1, h2,
                       out, y, count, dout, dh1, dh2);
    hipLaunchKernelGGL(k_mlp_grad_reduce, dim3(grid_for(kMlpParams, 64)), dim3(64), 0, s, x, h1, h2,
                       dout, dh1, dh2, count, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_pack(const float *master, MlpBlock *p, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_pack, dim3(grid_for(kMlpParams, 256)), dim3(256), 0, s, master, p);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *w, float *m, float *v, const float *g, int32_t step, float lr,
                           float b1, float b2, float eps, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_adam, dim3(grid_for(kMlpParams, 256)), dim3(256), 0, s, w, m, v, g, step,
                       lr, b1, b2, eps);
    return hipGetLastError();
}

hipError_t launch_features(const FeatArgs &a, int dist_bytes, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    if (dist_bytes == 1)
        hipLaunchKernelGGL((k_features<uint8_t>), dim3(grid_for(a.count, 256)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_features<uint16_t>), dim3(grid_for(a.count, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_select_top(const float *score, const int32_t *ids, int32_t count, int32_t take,
                             int32_t *out, hipStream_t s) {
    if (count < 0 || count > kSelectMax || take < 0 || take > count) return hipErrorInvalidValue;
    if (take == 0) return hipSuccess;
    hipLaunchKernelGGL(k_select_top, dim3(1), dim3(1024), 0, s, score, ids, count, take, out);
    return hipGetLastError();
}

}  // namespace gck

size_t gc_mlp_ws_bytes(int64_t n) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    // features (n x 8), scores, device copies of the lazy state
    return al((size_t)n * 8 * 4) + al((size_t)n * 4) + al((size_t)n * 8) + al((size_t)n * 4) +
           al((size_t)n * 2);
}
