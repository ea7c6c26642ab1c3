// Candidate-ordering MLP (features -> 8x64x64x1, bfloat16 weights, float32
// accumulation).  Internal interface; the kernels live in gc_mlp.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gck {

constexpr int kMlpIn = 8;
constexpr int kMlpHidden = 64;
// master vector layout (float32): W1 (64x8, row j = hidden unit), b1 (64),
// W2 (64x64, row j = output unit), b2 (64), W3 (64), b3 (1)
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpHidden * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpHidden;
constexpr int kOffB2 = kOffW2 + kMlpHidden * kMlpHidden;
constexpr int kOffW3 = kOffB2 + kMlpHidden;
constexpr int kOffB3 = kOffW3 + kMlpHidden;
constexpr int kMlpParams = kOffB3 + 1;  // 4801

// Inference block: bf16 weights (raw bits), float32 biases.
struct MlpBlock {
    uint16_t w1[kMlpHidden * kMlpIn];
    uint16_t w2[kMlpHidden * kMlpHidden];
    uint16_t w3[kMlpHidden];
    float b1[kMlpHidden];
    float b2[kMlpHidden];
    float b3;
    float pad[3];
};

struct FeatArgs {
    const int32_t *rp;
    const int32_t *ci;
    const void *dist;          // d(S,.) uint8/uint16
    const int32_t *cand;       // nodes (null: 0..count-1)
    int64_t count;
    const int64_t *ub;         // stale gain per node
    const int32_t *last_eval;  // round of the last evaluation (-1: never)
    const uint16_t *dist_at_eval;  // d(S,v) at that evaluation
    const int64_t *two64;      // the same as int64 (the workspace table), or null
    int32_t round, k, ecc1;
    float *feat;               // count x 8
};

// score[i] = min(2^out - 1, ub[cand ? cand[i] : i]) when score and ub are given
hipError_t launch_mlp_forward(const MlpBlock *p, const float *x, int32_t count, float *out,
                              float *h1, float *h2, const int64_t *ub, const int32_t *cand,
                              float *score, hipStream_t s);
// scratch: >= (round_up(count,64) + 2*count*64) floats
hipError_t launch_mlp_backward(const MlpBlock *p, const float *x, const float *h1, const float *h2,
                               const float *out, const float *y, int32_t count, float *grad,
                               float *scratch, hipStream_t s);
hipError_t launch_mlp_pack(const float *master, MlpBlock *p, hipStream_t s);
hipError_t launch_mlp_adam(float *w, float *m, float *v, const float *g, int32_t step, float lr,
                           float b1, float b2, float eps, hipStream_t s);
hipError_t launch_features(const FeatArgs &a, int dist_bytes, hipStream_t s);
// out[0..take) = the take ids of ids[0..count) with the largest scores
// (score[i] belongs to ids[i]; ties to the smaller id), in that order.
// count <= kSelectMax, take <= count; one workgroup.
constexpr int kSelectMax = 4096;
hipError_t launch_select_top(const float *score, const int32_t *ids, int32_t count, int32_t take,
                             int32_t *out, hipStream_t s);

}  // namespace gck

// Device workspace bytes the learned order needs for a graph of n nodes.
size_t gc_mlp_ws_bytes(int64_t n);
