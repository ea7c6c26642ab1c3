// Launchers of the bit-vector gain kernels (gc_bits.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gck {

// rows of b^i_S kept: d(S,.) in uint8 is below 255, so no term past 254 counts
constexpr int32_t kBitsMaxS = 256;

hipError_t launch_bits_identity(uint64_t *b0, int32_t n, hipStream_t s);
hipError_t launch_bits_level(const int32_t *rp, const int32_t *ci, int32_t n, const uint64_t *prev,
                             uint64_t *next, int32_t *changed, hipStream_t s);
hipError_t launch_bits_group(const void *dist, int dist_bytes, int32_t n, int32_t levels, uint64_t *bs,
                             hipStream_t s);
hipError_t launch_bits_gains(const uint64_t *bits, int32_t n, int32_t levels_b, const uint64_t *bs,
                             int32_t levels_s, const int32_t *cand, int64_t count, int64_t *gain,
                             unsigned long long *words, hipStream_t s);

}  // namespace gck
