// Internal interface between the host driver (gc_api.cpp) and the
// allocation-free entry point (gc_noalloc.hip).  Not part of the public C ABI.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime.h>

#include "gc.h"

namespace gck {

// Bytes the marginal-gain path needs for graph g with one batch of 64
// sources per launch (the smallest buffer gains_in_buffer accepts).
size_t gains_buffer_min_bytes(const gc_graph *g);

// gc_marginal_gains on a device buffer of buf_bytes bytes instead of a
// prepared workspace: the buffer is laid out for the gain path alone, and the
// parts the path reads before writing are zeroed first, so its earlier
// contents do not matter.  GC_EWORKSPACE if it is too small for one batch.
int gains_in_buffer(const gc_graph *g, const void *d_dist, int32_t dist_bytes, const int32_t *d_cand,
                    int32_t count, int64_t *d_gain, int64_t *d_edges, int32_t *d_visited, void *d_buf,
                    size_t buf_bytes, hipStream_t stream);

// the error message of the calling thread (gc_last_error) is set through this
int set_error(int code, const char *msg);

}  // namespace gck
