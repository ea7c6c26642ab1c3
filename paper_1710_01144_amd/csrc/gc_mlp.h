// Candidate-ordering MLP (features -> 8x64x64x1, bfloat16 weights, fp32
// accumulation).  Internal interface; the kernels live in gc_mlp.hip.
#pragma once
#include <stddef.h>
#include <stdint.h>

// Device workspace bytes the MLP path needs for a graph of n nodes.
size_t gc_mlp_ws_bytes(int64_t n);
