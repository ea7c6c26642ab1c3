#include "gc_mlp.h"

size_t gc_mlp_ws_bytes(int64_t n) { return 0; }
