// gc_batch.hip -- batched colouring entry points (filled in below).
#include <hip/hip_runtime.h>

#include "gc.h"

extern "C" size_t gc_batch_workspace_bytes(int64_t, const int64_t*, const int64_t*) { return 0; }
extern "C" int gc_color_batch(int64_t, const int64_t*, const int64_t*, const int32_t*,
                              const int32_t*, int32_t*, int32_t*, void*, size_t, void*) {
  return GC_EINVAL;
}
extern "C" size_t gc_batch_step_workspace_bytes(int64_t, int64_t) { return 0; }
extern "C" int gc_batch_step(int64_t, gc_graph_desc*, const int32_t*, const int32_t*, int32_t*,
                             int32_t, void*, size_t, void*) {
  return GC_EINVAL;
}
