// gfq_host.h -- host helpers shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gfq {

// Record a HIP failure for gfq_last_hip_error and return GFQ_EHIP.
int hip_fail(hipError_t e, const char *what);
// The calling thread's stream (gfq_set_stream).
hipStream_t current_stream();
// Field, dimension, pointer, alignment and aliasing checks of one product.
int validate_mm(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B, void *C);

}  // namespace gfq
