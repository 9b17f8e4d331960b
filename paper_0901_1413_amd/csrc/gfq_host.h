// gfq_host.h -- host helpers shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gfq.h"
#include "gfq_internal.h"

namespace gfq {

// Record a HIP failure for gfq_last_hip_error and return GFQ_EHIP.
int hip_fail(hipError_t e, const char *what);
// The calling thread's stream (gfq_set_stream).
hipStream_t current_stream();
// Build a batch; cfgs (optional, one per product) overrides the per-product configuration.
int batch_create_with(int count, const gfq_problem *problems, const gfq_config *cfgs, gfq_batch **out);
// Fill n words with pseudo-random bits (a hash of the index and the seed); timing data only.
hipError_t launch_fill_random(u32 *p, size_t n, u32 seed, hipStream_t st);
// Field, dimension, pointer, alignment and aliasing checks of one product.
int validate_mm(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B, void *C);

}  // namespace gfq
