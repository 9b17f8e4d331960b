// gfq_m4rm_gf8.hip -- product kernels for GF(8), row-wise and by the trinomial formula: single-product and strided.
#include "gfq_m4rm_launch.h"

namespace gfq {

template hipError_t launch_mm_q<false, 8>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);
template hipError_t launch_mm_q<true, 8>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);
template hipError_t launch_mm_q<false, GF8_TRINOMIAL>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);
template hipError_t launch_mm_q<true, GF8_TRINOMIAL>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);

}  // namespace gfq
