// gfq_m4rm_f3.hip -- product kernels for F_3: single-product and strided.
#include "gfq_m4rm_launch.h"

namespace gfq {

template hipError_t launch_mm_q<false, 3>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);
template hipError_t launch_mm_q<true, 3>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);

}  // namespace gfq
