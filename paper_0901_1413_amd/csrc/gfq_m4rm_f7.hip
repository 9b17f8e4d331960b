// gfq_m4rm_f7.hip -- product kernels for F_7: single-product and strided.
#include "gfq_m4rm_launch.h"

namespace gfq {

template hipError_t launch_mm_q<false, 7>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);
template hipError_t launch_mm_q<true, 7>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);

}  // namespace gfq
