// gfq_m4rm_f9.hip -- product kernels for F_9, row-wise and by Karatsuba: single-product and strided.
#include "gfq_m4rm_launch.h"

namespace gfq {

template hipError_t launch_mm_q<false, 9>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);
template hipError_t launch_mm_q<true, 9>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);
template hipError_t launch_mm_q<false, F9_KARATSUBA>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);
template hipError_t launch_mm_q<true, F9_KARATSUBA>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);

}  // namespace gfq
