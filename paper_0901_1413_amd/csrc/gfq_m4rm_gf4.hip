// gfq_m4rm_gf4.hip -- product kernels for GF(4), row-wise and by Karatsuba: single-product and strided.
#include "gfq_m4rm_launch.h"

namespace gfq {

template hipError_t launch_mm_q<false, 4>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);
template hipError_t launch_mm_q<true, 4>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);
template hipError_t launch_mm_q<false, GF4_KARATSUBA>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);
template hipError_t launch_mm_q<true, GF4_KARATSUBA>(const MMArgs &, const MMPlan &, const MMStrides &, hipStream_t);

}  // namespace gfq
