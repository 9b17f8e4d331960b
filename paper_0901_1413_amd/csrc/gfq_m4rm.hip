// gfq_m4rm.hip -- the field switch of the Four-Russians product launches: one product per
// launch (launch_matmul) or many products of one shape (launch_matmul_strided).  The
// kernels are instantiated per field in the gfq_m4rm_<field>.hip units; the tile
// computation itself is in gfq_m4rm_tile.h.
#include "gfq_internal.h"

namespace gfq {

template <bool STRIDED>
static hipError_t launch_field(int q, const MMArgs &a, const MMPlan &plan, const MMStrides &sd, hipStream_t st) {
    switch (q) {
    case 3: return launch_mm_q<STRIDED, 3>(a, plan, sd, st);
    case 4: return launch_mm_q<STRIDED, 4>(a, plan, sd, st);
    case GF4_KARATSUBA: return launch_mm_q<STRIDED, GF4_KARATSUBA>(a, plan, sd, st);
    case 5: return launch_mm_q<STRIDED, 5>(a, plan, sd, st);
    case 7: return launch_mm_q<STRIDED, 7>(a, plan, sd, st);
    case 8: return launch_mm_q<STRIDED, 8>(a, plan, sd, st);
    case GF8_TRINOMIAL: return launch_mm_q<STRIDED, GF8_TRINOMIAL>(a, plan, sd, st);
    case 9: return launch_mm_q<STRIDED, 9>(a, plan, sd, st);
    case F9_KARATSUBA: return launch_mm_q<STRIDED, F9_KARATSUBA>(a, plan, sd, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_matmul(int q, const MMArgs &a, const MMPlan &plan, hipStream_t st) {
    return launch_field<false>(q, a, plan, MMStrides{1, 0, 0, 0}, st);
}

hipError_t launch_matmul_strided(int q, const MMArgs &a, const MMPlan &plan, const MMStrides &sd, hipStream_t st) {
    if (sd.count < 1) return hipErrorInvalidValue;
    if (sd.count == 1) return launch_matmul(q, a, plan, st);
    return launch_field<true>(q, a, plan, sd, st);
}

}  // namespace gfq
