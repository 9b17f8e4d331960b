// gfq_m4rm.hip -- the plain (one product per launch) Four-Russians product kernel and its
// launcher.  The tile computation itself is in gfq_m4rm_tile.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gfq_m4rm_tile.h"

namespace gfq {

template <int Q, int TWD, int REP, int R, int NT>
__global__ __launch_bounds__(NT) void m4rm_kernel(MMArgs a) {
    m4rm_tile<Q, TWD, REP, R, NT>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

// ---------------------------------------------------------------------------------------
// Launch: layout (super-row bytes) and rows-per-lane variants.
// ---------------------------------------------------------------------------------------
template <int Q, int TWD, int REP, int R>
static hipError_t launch_mm(const MMArgs &a0, const MMPlan &plan, hipStream_t st) {
    constexpr int LPR = TWD / 4;
    constexpr int TM = (NT_MM / LPR) * R;
    if (plan.TM != TM || plan.lds > 163840) return hipErrorInvalidValue;
    MMArgs a = a0;
    a.tb1 = plan.tb1;
    dim3 grid((a.Wn + TWD - 1) / TWD, (a.m + TM - 1) / TM, (a.S + a.slabs_per_split - 1) / a.slabs_per_split);
    auto kern = m4rm_kernel<Q, TWD, REP, R, NT_MM>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)plan.lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, dim3(NT_MM), plan.lds, st, a);
    return hipGetLastError();
}

template <int Q, int TWD, int REP>
static hipError_t launch_mm_rows(const MMArgs &a, const MMPlan &plan, hipStream_t st) {
    if (plan.R == 2) return launch_mm<Q, TWD, REP, 2>(a, plan, st);
    if constexpr (Q == 5 || Q == 7) {
        return launch_mm<Q, TWD, REP, 4>(a, plan, st);       // eight rows per lane would spill
    } else {
        if (plan.R == 4) return launch_mm<Q, TWD, REP, 4>(a, plan, st);
        if constexpr (Q == 4 && TWD == 16) {
            if (plan.R == 16) return launch_mm<Q, TWD, REP, 16>(a, plan, st);   // two planes per word
        }
        return launch_mm<Q, TWD, REP, 8>(a, plan, st);
    }
}

template <int Q>
static hipError_t launch_mm_q(const MMArgs &a, const MMPlan &plan, hipStream_t st) {
    switch (plan.srb) {
    case 256: return launch_mm_rows<Q, 16, 4>(a, plan, st);
    case 128: return launch_mm_rows<Q, 16, 2>(a, plan, st);
    case 64: return launch_mm_rows<Q, 16, 1>(a, plan, st);
    case 32: return launch_mm_rows<Q, 8, 1>(a, plan, st);
    case 16: return launch_mm_rows<Q, 4, 1>(a, plan, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_matmul(int q, const MMArgs &a, const MMPlan &plan, hipStream_t st) {
    switch (q) {
    case 3: return launch_mm_q<3>(a, plan, st);
    case 4: return launch_mm_q<4>(a, plan, st);
    case 5: return launch_mm_q<5>(a, plan, st);
    default: return launch_mm_q<7>(a, plan, st);
    }
}

}  // namespace gfq
