// gfq_m4rm.hip -- the plain (one product per launch) Four-Russians product kernel and its
// launcher.  The tile computation itself is in gfq_m4rm_tile.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "gfq_m4rm_tile.h"

namespace gfq {

// grid (column tiles, row tiles, products x slab slices); row tile ty0 + blockIdx.y
template <int Q, int TWD, int REP, int R, int NT>
__global__ __launch_bounds__(NT) void m4rm_kernel(MMArgs a, int ty0, int splits, MMStrides sd) {
    const int prod = (int)blockIdx.z / splits;
    const int bz = (int)blockIdx.z - prod * splits;
    if (prod > 0) {
        a.A += (size_t)prod * sd.A;
        a.B += (size_t)prod * sd.B;
        a.out += (size_t)prod * sd.out;
    }
    m4rm_tile<Q, TWD, REP, R, NT>(a, blockIdx.x, ty0 + (int)blockIdx.y, bz);
}

// ---------------------------------------------------------------------------------------
// Launch: layout (super-row bytes) and rows-per-lane variants.
// ---------------------------------------------------------------------------------------
template <int Q, int TWD, int REP, int R>
static hipError_t launch_mm(const MMArgs &a0, const MMPlan &plan, const MMStrides &sd, hipStream_t st) {
    constexpr int LPR = TWD / 4;
    constexpr int TM = (NT_MM / LPR) * R;
    if (plan.TM != TM || plan.lds > 163840) return hipErrorInvalidValue;
    MMArgs a = a0;
    a.tb1 = plan.tb1;
    const int row_tiles = (a.m + TM - 1) / TM;
    auto kern = m4rm_kernel<Q, TWD, REP, R, NT_MM>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)plan.lds);
    if (e != hipSuccess) return e;
    const int splits = (a.S + a.slabs_per_split - 1) / a.slabs_per_split;
    if ((int64_t)splits * sd.count > 65535) return hipErrorInvalidValue;
    // a grid's y extent is at most 65535: taller products take several launches
    for (int ty0 = 0; ty0 < row_tiles; ty0 += 65535) {
        dim3 grid((a.Wn + TWD - 1) / TWD, std::min(65535, row_tiles - ty0), splits * sd.count);
        hipLaunchKernelGGL(kern, grid, dim3(NT_MM), plan.lds, st, a, ty0, splits, sd);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int Q, int TWD, int REP>
static hipError_t launch_mm_rows(const MMArgs &a, const MMPlan &plan, const MMStrides &sd, hipStream_t st) {
    constexpr bool two_only = Q == 9 || Q == F9_KARATSUBA;   // F_9: two rows per lane only
    if (plan.R == 2 || two_only) return launch_mm<Q, TWD, REP, 2>(a, plan, sd, st);
    if constexpr (two_only) {
        return hipErrorInvalidValue;
    } else if constexpr (Q == 5 || Q == 7 || ((Q == 8 || Q == GF8_TRINOMIAL) && TWD < 16)) {
        return launch_mm<Q, TWD, REP, 4>(a, plan, sd, st);       // eight rows per lane would spill
    } else {
        if (plan.R == 4) return launch_mm<Q, TWD, REP, 4>(a, plan, sd, st);
        if constexpr ((Q == 4 || Q == GF4_KARATSUBA) && TWD == 16) {
            if (plan.R == 16) return launch_mm<Q, TWD, REP, 16>(a, plan, sd, st);   // two planes per word
        }
        return launch_mm<Q, TWD, REP, 8>(a, plan, sd, st);
    }
}

template <int Q>
static hipError_t launch_mm_q(const MMArgs &a, const MMPlan &plan, const MMStrides &sd, hipStream_t st) {
    switch (plan.srb) {
    case 256: return launch_mm_rows<Q, 16, 4>(a, plan, sd, st);
    case 128: return launch_mm_rows<Q, 16, 2>(a, plan, sd, st);
    case 64: return launch_mm_rows<Q, 16, 1>(a, plan, sd, st);
    case 32: return launch_mm_rows<Q, 8, 1>(a, plan, sd, st);
    case 16: return launch_mm_rows<Q, 4, 1>(a, plan, sd, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_matmul(int q, const MMArgs &a, const MMPlan &plan, hipStream_t st) {
    return launch_matmul_strided(q, a, plan, MMStrides{1, 0, 0, 0}, st);
}

hipError_t launch_matmul_strided(int q, const MMArgs &a, const MMPlan &plan, const MMStrides &sd, hipStream_t st) {
    if (sd.count < 1) return hipErrorInvalidValue;
    switch (q) {
    case 3: return launch_mm_q<3>(a, plan, sd, st);
    case 4: return launch_mm_q<4>(a, plan, sd, st);
    case GF4_KARATSUBA: return launch_mm_q<GF4_KARATSUBA>(a, plan, sd, st);
    case 5: return launch_mm_q<5>(a, plan, sd, st);
    case 8: return launch_mm_q<8>(a, plan, sd, st);
    case 9: return launch_mm_q<9>(a, plan, sd, st);
    case GF8_TRINOMIAL: return launch_mm_q<GF8_TRINOMIAL>(a, plan, sd, st);
    case F9_KARATSUBA: return launch_mm_q<F9_KARATSUBA>(a, plan, sd, st);
    default: return launch_mm_q<7>(a, plan, sd, st);
    }
}

}  // namespace gfq
