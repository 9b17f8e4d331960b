// gfq_m4rm_launch.h -- the Four-Russians product kernels and their launch templates: the
// single-product kernel (grid.z = slab slices) and the strided kernel for many products of
// one shape (grid.z = product x slab slices).  Included only by the gfq_m4rm_<field>.hip
// units, each of which instantiates launch_mm_q for its fields (so the kernels of
// different fields compile in parallel); gfq_m4rm.hip holds the field switch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "gfq_m4rm_tile.h"

namespace gfq {

// The tile a workgroup runs.  The dispatcher hands workgroups to the chip's XCDs in turn
// (workgroup i of a launch to XCD i mod 8), and each XCD has an L2 of its own.  Workgroup i
// therefore runs tile L(i) of the grid, numbered column tile fastest, then row tile, then
// slice, where L gives each XCD one contiguous range of tiles: the workgroups running
// together on an XCD are neighbours, which read the same rows of A (the column tiles of a
// row tile) and of B (the row tiles of a column tile), and share them in that XCD's L2
// instead of every XCD fetching them from HBM.  L is a bijection of 0 .. total - 1 for any
// total (the first total mod 8 XCDs take one tile more).
__device__ __forceinline__ void xcd_tile(int &bx, int &by, int &bz) {
    constexpr uint64_t NXCD = 8;
    const uint64_t X = gridDim.x, Y = gridDim.y;
    const uint64_t total = X * Y * gridDim.z;
    const uint64_t flat = blockIdx.x + X * (blockIdx.y + Y * (uint64_t)blockIdx.z);
    const uint64_t per = total / NXCD, rem = total % NXCD;
    const uint64_t xcd = flat % NXCD, local = flat / NXCD;
    const uint64_t L = xcd * per + (xcd < rem ? xcd : rem) + local;
    bx = (int)(L % X);
    by = (int)((L / X) % Y);
    bz = (int)(L / (X * Y));
}

// grid (column tiles, row tiles, slab slices); row tile ty0 + the grid's row tile
template <int Q, int TWD, int REP, int R, int NT>
__global__ __launch_bounds__(NT) void m4rm_kernel(MMArgs a, int ty0) {
    int bx, by, bz;
    xcd_tile(bx, by, bz);
    m4rm_tile<Q, TWD, REP, R, NT>(a, bx, ty0 + by, bz);
}

// many products of one shape: grid.z = product x slab slices, operands at uniform strides
// (a kernel of its own, so that the single-product kernel keeps its plain argument use)
template <int Q, int TWD, int REP, int R, int NT>
__global__ __launch_bounds__(NT) void m4rm_strided_kernel(MMArgs a, int ty0, int splits, MMStrides sd) {
    int bx, by, bzp;
    xcd_tile(bx, by, bzp);
    const int prod = bzp / splits;
    const int bz = bzp - prod * splits;
    a.A += (size_t)prod * sd.A;
    a.B += (size_t)prod * sd.B;
    a.out += (size_t)prod * sd.out;
    m4rm_tile<Q, TWD, REP, R, NT>(a, bx, ty0 + by, bz);
}

// ---------------------------------------------------------------------------------------
// Launch: layout (super-row bytes) and rows-per-lane variants.
// ---------------------------------------------------------------------------------------
template <bool STRIDED, int Q, int TWD, int REP, int R>
static hipError_t launch_mm(const MMArgs &a0, const MMPlan &plan, const MMStrides &sd, hipStream_t st) {
    constexpr int LPR = TWD / 4;
    constexpr int TM = (NT_MM / LPR) * R;
    if (plan.TM != TM || plan.lds > 163840) return hipErrorInvalidValue;
    // byte-permuted gather addresses take the second table at a multiple of 64 KiB
    if (perm_addr_tile<Q, TWD, REP>() && plan.tb1 % 65536u != 0) return hipErrorInvalidValue;
    MMArgs a = a0;
    a.tb1 = plan.tb1;
    const int row_tiles = (a.m + TM - 1) / TM;
    const void *kern = STRIDED ? (const void *)m4rm_strided_kernel<Q, TWD, REP, R, NT_MM>
                               : (const void *)m4rm_kernel<Q, TWD, REP, R, NT_MM>;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)plan.lds);
    if (e != hipSuccess) return e;
    const int splits = (a.S + a.slabs_per_split - 1) / a.slabs_per_split;
    if ((int64_t)splits * sd.count > 65535) return hipErrorInvalidValue;
    // a grid's y extent is at most 65535: taller products take several launches
    for (int ty0 = 0; ty0 < row_tiles; ty0 += 65535) {
        dim3 grid((a.Wn + TWD - 1) / TWD, std::min(65535, row_tiles - ty0), splits * sd.count);
        if constexpr (STRIDED)
            hipLaunchKernelGGL((m4rm_strided_kernel<Q, TWD, REP, R, NT_MM>), grid, dim3(NT_MM), plan.lds, st, a, ty0,
                               splits, sd);
        else
            hipLaunchKernelGGL((m4rm_kernel<Q, TWD, REP, R, NT_MM>), grid, dim3(NT_MM), plan.lds, st, a, ty0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <bool STRIDED, int Q, int TWD, int REP>
static hipError_t launch_mm_rows(const MMArgs &a, const MMPlan &plan, const MMStrides &sd, hipStream_t st) {
    // two rows per lane only: F_9 by Karatsuba, and F_9 on narrow tiles (four would spill)
    constexpr bool two_only = Q == F9_KARATSUBA || (Q == 9 && TWD < 16);
    if (plan.R == 2 || two_only) return launch_mm<STRIDED, Q, TWD, REP, 2>(a, plan, sd, st);
    if constexpr (two_only) {
        return hipErrorInvalidValue;
    } else if constexpr (Q == 7 || (Q == 9 && TWD < 32) || ((Q == 5 || Q == 8 || Q == GF8_TRINOMIAL) && TWD < 16)) {
        return launch_mm<STRIDED, Q, TWD, REP, 4>(a, plan, sd, st);       // eight rows per lane would spill
    } else {
        if (plan.R == 4) return launch_mm<STRIDED, Q, TWD, REP, 4>(a, plan, sd, st);
        if constexpr ((Q == GF4_KARATSUBA && TWD == 16) || ((Q == 3 || Q == 4) && (TWD == 16 || TWD == 32))) {
            if (plan.R == 16) return launch_mm<STRIDED, Q, TWD, REP, 16>(a, plan, sd, st);   // two planes per word
        }
        return launch_mm<STRIDED, Q, TWD, REP, 8>(a, plan, sd, st);
    }
}

template <bool STRIDED, int Q>
hipError_t launch_mm_q(const MMArgs &a, const MMPlan &plan, const MMStrides &sd, hipStream_t st) {
    switch (plan.srb) {
    case 256: return launch_mm_rows<STRIDED, Q, 16, 4>(a, plan, sd, st);
    case 128: return launch_mm_rows<STRIDED, Q, 32, 1>(a, plan, sd, st);
    case 64: return launch_mm_rows<STRIDED, Q, 16, 1>(a, plan, sd, st);
    case 32: return launch_mm_rows<STRIDED, Q, 8, 1>(a, plan, sd, st);
    case 16: return launch_mm_rows<STRIDED, Q, 4, 1>(a, plan, sd, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace gfq
