// gfq_reduce.h -- the sum of the slab-slice partial products of one product, shared by the
// single-product partial-sum kernel and the batched one.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gfq_device.h"

namespace gfq {

// Row `row`, words w .. w + 3 of every plane: the sum of `splits` canonical partial products
// (same packed layout, split_stride words apart), canonicalised, pad columns zeroed, into C.
template <int Q>
__device__ __forceinline__ void reduce_group(const u32 *part, u32 *C, int row, int w, int n, int Wn, int splits,
                                             size_t split_stride) {
    typedef FT<Q> F;
    constexpr int P = F::P;
    u32 v[4][P];
#pragma unroll
    for (int p = 0; p < P; p++) {
        const uint4 x = *reinterpret_cast<const uint4 *>(part + ((size_t)row * P + p) * Wn + w);
        v[0][p] = x.x; v[1][p] = x.y; v[2][p] = x.z; v[3][p] = x.w;
    }
    // partials four at a time: their loads are all in flight before the first addition
    // (field addition is associative and commutative, so the order of the sums is free)
    int z = 1;
    for (; z + 4 <= splits; z += 4) {
        uint4 x[4][P];
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int p = 0; p < P; p++)
                x[j][p] = *reinterpret_cast<const uint4 *>(part + (size_t)(z + j) * split_stride +
                                                           ((size_t)row * P + p) * Wn + w);
#pragma unroll
        for (int j = 0; j < 4; j++) {
            u32 y[4][P];
#pragma unroll
            for (int p = 0; p < P; p++) {
                y[0][p] = x[j][p].x; y[1][p] = x[j][p].y; y[2][p] = x[j][p].z; y[3][p] = x[j][p].w;
            }
#pragma unroll
            for (int i = 0; i < 4; i++) {
                u32 r[P];
                F::sadd(v[i], y[i], r);
#pragma unroll
                for (int p = 0; p < P; p++) v[i][p] = r[p];
            }
        }
    }
    for (; z < splits; z++) {
        const u32 *pz = part + z * split_stride;
        u32 y[4][P];
#pragma unroll
        for (int p = 0; p < P; p++) {
            const uint4 x = *reinterpret_cast<const uint4 *>(pz + ((size_t)row * P + p) * Wn + w);
            y[0][p] = x.x; y[1][p] = x.y; y[2][p] = x.z; y[3][p] = x.w;
        }
#pragma unroll
        for (int i = 0; i < 4; i++) {
            u32 r[P];
            F::sadd(v[i], y[i], r);
#pragma unroll
            for (int p = 0; p < P; p++) v[i][p] = r[p];
        }
    }
    u32 msk[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int rem = n - (w + i) * 32;
        msk[i] = rem >= 32 ? 0xffffffffu : (rem <= 0 ? 0u : ((1u << rem) - 1u));
        F::scanon(v[i]);
    }
#pragma unroll
    for (int p = 0; p < P; p++)
        *reinterpret_cast<uint4 *>(C + ((size_t)row * P + p) * Wn + w) =
            make_uint4(v[0][p] & msk[0], v[1][p] & msk[1], v[2][p] & msk[2], v[3][p] & msk[3]);
}

}  // namespace gfq
