// gfq_pack.hip -- pack / unpack between uint8 matrices and the packed bitsliced format
// (paper, Section 3 with the element encodings of Section 4), and the reduction of the
// partial products of split inner dimensions.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gfq_device.h"
#include "gfq_internal.h"

namespace gfq {

// Sum of `splits` canonical partial products (same packed layout, split_stride words
// apart), canonicalise and zero the pad columns.  One thread per (row, 4-word group).
template <int Q>
__global__ __launch_bounds__(256) void reduce_partials_kernel(const u32 *part, u32 *C, int m, int n, int Wn,
                                                              int splits, size_t split_stride) {
    typedef FT<Q> F;
    constexpr int P = F::P;
    const int groups = Wn / 4;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)m * groups) return;
    const int row = (int)(idx / groups), w = (int)(idx % groups) * 4;
    u32 v[4][P];
#pragma unroll
    for (int p = 0; p < P; p++) {
        const uint4 x = *reinterpret_cast<const uint4 *>(part + ((size_t)row * P + p) * Wn + w);
        v[0][p] = x.x; v[1][p] = x.y; v[2][p] = x.z; v[3][p] = x.w;
    }
    for (int z = 1; z < splits; z++) {
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

// ---------------------------------------------------------------------------------------
// Pack / unpack.  One wave per (row, 64 columns): each lane takes one element, and a
// wave-wide ballot of one plane bit yields that plane's 64-bit word pair.
// ---------------------------------------------------------------------------------------
template <int Q>
__device__ __forceinline__ void encode(u32 v, u32 *bits) {
    if (Q == 3) {
        v %= 3u;
        bits[0] = v != 0u;
        bits[1] = v == 2u;
    } else if (Q == 4) {
        bits[0] = v & 1u;
        bits[1] = (v >> 1) & 1u;
    } else {
        v %= (u32)Q;
        bits[0] = v & 1u; bits[1] = (v >> 1) & 1u; bits[2] = (v >> 2) & 1u;
    }
}

template <int Q>
__global__ __launch_bounds__(256) void pack_kernel(const uint8_t *src, int64_t ld, u32 *dst, int rows, int cols, int W) {
    constexpr int P = FT<Q>::P;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int chunks = W / 2;                    // 64-column chunks per row
    const int64_t items = (int64_t)rows * chunks;
    for (int64_t it = wave; it < items; it += nwaves) {
        const int row = (int)(it / chunks), ch = (int)(it % chunks);
        const int col = ch * 64 + lane;
        u32 v = col < cols ? src[(int64_t)row * ld + col] : 0u;
        u32 bits[P];
        encode<Q>(v, bits);
        if (col >= cols) {
#pragma unroll
            for (int p = 0; p < P; p++) bits[p] = 0u;
        }
#pragma unroll
        for (int p = 0; p < P; p++) {
            const uint64_t b = __ballot(bits[p] != 0u);
            if (lane == 0) {
                uint2 wv = make_uint2((u32)b, (u32)(b >> 32));
                *reinterpret_cast<uint2 *>(dst + ((size_t)row * P + p) * W + ch * 2) = wv;
            }
        }
    }
}

template <int Q>
__global__ __launch_bounds__(256) void unpack_kernel(const u32 *src, uint8_t *dst, int64_t ld, int rows, int cols, int W) {
    constexpr int P = FT<Q>::P;
    const int64_t total = (int64_t)rows * cols;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int row = (int)(idx / cols), col = (int)(idx % cols);
        u32 b[P];
#pragma unroll
        for (int p = 0; p < P; p++) b[p] = (src[((size_t)row * P + p) * W + (col >> 5)] >> (col & 31)) & 1u;
        u32 v;
        if (Q == 3) v = b[0] ? (b[1] ? 2u : 1u) : 0u;
        else if (Q == 4) v = b[0] | (b[1] << 1);
        else v = (b[0] | (b[1] << 1) | (b[2] << 2)) % (u32)Q;
        dst[(int64_t)row * ld + col] = (uint8_t)v;
    }
}

hipError_t launch_reduce(int q, const u32 *part, u32 *C, int m, int n, int Wn, int splits, size_t stride, hipStream_t st) {
    const size_t threads = (size_t)m * (Wn / 4);
    dim3 grid((unsigned)((threads + 255) / 256));
    switch (q) {
    case 3: hipLaunchKernelGGL(reduce_partials_kernel<3>, grid, dim3(256), 0, st, part, C, m, n, Wn, splits, stride); break;
    case 4: hipLaunchKernelGGL(reduce_partials_kernel<4>, grid, dim3(256), 0, st, part, C, m, n, Wn, splits, stride); break;
    case 5: hipLaunchKernelGGL(reduce_partials_kernel<5>, grid, dim3(256), 0, st, part, C, m, n, Wn, splits, stride); break;
    default: hipLaunchKernelGGL(reduce_partials_kernel<7>, grid, dim3(256), 0, st, part, C, m, n, Wn, splits, stride); break;
    }
    return hipGetLastError();
}

static unsigned grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g > 256 * 64) g = 256 * 64;
    if (g < 1) g = 1;
    return (unsigned)g;
}

hipError_t launch_pack(int q, const uint8_t *src, int64_t ld, u32 *dst, int rows, int cols, int W, hipStream_t st) {
    const int64_t items = (int64_t)rows * (W / 2);
    dim3 grid(grid_for(items, 4));
    switch (q) {
    case 3: hipLaunchKernelGGL(pack_kernel<3>, grid, dim3(256), 0, st, src, ld, dst, rows, cols, W); break;
    case 4: hipLaunchKernelGGL(pack_kernel<4>, grid, dim3(256), 0, st, src, ld, dst, rows, cols, W); break;
    case 5: hipLaunchKernelGGL(pack_kernel<5>, grid, dim3(256), 0, st, src, ld, dst, rows, cols, W); break;
    default: hipLaunchKernelGGL(pack_kernel<7>, grid, dim3(256), 0, st, src, ld, dst, rows, cols, W); break;
    }
    return hipGetLastError();
}

hipError_t launch_unpack(int q, const u32 *src, uint8_t *dst, int64_t ld, int rows, int cols, int W, hipStream_t st) {
    dim3 grid(grid_for((int64_t)rows * cols, 256));
    switch (q) {
    case 3: hipLaunchKernelGGL(unpack_kernel<3>, grid, dim3(256), 0, st, src, dst, ld, rows, cols, W); break;
    case 4: hipLaunchKernelGGL(unpack_kernel<4>, grid, dim3(256), 0, st, src, dst, ld, rows, cols, W); break;
    case 5: hipLaunchKernelGGL(unpack_kernel<5>, grid, dim3(256), 0, st, src, dst, ld, rows, cols, W); break;
    default: hipLaunchKernelGGL(unpack_kernel<7>, grid, dim3(256), 0, st, src, dst, ld, rows, cols, W); break;
    }
    return hipGetLastError();
}

}  // namespace gfq
