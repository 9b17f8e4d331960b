// gfq_pack.hip -- pack / unpack between uint8 matrices and the packed bitsliced format
// (paper, Section 3 with the element encodings of Section 4), and the reduction of the
// partial products of split inner dimensions.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gfq_device.h"
#include "gfq_internal.h"
#include "gfq_reduce.h"

namespace gfq {

// Sum of `splits` canonical partial products (same packed layout, split_stride words
// apart), canonicalise and zero the pad columns.  One thread per (row, 4-word group).
template <int Q>
__global__ __launch_bounds__(256) void reduce_partials_kernel(const u32 *part, u32 *C, int m, int n, int Wn,
                                                              int splits, size_t split_stride) {
    const int groups = Wn / 4;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)m * groups) return;
    reduce_group<Q>(part, C, (int)(idx / groups), (int)(idx % groups) * 4, n, Wn, splits, split_stride);
}

// ---------------------------------------------------------------------------------------
// Pack / unpack.  One thread per (row, 32-column word): it owns bit j of that word in
// every plane for the 32 elements of its columns.
// ---------------------------------------------------------------------------------------

// Plane bits of the residue of byte v, bit p of the code at bit 8p (p < P).
template <int Q> __device__ __forceinline__ u32 encode_spread(u32 v) {
    if (Q == 3) {
        v %= 3u;                                  // 0 = 00, 1 = 10, -1 = 11 (unit, sign)
        return (v != 0u ? 1u : 0u) | (v == 2u ? 1u << 8 : 0u);
    }
    if (Q == 4) return (v & 1u) | ((v >> 1) & 1u) << 8;
    if (Q == 9) {                                 // a0 + 3 a1: the F_3 code of a0, then of a1
        v %= 9u;
        const u32 a0 = v % 3u, a1 = v / 3u;
        return (a0 != 0u ? 1u : 0u) | (a0 == 2u ? 1u << 8 : 0u) | (a1 != 0u ? 1u << 16 : 0u) |
               (a1 == 2u ? 1u << 24 : 0u);
    }
    if (Q != 8) v %= (u32)Q;                      // binary digits (F_5, F_7; GF(8): c0, c1, c2)
    return (v & 1u) | ((v >> 1) & 1u) << 8 | ((v >> 2) & 1u) << 16;
}

// Pack the 32 elements of (row, word w) into their P plane words.  enc: encode_spread<Q>
// of every byte value.
template <int Q>
__device__ __forceinline__ void pack_unit(const uint8_t *src, int64_t ld, u32 *dst, int cols, int W, int aligned,
                                          const u32 *enc, int row, int w) {
    constexpr int P = FT<Q>::P;
    const int c0 = w * 32;
    u32 b[8];
    const uint8_t *rp = src + (int64_t)row * ld + c0;
    if (aligned && c0 + 32 <= cols) {
        const uint4 x = *reinterpret_cast<const uint4 *>(rp);
        const uint4 y = *reinterpret_cast<const uint4 *>(rp + 16);
        b[0] = x.x; b[1] = x.y; b[2] = x.z; b[3] = x.w; b[4] = y.x; b[5] = y.y; b[6] = y.z; b[7] = y.w;
    } else {
#pragma unroll
        for (int i = 0; i < 8; i++) {
            u32 v = 0u;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int c = c0 + 4 * i + j;
                v |= (c < cols ? (u32)rp[4 * i + j] : 0u) << (8 * j);   // 0 encodes as 0
            }
            b[i] = v;
        }
    }
    u32 out[P];
#pragma unroll
    for (int p = 0; p < P; p++) out[p] = 0u;
#pragma unroll
    for (int g = 0; g < 4; g++) {             // eight elements per group
        u32 acc = 0u;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const u32 byte = (b[2 * g + (i >> 2)] >> (8 * (i & 3))) & 0xffu;
            acc |= enc[byte] << i;
        }
#pragma unroll
        for (int p = 0; p < P; p++) out[p] |= ((acc >> (8 * p)) & 0xffu) << (8 * g);
    }
#pragma unroll
    for (int p = 0; p < P; p++) dst[((size_t)row * P + p) * W + w] = out[p];
}

template <int Q>
__global__ __launch_bounds__(256) void pack_kernel(const uint8_t *src, int64_t ld, u32 *dst, int rows, int cols, int W,
                                                   int aligned) {
    __shared__ u32 enc[256];
    enc[threadIdx.x] = encode_spread<Q>(threadIdx.x);
    __syncthreads();
    const int64_t total = (int64_t)rows * W;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x)
        pack_unit<Q>(src, ld, dst, cols, W, aligned, enc, (int)(idx / W), (int)(idx % W));
}

// Four bits (n < 16) to bit 0 of four bytes: n * (1 + 2^7 + 2^14 + 2^21) has no carries.
__device__ __forceinline__ u32 spread4(u32 n) { return (n * 0x00204081u) & 0x01010101u; }

// Unpack (row, word w): 32 canonical bytes (fewer in the last word of a row).
template <int Q>
__device__ __forceinline__ void unpack_unit(const u32 *src, uint8_t *dst, int64_t ld, int cols, int W, int aligned,
                                            int row, int w) {
    constexpr int P = FT<Q>::P;
    u32 pw[P];
#pragma unroll
    for (int p = 0; p < P; p++) pw[p] = src[((size_t)row * P + p) * W + w];
    u32 o[8];
#pragma unroll
    for (int g = 0; g < 8; g++) {             // four elements per group, one per byte
        u32 code = 0u;
#pragma unroll
        for (int p = 0; p < P; p++) code |= spread4((pw[p] >> (4 * g)) & 0xfu) << p;
        u32 v;
        if (Q == 3) {
            v = (code & 0x01010101u) + ((code >> 1) & 0x01010101u);            // unit + sign
        } else if (Q == 4 || Q == 8) {
            v = code;
        } else if (Q == 9) {
            const u32 a0 = (code & 0x01010101u) + ((code >> 1) & 0x01010101u);     // unit + sign
            const u32 a1 = ((code >> 2) & 0x01010101u) + ((code >> 3) & 0x01010101u);
            v = a0 + 3u * a1;
        } else if (Q == 7) {
            const u32 is7 = code & (code >> 1) & (code >> 2) & 0x01010101u;    // 7 = 0
            v = code ^ (is7 * 7u);
        } else {
            const u32 ge5 = (code >> 2) & (code | (code >> 1)) & 0x01010101u;  // 5, 6, 7
            v = code - ge5 * 5u;
        }
        o[g] = v;
    }
    uint8_t *rp = dst + (int64_t)row * ld + w * 32;
    if (aligned && w * 32 + 32 <= cols) {
        *reinterpret_cast<uint4 *>(rp) = make_uint4(o[0], o[1], o[2], o[3]);
        *reinterpret_cast<uint4 *>(rp + 16) = make_uint4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
        for (int g = 0; g < 8; g++)
#pragma unroll
            for (int j = 0; j < 4; j++)
                if (w * 32 + 4 * g + j < cols) rp[4 * g + j] = (uint8_t)(o[g] >> (8 * j));
    }
}

template <int Q>
__global__ __launch_bounds__(256) void unpack_kernel(const u32 *src, uint8_t *dst, int64_t ld, int rows, int cols, int W,
                                                     int aligned) {
    const int Wc = (cols + 31) / 32;
    const int64_t total = (int64_t)rows * Wc;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x)
        unpack_unit<Q>(src, dst, ld, cols, W, aligned, (int)(idx / Wc), (int)(idx % Wc));
}

// ---------------------------------------------------------------------------------------
// Conversion lists: many pack or unpack jobs of any fields and shapes in one launch.
// Workgroup b serves the job whose first block is the largest one <= b, one (row, word)
// unit per thread.
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ u32 encode_spread_q(int q, u32 v) {
    switch (q) {
    case 3: return encode_spread<3>(v);
    case 4: return encode_spread<4>(v);
    case 5: return encode_spread<5>(v);
    case 8: return encode_spread<8>(v);
    case 9: return encode_spread<9>(v);
    default: return encode_spread<7>(v);
    }
}

__global__ __launch_bounds__(256) void conv_list_kernel(const ConvJob *jobs, int njobs) {
    __shared__ u32 enc[256];
    const u32 b = blockIdx.x;
    int lo = 0, hi = njobs - 1;                   // last job with first_block <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].first_block <= b) lo = mid; else hi = mid - 1;
    }
    const ConvJob j = jobs[lo];
    const int units_w = j.pack ? j.W : (j.cols + 31) / 32;
    const int64_t unit = (int64_t)(b - j.first_block) * 256 + threadIdx.x;
    if (j.pack) {
        enc[threadIdx.x] = encode_spread_q(j.q, threadIdx.x);
        __syncthreads();
    }
    if (unit >= (int64_t)j.rows * units_w) return;
    const int row = (int)(unit / units_w), w = (int)(unit % units_w);
    if (j.pack) {
        const uint8_t *src = (const uint8_t *)j.src;
        u32 *dst = (u32 *)j.dst;
        switch (j.q) {
        case 3: pack_unit<3>(src, j.ld, dst, j.cols, j.W, j.aligned, enc, row, w); break;
        case 4: pack_unit<4>(src, j.ld, dst, j.cols, j.W, j.aligned, enc, row, w); break;
        case 5: pack_unit<5>(src, j.ld, dst, j.cols, j.W, j.aligned, enc, row, w); break;
        case 8: pack_unit<8>(src, j.ld, dst, j.cols, j.W, j.aligned, enc, row, w); break;
        case 9: pack_unit<9>(src, j.ld, dst, j.cols, j.W, j.aligned, enc, row, w); break;
        default: pack_unit<7>(src, j.ld, dst, j.cols, j.W, j.aligned, enc, row, w); break;
        }
    } else {
        const u32 *src = (const u32 *)j.src;
        uint8_t *dst = (uint8_t *)j.dst;
        switch (j.q) {
        case 3: unpack_unit<3>(src, dst, j.ld, j.cols, j.W, j.aligned, row, w); break;
        case 4: unpack_unit<4>(src, dst, j.ld, j.cols, j.W, j.aligned, row, w); break;
        case 5: unpack_unit<5>(src, dst, j.ld, j.cols, j.W, j.aligned, row, w); break;
        case 8: unpack_unit<8>(src, dst, j.ld, j.cols, j.W, j.aligned, row, w); break;
        case 9: unpack_unit<9>(src, dst, j.ld, j.cols, j.W, j.aligned, row, w); break;
        default: unpack_unit<7>(src, dst, j.ld, j.cols, j.W, j.aligned, row, w); break;
        }
    }
}

u32 conv_job_blocks(const ConvJob &j) {
    const int64_t units = (int64_t)j.rows * (j.pack ? j.W : (j.cols + 31) / 32);
    return (u32)((units + 255) / 256);
}

hipError_t launch_conv_list(const ConvJob *jobs, int njobs, u32 blocks, hipStream_t st) {
    if (njobs <= 0 || blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(conv_list_kernel, dim3(blocks), dim3(256), 0, st, jobs, njobs);
    return hipGetLastError();
}

static unsigned grid_for(int64_t work, int per_block);

// Pseudo-random words for the tuner's scratch operands (timing only): a 32-bit mix of the
// word index and a seed.
__global__ __launch_bounds__(256) void fill_random_kernel(u32 *p, size_t n, u32 seed) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        u32 x = (u32)i * 0x9e3779b9u ^ seed ^ (u32)(i >> 32);
        x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
        p[i] = x;
    }
}

// Zero n words (a kernel rather than a memset node, so that captured graphs replay it).
__global__ __launch_bounds__(256) void fill_zero_kernel(uint4 *p, size_t n16) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st) {
    const size_t n16 = bytes / 16;             // packed buffers are whole 16-byte groups
    if (n16 == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for((int64_t)n16, 256)), dim3(256), 0, st, (uint4 *)p, n16);
    return hipGetLastError();
}

hipError_t launch_fill_random(u32 *p, size_t n, u32 seed, hipStream_t st) {
    hipLaunchKernelGGL(fill_random_kernel, dim3(1024), dim3(256), 0, st, p, n, seed);
    return hipGetLastError();
}

hipError_t launch_reduce(int q, const u32 *part, u32 *C, int m, int n, int Wn, int splits, size_t stride, hipStream_t st) {
    const size_t threads = (size_t)m * (Wn / 4);
    dim3 grid((unsigned)((threads + 255) / 256));
    switch (q) {
    case 3: hipLaunchKernelGGL(reduce_partials_kernel<3>, grid, dim3(256), 0, st, part, C, m, n, Wn, splits, stride); break;
    case 4: hipLaunchKernelGGL(reduce_partials_kernel<4>, grid, dim3(256), 0, st, part, C, m, n, Wn, splits, stride); break;
    case 5: hipLaunchKernelGGL(reduce_partials_kernel<5>, grid, dim3(256), 0, st, part, C, m, n, Wn, splits, stride); break;
    case 8: hipLaunchKernelGGL(reduce_partials_kernel<8>, grid, dim3(256), 0, st, part, C, m, n, Wn, splits, stride); break;
    case 9: hipLaunchKernelGGL(reduce_partials_kernel<9>, grid, dim3(256), 0, st, part, C, m, n, Wn, splits, stride); break;
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
    const int aligned = ((uintptr_t)src % 16 == 0) && (ld % 16 == 0);
    dim3 grid(grid_for((int64_t)rows * W, 256));
    switch (q) {
    case 3: hipLaunchKernelGGL(pack_kernel<3>, grid, dim3(256), 0, st, src, ld, dst, rows, cols, W, aligned); break;
    case 4: hipLaunchKernelGGL(pack_kernel<4>, grid, dim3(256), 0, st, src, ld, dst, rows, cols, W, aligned); break;
    case 5: hipLaunchKernelGGL(pack_kernel<5>, grid, dim3(256), 0, st, src, ld, dst, rows, cols, W, aligned); break;
    case 8: hipLaunchKernelGGL(pack_kernel<8>, grid, dim3(256), 0, st, src, ld, dst, rows, cols, W, aligned); break;
    case 9: hipLaunchKernelGGL(pack_kernel<9>, grid, dim3(256), 0, st, src, ld, dst, rows, cols, W, aligned); break;
    default: hipLaunchKernelGGL(pack_kernel<7>, grid, dim3(256), 0, st, src, ld, dst, rows, cols, W, aligned); break;
    }
    return hipGetLastError();
}

hipError_t launch_unpack(int q, const u32 *src, uint8_t *dst, int64_t ld, int rows, int cols, int W, hipStream_t st) {
    const int aligned = ((uintptr_t)dst % 16 == 0) && (ld % 16 == 0);
    dim3 grid(grid_for((int64_t)rows * ((cols + 31) / 32), 256));
    switch (q) {
    case 3: hipLaunchKernelGGL(unpack_kernel<3>, grid, dim3(256), 0, st, src, dst, ld, rows, cols, W, aligned); break;
    case 4: hipLaunchKernelGGL(unpack_kernel<4>, grid, dim3(256), 0, st, src, dst, ld, rows, cols, W, aligned); break;
    case 5: hipLaunchKernelGGL(unpack_kernel<5>, grid, dim3(256), 0, st, src, dst, ld, rows, cols, W, aligned); break;
    case 8: hipLaunchKernelGGL(unpack_kernel<8>, grid, dim3(256), 0, st, src, dst, ld, rows, cols, W, aligned); break;
    case 9: hipLaunchKernelGGL(unpack_kernel<9>, grid, dim3(256), 0, st, src, dst, ld, rows, cols, W, aligned); break;
    default: hipLaunchKernelGGL(unpack_kernel<7>, grid, dim3(256), 0, st, src, dst, ld, rows, cols, W, aligned); break;
    }
    return hipGetLastError();
}

}  // namespace gfq
