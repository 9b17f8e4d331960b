// gfq_sw.hip -- the elementwise levels of the Strassen–Winograd recursion on packed
// matrices: splitting operands into the seven signed quadrant sums, and merging seven
// half-size products into the quadrants of their parent.  The products themselves are
// Four-Russians products (one strided launch of the plain kernel for all of a level's
// leaves).
//
// Both kernels work on one 32-bit word of every plane per thread (32 elements), with the
// field's addition and negation on the storage code (FT<Q>::sadd, sneg).  A quadrant
// starts at a word boundary (column halves are whole words); rows and columns beyond the
// parent's are read as zero.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gfq_device.h"
#include "gfq_sw.h"

namespace gfq {

namespace {

template <int Q> struct SwDims {
    int rows, cols;        // parent
    int W;                 // words per plane-row of the parent
    int hrows, hcols;      // half (child)
    int hW;                // words per plane-row of a child
};

// r = sum_j coef[j] * x_j over the code planes of one word
template <int Q>
__device__ __forceinline__ void signed_sum(const int *coef, int nterms, const u32 (*x)[FT<Q>::P], u32 *r) {
    constexpr int P = FT<Q>::P;
    bool first = true;
#pragma unroll
    for (int j = 0; j < nterms; j++) {
        if (coef[j] == 0) continue;
        u32 t[P];
        if (coef[j] < 0) FT<Q>::sneg(x[j], t);
        else {
#pragma unroll
            for (int p = 0; p < P; p++) t[p] = x[j][p];
        }
        if (first) {
#pragma unroll
            for (int p = 0; p < P; p++) r[p] = t[p];
            first = false;
        } else {
            u32 s[P];
            FT<Q>::sadd(r, t, s);
#pragma unroll
            for (int p = 0; p < P; p++) r[p] = s[p];
        }
    }
    if (first) {
#pragma unroll
        for (int p = 0; p < P; p++) r[p] = 0u;
    }
}

// Thread = (parent, child row r, child word w): reads the four quadrant words of every
// plane and writes the seven children's words.  Child words at or beyond hcols / 32 are
// pad words and written as zero.
template <int Q, bool LEFT>
__global__ __launch_bounds__(256) void sw_split_kernel(const u32 *in, size_t in_stride, u32 *out, size_t out_stride,
                                                       int parents, SwDims<Q> d) {
    constexpr int P = FT<Q>::P;
    const int hw_valid = d.hcols / 32;
    const int w_valid = (d.cols + 31) / 32;               // parent words holding columns
    const int64_t per = (int64_t)d.hrows * d.hW;
    const int64_t total = per * parents;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int par = (int)(idx / per);
        const int r = (int)((idx % per) / d.hW), w = (int)(idx % d.hW);
        const u32 *src = in + (size_t)par * in_stride;
        u32 *dst = out + (size_t)par * 7 * out_stride;
        u32 x[4][P];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int row = r + (j >> 1) * d.hrows;
            const int word = w + (j & 1) * hw_valid;
            const bool ok = w < hw_valid && row < d.rows && word < w_valid;
#pragma unroll
            for (int p = 0; p < P; p++) x[j][p] = ok ? src[((size_t)row * P + p) * d.W + word] : 0u;
        }
#pragma unroll
        for (int c = 0; c < 7; c++) {
            u32 v[P];
            signed_sum<Q>(LEFT ? SW_A[c] : SW_B[c], 4, x, v);
#pragma unroll
            for (int p = 0; p < P; p++)
                dst[(size_t)c * out_stride + ((size_t)r * P + p) * d.hW + w] = w < hw_valid ? v[p] : 0u;
        }
    }
}

// quadrant QD of a parent product at one word: src points at that word of product 0
template <int Q, int QD>
__device__ __forceinline__ void quadrant_sum(const u32 *src, size_t prod_stride, int hW, u32 *v) {
    constexpr int P = FT<Q>::P;
    u32 x[7][P];
#pragma unroll
    for (int c = 0; c < 7; c++)
#pragma unroll
        for (int p = 0; p < P; p++) x[c][p] = SW_C[QD][c] != 0 ? src[(size_t)c * prod_stride + (size_t)p * hW] : 0u;
    signed_sum<Q>(SW_C[QD], 7, x, v);
}

// Thread = (parent, row r, word w) of the parent product: the quadrant it lies in is a
// signed sum of the seven products at the same position; the result is canonicalised
// and its columns beyond the parent's are zeroed.
template <int Q>
__global__ __launch_bounds__(256) void sw_merge_kernel(const u32 *prods, size_t prod_stride, u32 *out,
                                                       size_t out_stride, int parents, SwDims<Q> d) {
    constexpr int P = FT<Q>::P;
    const int hw_valid = d.hcols / 32;
    const int64_t per = (int64_t)d.rows * d.W;
    const int64_t total = per * parents;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int par = (int)(idx / per);
        const int r = (int)((idx % per) / d.W), w = (int)(idx % d.W);
        const bool top = r < d.hrows, left = w < hw_valid;
        const int rr = top ? r : r - d.hrows, ww = left ? w : w - hw_valid;
        const int cw = w * 32;
        const u32 msk = cw >= d.cols ? 0u : (d.cols - cw >= 32 ? 0xffffffffu : ((1u << (d.cols - cw)) - 1u));
        u32 v[P];
        if (msk != 0u && ww < hw_valid) {
            const u32 *src = prods + (size_t)par * 7 * prod_stride + ((size_t)rr * P) * d.hW + ww;
            switch ((top ? 0 : 2) + (left ? 0 : 1)) {
            case 0: quadrant_sum<Q, 0>(src, prod_stride, d.hW, v); break;
            case 1: quadrant_sum<Q, 1>(src, prod_stride, d.hW, v); break;
            case 2: quadrant_sum<Q, 2>(src, prod_stride, d.hW, v); break;
            default: quadrant_sum<Q, 3>(src, prod_stride, d.hW, v); break;
            }
            FT<Q>::scanon(v);
        } else {
#pragma unroll
            for (int p = 0; p < P; p++) v[p] = 0u;
        }
        u32 *dst = out + (size_t)par * out_stride;
#pragma unroll
        for (int p = 0; p < P; p++) dst[((size_t)r * P + p) * d.W + w] = v[p] & msk;
    }
}

unsigned grid_of(int64_t work) {
    int64_t g = (work + 255) / 256;
    if (g > 256 * 64) g = 256 * 64;
    return (unsigned)(g < 1 ? 1 : g);
}

template <int Q>
hipError_t split_q(bool left, const u32 *in, size_t in_stride, u32 *out, size_t out_stride, int parents, int rows,
                   int cols, int hrows, int hcols, hipStream_t st) {
    const SwDims<Q> d = {rows, cols, words_of(cols), hrows, hcols, words_of(hcols)};
    const dim3 grid(grid_of((int64_t)hrows * d.hW * parents));
    if (left)
        hipLaunchKernelGGL((sw_split_kernel<Q, true>), grid, dim3(256), 0, st, in, in_stride, out, out_stride, parents, d);
    else
        hipLaunchKernelGGL((sw_split_kernel<Q, false>), grid, dim3(256), 0, st, in, in_stride, out, out_stride, parents, d);
    return hipGetLastError();
}

template <int Q>
hipError_t merge_q(const u32 *prods, size_t prod_stride, u32 *out, size_t out_stride, int parents, int rows, int cols,
                   int hrows, int hcols, hipStream_t st) {
    const SwDims<Q> d = {rows, cols, words_of(cols), hrows, hcols, words_of(hcols)};
    const dim3 grid(grid_of((int64_t)rows * d.W * parents));
    hipLaunchKernelGGL(sw_merge_kernel<Q>, grid, dim3(256), 0, st, prods, prod_stride, out, out_stride, parents, d);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sw_split(int q, bool left, const u32 *in, size_t in_stride, u32 *out, size_t out_stride,
                           int parents, int rows, int cols, int hrows, int hcols, hipStream_t st) {
    if (hcols % 32 != 0 || 2 * (int64_t)hcols < cols || 2 * (int64_t)hrows < rows) return hipErrorInvalidValue;
    switch (q) {
    case 3: return split_q<3>(left, in, in_stride, out, out_stride, parents, rows, cols, hrows, hcols, st);
    case 4: return split_q<4>(left, in, in_stride, out, out_stride, parents, rows, cols, hrows, hcols, st);
    case 5: return split_q<5>(left, in, in_stride, out, out_stride, parents, rows, cols, hrows, hcols, st);
    case 7: return split_q<7>(left, in, in_stride, out, out_stride, parents, rows, cols, hrows, hcols, st);
    case 8: return split_q<8>(left, in, in_stride, out, out_stride, parents, rows, cols, hrows, hcols, st);
    case 9: return split_q<9>(left, in, in_stride, out, out_stride, parents, rows, cols, hrows, hcols, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sw_merge(int q, const u32 *prods, size_t prod_stride, u32 *out, size_t out_stride, int parents,
                           int rows, int cols, int hrows, int hcols, hipStream_t st) {
    if (hcols % 32 != 0 || 2 * (int64_t)hcols < cols || 2 * (int64_t)hrows < rows) return hipErrorInvalidValue;
    switch (q) {
    case 3: return merge_q<3>(prods, prod_stride, out, out_stride, parents, rows, cols, hrows, hcols, st);
    case 4: return merge_q<4>(prods, prod_stride, out, out_stride, parents, rows, cols, hrows, hcols, st);
    case 5: return merge_q<5>(prods, prod_stride, out, out_stride, parents, rows, cols, hrows, hcols, st);
    case 7: return merge_q<7>(prods, prod_stride, out, out_stride, parents, rows, cols, hrows, hcols, st);
    case 8: return merge_q<8>(prods, prod_stride, out, out_stride, parents, rows, cols, hrows, hcols, st);
    case 9: return merge_q<9>(prods, prod_stride, out, out_stride, parents, rows, cols, hrows, hcols, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace gfq
