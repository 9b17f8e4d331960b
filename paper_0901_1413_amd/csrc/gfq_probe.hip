// gfq_probe.hip -- microbenchmarks of the machine rates the product kernels are measured
// against: three-input bitwise VALU instructions, 128-bit LDS reads in the product's access
// shape, and an HBM copy.  Measurement helpers only; the product never calls them.
#include <hip/hip_runtime.h>

#include "gfq.h"
#include "gfq_host.h"
#include "gfq_internal.h"

using namespace gfq;

namespace {

constexpr int PROBE_NT = 512;
constexpr int VALU_CHAINS = 16;

// Sixteen independent chains of v_bitop3_b32 per lane (three-input XOR, the full adder's sum);
// iters x 16 instructions per lane.  The result is stored only when it equals a value the
// caller's seed makes impossible to know in advance, so nothing is folded away.
__global__ __launch_bounds__(PROBE_NT) void valu_probe_kernel(u32 seed, int iters, u32 *sink) {
    u32 x[VALU_CHAINS];
#pragma unroll
    for (int c = 0; c < VALU_CHAINS; c++) x[c] = seed * (threadIdx.x + 1) + c * 0x9E3779B9u;
    u32 y = seed ^ blockIdx.x, z = seed + threadIdx.x;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int c = 0; c < VALU_CHAINS; c++) x[c] = __builtin_amdgcn_bitop3_b32(x[c], y, z, 0x96);
        y = __builtin_amdgcn_bitop3_b32(y, x[0], z, 0xE8);
    }
    u32 r = 0;
#pragma unroll
    for (int c = 0; c < VALU_CHAINS; c++) r ^= x[c];
    if (r == seed + 0x5bd1e995u) sink[blockIdx.x * PROBE_NT + threadIdx.x] = r;
}

// 128-bit LDS reads: lane l of every 16-lane group reads bytes 16 (l mod 16) .. of a 256-byte
// row (one pass of the 64 banks, conflict-free), sixteen rows per iteration at immediate
// offsets; the four words of each read are folded into two accumulators (two three-input
// XORs per read, so that the VALU stays below the LDS port).
__global__ __launch_bounds__(PROBE_NT) void lds_probe_kernel(u32 seed, int iters, u32 *sink) {
    extern __shared__ __align__(16) uint4 buf[];           // 64 KiB: 256 rows of 256 bytes
    for (int i = threadIdx.x; i < 4096; i += PROBE_NT) buf[i] = make_uint4(seed + i, seed ^ i, i, ~seed);
    __syncthreads();
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    const int lane16 = threadIdx.x & 15;
    const int row0 = (threadIdx.x >> 4) & 15;
    for (int it = 0; it < iters; it++) {
        const uint4 *p = buf + ((row0 + it) & 15) * 16 + lane16;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const uint4 v = p[j * 256];                 // row + 16 j, 4 KiB apart
            acc.x = __builtin_amdgcn_bitop3_b32(acc.x, v.x, v.y, 0x96);
            acc.y = __builtin_amdgcn_bitop3_b32(acc.y, v.z, v.w, 0x96);
        }
    }
    const u32 r = acc.x ^ acc.y;
    if (r == seed + 0x5bd1e995u) sink[blockIdx.x * PROBE_NT + threadIdx.x] = r;
}

// HBM copy in 128-bit words, grid-stride.
__global__ __launch_bounds__(256) void copy_probe_kernel(const uint4 *src, uint4 *dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

// Time `launch` with events on the calling thread's stream; waits for it.
template <typename L> int timed_probe(L launch, float *ms) {
    hipStream_t st = current_stream();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = launch(st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return e == hipSuccess ? GFQ_OK : hip_fail(e, "probe");
}

}  // namespace

extern "C" {

int gfq_probe_valu(int blocks, int iters, u32 *sink, double *lane_ops, float *ms) {
    if (blocks < 1 || iters < 1 || !sink || !lane_ops || !ms) return GFQ_EINVAL;
    *lane_ops = (double)blocks * PROBE_NT * iters * (VALU_CHAINS + 1);
    return timed_probe([&](hipStream_t st) {
        hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(PROBE_NT), 0, st, 0x1234567u, iters, sink);
        return hipGetLastError();
    }, ms);
}

int gfq_probe_lds(int blocks, int iters, u32 *sink, double *bytes, float *ms) {
    if (blocks < 1 || iters < 1 || !sink || !bytes || !ms) return GFQ_EINVAL;
    *bytes = (double)blocks * PROBE_NT * iters * 16 * 16;
    return timed_probe([&](hipStream_t st) {
        hipLaunchKernelGGL(lds_probe_kernel, dim3(blocks), dim3(PROBE_NT), 65536, st, 0x1234567u, iters, sink);
        return hipGetLastError();
    }, ms);
}

int gfq_probe_copy(const void *src, void *dst, size_t bytes, float *ms) {
    if (!src || !dst || !ms || bytes < 16 || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
        return GFQ_EINVAL;
    return timed_probe([&](hipStream_t st) {
        hipLaunchKernelGGL(copy_probe_kernel, dim3(4096), dim3(256), 0, st, (const uint4 *)src, (uint4 *)dst,
                           bytes / 16);
        return hipGetLastError();
    }, ms);
}

}  // extern "C"
