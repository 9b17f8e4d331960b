// gfq_batch.hip -- many independent products in one launch per (field, tile height): the
// grid is a work list of (product, row tile, column tile, slab slice) items, longest first.
//
// Each product keeps its own shape and slab width k; the items of one list share a field
// and a tile height (rows per lane R), so one kernel instance serves them.  Workgroup b
// takes item b and runs the tile with the same body as the single-product kernel; the
// hardware dispatcher hands items to compute units as they free up, in list order, so the
// longest items start first and the tail of the launch is short.  A product whose tiles
// would each take a large share of the batch (few tiles, a long inner dimension) is cut
// into slab slices as well: each slice's items write a partial product, and a partial-sum
// list (one launch for every sliced product, after the work lists) adds them into C.  The
// workgroup that finishes a product's last unit of work stamps the product's completion
// time (100 MHz constant clock) and clears the product's count, so the same lists can be
// launched again.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gfq_batch.h"
#include "gfq_m4rm_tile.h"
#include "gfq_reduce.h"
#define GFQ_DRAIN_FN __device__ __forceinline__
#include "gfq_drain.h"

namespace gfq {


// One item of a work list: the tile, then (after every thread has stored) the product's
// completion count and stamp.
template <int Q, int TWD, int REP, int R, int NT>
__device__ __forceinline__ void run_item(const BatchList &bl, u32 i) {
    const BatchItem item = bl.items[i];
    const MMArgs a = bl.prods[item.prod].a;
    m4rm_tile_fit<Q, TWD, REP, R, NT>(a, item.tx, item.ty, (int)item.slice);
    __syncthreads();
    if (threadIdx.x == 0) {
        const u32 d = atomicAdd(&bl.prod_done[item.prod], 1u);
        if (d + 1 == bl.prods[item.prod].units) {
            bl.prod_time[item.prod] = __builtin_amdgcn_s_memrealtime();
            bl.prod_done[item.prod] = 0u;
        }
    }
}

template <int Q, int TWD, int REP, int R, int NT>
__global__ __launch_bounds__(NT) void m4rm_list_kernel(BatchList bl) {
    run_item<Q, TWD, REP, R, NT>(bl, blockIdx.x);
}

// The persistent workgroup's side of the drain loop (gfq_drain.h): the barrier, an LDS word
// past the tile's buffers for the published index, and the list's queue head.
template <int Q, int TWD, int REP, int R, int NT>
struct QueueCtx {
    const BatchList &bl;
    u32 *head;
    u32 *slot;
    // the first wave, by a value the compiler knows to be uniform
    __device__ bool leader() const { return __builtin_amdgcn_readfirstlane(threadIdx.x / 64u) == 0u; }
    __device__ void barrier() { __syncthreads(); }
    // every lane of the wave adds (lane 0 adds 1, the others 0), so no lane branches; lane 0's
    // result is the ticket
    __device__ u32 fetch_head() {
        const u32 r = atomicAdd(head, (threadIdx.x & 63u) == 0u ? 1u : 0u);
        return __builtin_amdgcn_readlane(r, 0);
    }
    __device__ void slot_store(u32 v) { *slot = v; }
    __device__ u32 slot_load() { return *slot; }
    __device__ u32 uniform(u32 v) { return __builtin_amdgcn_readfirstlane(v); }
    __device__ void run(u32 i) { run_item<Q, TWD, REP, R, NT>(bl, i); }
};

// Persistent workgroups (as many as the device holds at once) draining the list's items in
// order: workgroup w takes the next index from the queue head until the list is exhausted.
// The head is zeroed by queue_reset_kernel before every launch.
template <int Q, int TWD, int REP, int R, int NT>
__global__ __launch_bounds__(NT) void m4rm_queue_kernel(BatchList bl, u32 items, u32 *head, u32 slot_off) {
    extern __shared__ __align__(16) unsigned char smem[];
    QueueCtx<Q, TWD, REP, R, NT> c{bl, head, reinterpret_cast<u32 *>(smem + slot_off)};
    drain_queue(c, items);
}

__global__ void queue_reset_kernel(u32 *heads, int n) {
    if ((int)threadIdx.x < n) heads[threadIdx.x] = 0u;
}

// Partial sums of sliced products: item b adds the slices of its groups into C; the item
// that finishes a product's last unit stamps and clears it, as the work lists do.
__global__ __launch_bounds__(256) void reduce_list_kernel(ReduceList rl) {
    const ReduceItem it = rl.items[blockIdx.x];
    const BatchProd &p = rl.prods[it.prod];
    const u32 *part = p.a.out;
    u32 *C = p.C;
    const int n = p.a.n, Wn = p.a.Wn, slices = (int)p.slices, q = p.q;
    const size_t stride = p.a.split_stride;
    const u32 groups = (u32)(Wn / 4);
    for (u32 u = it.first + threadIdx.x; u < it.first + it.count; u += blockDim.x) {
        const int row = (int)(u / groups), w = (int)(u % groups) * 4;
        switch (q) {                             // one field per item: a uniform branch
        case 3: reduce_group<3>(part, C, row, w, n, Wn, slices, stride); break;
        case 4: reduce_group<4>(part, C, row, w, n, Wn, slices, stride); break;
        case 5: reduce_group<5>(part, C, row, w, n, Wn, slices, stride); break;
        case 8: reduce_group<8>(part, C, row, w, n, Wn, slices, stride); break;
        case 9: reduce_group<9>(part, C, row, w, n, Wn, slices, stride); break;
        default: reduce_group<7>(part, C, row, w, n, Wn, slices, stride); break;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const u32 d = atomicAdd(&rl.prod_done[it.prod], 1u);
        if (d + 1 == p.units) {
            rl.prod_time[it.prod] = __builtin_amdgcn_s_memrealtime();
            rl.prod_done[it.prod] = 0u;
        }
    }
}

// Start of a batch launch on the same clock (completion times are relative to it).
__global__ void batch_stamp_kernel(unsigned long long *t) {
    if (threadIdx.x == 0) t[0] = __builtin_amdgcn_s_memrealtime();
}

template <bool QUEUE, int Q, int TWD, int REP, int R>
static const void *kernel_ptr() {
    return QUEUE ? (const void *)m4rm_queue_kernel<Q, TWD, REP, R, NT_MM> : (const void *)m4rm_list_kernel<Q, TWD, REP, R, NT_MM>;
}

template <bool QUEUE, int Q, int R, int REP = 4>
static const void *list_kernel_ptr() {
    return kernel_ptr<QUEUE, Q, 16, REP, R>();
}

// narrow tiles: two rows per lane, TWD words per plane, 64 / TWD copies per 256-byte super-row
template <bool QUEUE, int Q>
static const void *narrow_kernel_ptr(int twd) {
    return twd == 8 ? kernel_ptr<QUEUE, Q, 8, 8, 2>() : kernel_ptr<QUEUE, Q, 4, 16, 2>();
}

template <bool QUEUE>
static const void *kernel_for(int q, int R, int twd) {
    if (twd != 16) {
        switch (q) {
        case 3: return narrow_kernel_ptr<QUEUE, 3>(twd);
        case 4: return narrow_kernel_ptr<QUEUE, 4>(twd);
        case 5: return narrow_kernel_ptr<QUEUE, 5>(twd);
        case 8: return narrow_kernel_ptr<QUEUE, 8>(twd);
        case 9: return narrow_kernel_ptr<QUEUE, 9>(twd);
        default: return narrow_kernel_ptr<QUEUE, 7>(twd);
        }
    }
    switch (q) {
    case 3: return R == 2 ? list_kernel_ptr<QUEUE, 3, 2>() : list_kernel_ptr<QUEUE, 3, 8>();
    case 4: return R == 2 ? list_kernel_ptr<QUEUE, 4, 2>() : list_kernel_ptr<QUEUE, 4, 8>();
    case 5: return R == 2 ? list_kernel_ptr<QUEUE, 5, 2>() : list_kernel_ptr<QUEUE, 5, 4, 1>();   // batch_srb: 64 at R = 4
    case 8: return R == 2 ? list_kernel_ptr<QUEUE, 8, 2>() : list_kernel_ptr<QUEUE, 8, 8>();
    case 9: return R == 2 ? list_kernel_ptr<QUEUE, 9, 2>() : list_kernel_ptr<QUEUE, 9, 4>();
    default: return R == 2 ? list_kernel_ptr<QUEUE, 7, 2>() : list_kernel_ptr<QUEUE, 7, 4, 1>();   // batch_srb: 64 at R = 4
    }
}

const void *batched_kernel(int q, int R, int twd) { return kernel_for<false>(q, R, twd); }
const void *queue_kernel(int q, int R, int twd) { return kernel_for<true>(q, R, twd); }

hipError_t launch_batched(int q, int R, int twd, const BatchList &bl, int items, size_t lds, hipStream_t st) {
    const void *k = batched_kernel(q, R, twd);
    if (!k) return hipErrorInvalidValue;
    void *args[] = {(void *)&bl};
    return hipLaunchKernel(k, dim3(items), dim3(NT_MM), args, lds, st);
}

hipError_t launch_queue(int q, int R, int twd, const BatchList &bl, int items, size_t lds, u32 *head, int workgroups,
                        hipStream_t st) {
    const void *k = queue_kernel(q, R, twd);
    if (!k || workgroups < 1) return hipErrorInvalidValue;
    u32 n = (u32)items, slot_off = (u32)((lds + 15) & ~(size_t)15);
    void *args[] = {(void *)&bl, (void *)&n, (void *)&head, (void *)&slot_off};
    return hipLaunchKernel(k, dim3(workgroups), dim3(NT_MM), args, queue_lds(lds), st);
}

hipError_t launch_queue_reset(u32 *heads, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, st, heads, n);
    return hipGetLastError();
}

hipError_t launch_reduce_list(const ReduceList &rl, int items, hipStream_t st) {
    if (items <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_list_kernel, dim3(items), dim3(256), 0, st, rl);
    return hipGetLastError();
}

hipError_t launch_batch_stamp(unsigned long long *t, hipStream_t st) {
    hipLaunchKernelGGL(batch_stamp_kernel, dim3(1), dim3(64), 0, st, t);
    return hipGetLastError();
}

}  // namespace gfq
