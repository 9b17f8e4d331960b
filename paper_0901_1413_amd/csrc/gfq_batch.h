// gfq_batch.h -- device-side descriptors of a batched launch (shared by the work-list
// kernel and the host code that builds the lists).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gfq_internal.h"

namespace gfq {

struct BatchProd {
    MMArgs a;              // the product as a single-product launch sees it: with slab slices
                           // a.out is the first slice's partial product (a.split_stride apart)
    u32 units;             // work units until the product is complete: tiles x slices, plus
                           // one partial-sum item per chunk of a sliced product
    u32 slices;            // slab slices (1: the tiles write C directly)
    u32 *C;                // the product
    int q;                 // field (the storage addition of the partial sums)
    int pad;
};

struct BatchItem {
    u32 prod;              // index into the product table
    uint16_t tx, ty;       // column tile, row tile
    u32 slice;             // slab slice
};

struct BatchList {
    const BatchProd *prods;
    const BatchItem *items;            // this list's items, longest first (one per workgroup)
    u32 *prod_done;                    // work units finished per product (cleared on completion)
    unsigned long long *prod_time;     // completion time per product (100 MHz clock)
};

// A partial-sum item: groups [first, first + count) of a sliced product, a group being one
// row's four words of every plane (row = group / (Wn / 4)).
struct ReduceItem {
    u32 prod;
    u32 first, count;
};

struct ReduceList {
    const BatchProd *prods;
    const ReduceItem *items;
    u32 *prod_done;
    unsigned long long *prod_time;
};

// Work-list kernel for field q with R rows per lane and tiles TWD words wide per plane: 16
// (512 columns; super-rows of batch_srb(q, R) bytes), or 8 and 4 (256 and 128 columns, two
// rows per lane, 8 and 16 copies per 256-byte super-row) for products narrower than a wide
// tile.
const void *batched_kernel(int q, int R, int twd);
hipError_t launch_batched(int q, int R, int twd, const BatchList &bl, int items, size_t lds, hipStream_t st);
// The same lists drained by persistent workgroups (gfq_drain.h): `workgroups` of them take
// items in list order from the queue head *head, which launch_queue_reset zeroes (up to 64
// heads) and which must be zero when the launch starts.  Dynamic LDS: the list's plus one
// 16-byte slot for the published index (queue_lds).
const void *queue_kernel(int q, int R, int twd);
inline size_t queue_lds(size_t lds) { return ((lds + 15) & ~(size_t)15) + 16; }
hipError_t launch_queue(int q, int R, int twd, const BatchList &bl, int items, size_t lds, u32 *head, int workgroups,
                        hipStream_t st);
hipError_t launch_queue_reset(u32 *heads, int n, hipStream_t st);
// The partial sums of every sliced product of a batch: one workgroup per item, any fields.
hipError_t launch_reduce_list(const ReduceList &rl, int items, hipStream_t st);
hipError_t launch_batch_stamp(unsigned long long *t, hipStream_t st);

}  // namespace gfq
