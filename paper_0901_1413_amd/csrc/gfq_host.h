// gfq_host.h -- host helpers shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "gfq.h"
#include "gfq_batch.h"
#include "gfq_internal.h"

namespace gfq {

// Record a HIP failure for gfq_last_hip_error and return GFQ_EHIP.
int hip_fail(hipError_t e, const char *what);
// The calling thread's stream (gfq_set_stream).
hipStream_t current_stream();
// Build a batch; cfgs (optional, one per product) overrides the per-product configuration.
int batch_create_with(int count, const gfq_problem *problems, const gfq_config *cfgs, gfq_batch **out);
// The tiles of one (field, rows per lane) work list of a batch.
struct BatchGroup {
    int q = 0, R = 0, twd = 16, kmax = 1;
    size_t lds = 0;                  // dynamic LDS of the list's launch
    size_t item_off = 0;             // index of the group's first item in the batch's item array
    int queue_wgs = 0;               // persistent workgroups of the list's queue launch
    std::vector<BatchItem> items;    // longest first
    std::vector<double> cost;        // planning only
};
// Slab slices of a batch's products.  A product whose tiles would each take more than half of
// a compute unit's share of the batch (few tiles, a long inner dimension) is cut into slices
// of at least 8 slabs; product i's partial products take slices x m x P x Wn words at word
// offset part_off[i] of a workspace of partial_words words (the caller points a.out there),
// and `reduce` lists the partial-sum items of every sliced product.
struct BatchSlicing {
    int cus = 256;                     // compute units of the device
    size_t partial_words = 0;
    std::vector<size_t> part_off;
    std::vector<ReduceItem> reduce;
};
// Per-product launch parameters (prods[0 .. count)) and the non-empty work lists, with
// consecutive item offsets; *nitems = total items.  Without `slicing` every product is whole
// tiles.  The problems must be valid.
void plan_batch(int count, const gfq_problem *problems, const gfq_config *cfgs, BatchProd *prods,
                std::vector<BatchGroup> *groups, size_t *nitems, BatchSlicing *slicing = nullptr);
// Launch every group's work list: the first on st, the others forked onto side streams of
// st and joined back into it (one after another on st while st is captured and has no side
// streams yet).  base: the batch's lists with items pointing at item 0.  With queue_heads
// (one zeroed head per group), each list is drained by its persistent workgroups instead.
hipError_t launch_group_lists(const std::vector<BatchGroup> &groups, const BatchList &base, hipStream_t st,
                              u32 *queue_heads = nullptr);
// Upper bound of the tiles of an m x n product in any batch (the smallest tile height).
size_t batch_tiles_bound(int64_t m, int64_t n);
// Allow every batched work-list kernel the dynamic LDS of its largest slab width.
hipError_t set_batched_lds_limits();
// Fill n words with pseudo-random bits (a hash of the index and the seed); timing data only.
hipError_t launch_fill_random(u32 *p, size_t n, u32 seed, hipStream_t st);
// Tile height and inner-dimension slices of an m x l x n product for slab width c->k, by a
// cost model of slab steps per compute unit, slices of at least min_slabs slabs (keep_rows:
// only the slices, for c->rows).
void fit_tiles(int q, int64_t m, int64_t l, int64_t n, gfq_config *c, bool keep_rows = false, int min_slabs = 32);
// Field, dimension, pointer, alignment and aliasing checks of one product.
int validate_mm(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B, void *C);
// Range checks of an explicit configuration for field q (GFQ_OK or GFQ_EINVAL).
int check_config(int q, const gfq_config &c);
// One product as gfq_matmul_config (cfg NULL: the chosen configuration).  With fixed_ws, the
// split-l partial products go to that device region of fixed_bytes instead of the
// per-(device, stream) workspace, nothing is allocated and no launch is timed; a chosen split
// is lowered until its partials fit, an explicit one whose partials do not fit returns
// GFQ_EBUDGET.
int matmul_into(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B, void *C,
                const gfq_config *cfg, void *fixed_ws, size_t fixed_bytes);

}  // namespace gfq
