// gfq_internal.h -- declarations shared by the C-ABI layer and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gfq {

typedef uint32_t u32;

constexpr int KMAX = 10;          // largest slab width
constexpr int NT_MM = 512;        // threads per product workgroup
constexpr size_t TABLES_LDS = 131072;   // LDS for the two table buffers

constexpr int log2_floor(int x) { return x <= 1 ? 0 : 1 + log2_floor(x / 2); }

struct MMArgs {
    const u32 *A;          // packed m x l
    const u32 *B;          // packed l x n
    u32 *out;              // packed m x n (C, or the first partial product)
    int m, l, n;           // elements
    int Wl, Wn;            // words per plane-row of A, of B and C
    int k;                 // slab width
    int S;                 // slabs = ceil(l / k)
    int slabs_per_split;   // slabs per grid.z slice
    size_t split_stride;   // words between consecutive partial products
    u32 tb1;               // LDS offset of the second table (set by the launcher)
};

// Kernel fields of the matrix-level product routes (chosen by gfq_config.variant for the
// API fields q = 4, 8, 9): GF(4) by Karatsuba over F_2, GF(8) by the trinomial formula over
// F_2, F_9 by Karatsuba over F_3.
constexpr int GF4_KARATSUBA = 40;
constexpr int GF8_TRINOMIAL = 80;
constexpr int F9_KARATSUBA = 90;

// API fields with a matrix-level product route (gfq_config.variant 1), and the kernel
// field of a product over API field q in route `variant` (0: row-wise)
inline bool has_matrix_route(int q) { return q == 4 || q == 8 || q == 9; }
inline int route_field(int q, int variant) {
    if (variant != 1) return q;
    return q == 4 ? GF4_KARATSUBA : (q == 8 ? GF8_TRINOMIAL : (q == 9 ? F9_KARATSUBA : q));
}

// fields of the C ABI: F_3, F_5, F_7, GF(4) (q = 4), GF(8) (q = 8) and F_9 (q = 9)
inline bool valid_field(int q) { return q == 3 || q == 4 || q == 5 || q == 7 || q == 8 || q == 9; }

// planes per packed row; planes per table entry; table rows gathered per slab
inline int planes_of(int q) {
    return (q == 3 || q == 4 || q == GF4_KARATSUBA) ? 2 : ((q == 9 || q == F9_KARATSUBA) ? 4 : 3);
}
inline int table_planes(int q) {
    return q == GF4_KARATSUBA ? 3 : ((q == GF8_TRINOMIAL || q == F9_KARATSUBA) ? 6 : planes_of(q));
}

// Table slots per entry: its planes, and for F_7 and GF(8) at 128-byte super-rows one more
// slot in front (the second row of every read pass reads a fixed multiple of the entry through
// it, conflict-free; see the product tile).
inline int table_slots(int q, int srb) { return ((q == 7 || q == 8) && srb == 128) ? 4 : table_planes(q); }
inline int gathers_of(int q) {
    return (q == 3 || q == 4) ? 2 : (q == 9 ? 4 : ((q == GF8_TRINOMIAL || q == F9_KARATSUBA) ? 6 : 3));
}
inline bool split_prefix(int q) { return q == 5 || q == 7; }   // FT<q>::SPLIT_PREFIX
inline int words_of(int64_t cols) { return (int)(((cols + 127) / 128) * 4); }
// Rows of C per lane: bounded by the accumulator registers (6 planes per word for F_7, 4 for
// F_9, 3 for F_5 and GF(8), 2 for F_3 and GF(4)) and the gathered table rows in flight (F_9
// by Karatsuba: two rows of twelve 128-bit reads and 12 accumulator planes).  The work-list
// kernels of batches use at most 8.
inline int max_rows_per_lane(int q) {
    return q == F9_KARATSUBA ? 2 : (q == 7 ? 4 : (q == 3 || q == 4 || q == GF4_KARATSUBA ? 16 : 8));
}
inline int max_rows_per_lane_batch(int q) { return q == 5 || q == 7 || q == 9 ? 4 : 8; }

// Table super-row bytes for field q and slab width k: the widest of 256, 128, 64, 32, 16
// such that both table buffers fit TABLES_LDS (0 if none does).
inline int srb_for(int q, int k) {
    for (int srb = 256; srb >= 16; srb >>= 1)
        if (2 * ((size_t)1 << k) * table_slots(q, srb) * srb <= TABLES_LDS) return srb;
    return 0;
}
// tile words per plane: 128-byte super-rows hold one 32-word row, 256-byte ones four copies
// of a 16-word row, 64-byte ones one 16-word row, narrower ones one row of srb / 4 words
inline int twd_of(int srb) { return srb == 128 ? 32 : (srb >= 64 ? 16 : srb / 4); }

// Super-row bytes of the batched (work-list) kernels of field q at R rows per lane: 256 (four
// copies of the 16-word tile row, conflict-free reads), except F_5 and F_7 at four rows per
// lane: one copy (64 bytes; reads may conflict, but the tables then hold slabs up to k = 8,
// and F_5 fits its registers only so).  Measured on the 4096-product batch: F_5 4.06 -> 3.14
// ms, F_7 3.81 -> 3.41 ms; F_3 at 128 bytes gained nothing.
inline int batch_srb(int q, int R) { return ((q == 5 || q == 7) && R == 4) ? 64 : 256; }
// largest slab width whose two tables fit LDS with super-rows of batch_srb(q, R) bytes
inline int batch_kmax(int q, int R) {
    const int srb = batch_srb(q, R);
    int k = 1;
    while (k < KMAX && 2 * ((size_t)1 << (k + 1)) * table_slots(q, srb) * srb <= TABLES_LDS) k++;
    return k;
}

// Everything a product launch needs, derived from (field, slab width, requested tile rows).
struct MMPlan {
    int srb;      // table super-row bytes
    int twd;      // tile width in words per plane
    int rep;      // copies of the tile row per super-row
    int R;        // rows of C per lane (2, 4, 8 or 16)
    int TM;       // rows of C per workgroup
    u32 tb1;      // LDS offset of the second table
    size_t lds;   // dynamic LDS bytes
};

inline size_t mm_lds_bytes(int q, int k, int srb, int TM, u32 *tb1_out) {
    const int P = planes_of(q), PT = table_planes(q), D = gathers_of(q);
    const u32 tbytes = (u32)(1u << k) * table_slots(q, srb) * srb;
    u32 tb1 = 16;
    while (tb1 < tbytes) tb1 <<= 1;
    if (tb1_out) *tb1_out = tb1;
    // two tables, B staging [3][KMAX][P][TWD], chunk prefixes [2][NT/TWD][PT][TWD] (F_5,
    // F_7 only), table offsets [3][TM][(D+1)/2]
    return (size_t)tb1 + tbytes + 3 * KMAX * P * twd_of(srb) * 4 + (split_prefix(q) ? 2 * (size_t)NT_MM * PT * 4 : 0) +
           3 * (size_t)TM * ((D + 1) / 2) * 4;
}

// srb = 0 when k is out of range; otherwise the largest R (rows per lane) not above the
// request whose LDS footprint fits the 160 KiB of a workgroup.
inline MMPlan mm_plan(int q, int k, int rowsTile) {
    MMPlan p = {};
    if (k < 1 || k > KMAX) return p;
    p.srb = srb_for(q, k);
    if (!p.srb) return p;
    p.twd = twd_of(p.srb);
    p.rep = p.srb / (4 * p.twd);
    const int lpr = p.twd / 4;
    int r = rowsTile * lpr / NT_MM;
    r = r <= 2 ? 2 : (r <= 4 ? 4 : (r <= 8 ? 8 : 16));
    if (r > max_rows_per_lane(q)) r = max_rows_per_lane(q);
    if (r > 8 && p.twd != 16 && !((q == 3 || q == 4) && p.twd == 32)) r = 8;   // 16 rows per lane: 16-word tiles (F_3, GF(4): and 32)
    if (r > 4 && p.twd < 16 && (q == 5 || q == 8 || q == GF8_TRINOMIAL)) r = 4;   // ... for F_5, GF(8) eight would
    if (r > 4 && p.twd < 32 && q == 9) r = 4;           // F_9: eight rows per lane on 32-word tiles only,
    if (r > 2 && p.twd < 16 && q == 9) r = 2;           // two on narrow ones (four would spill)
    if (p.twd == 4 && q == 3 && r > 4) r = 4;            // 4-word tiles stage R * 4 rows per thread:
    if (p.twd == 4 && q == 7 && r > 2) r = 2;            // F_3 at eight and F_7 at four would spill
    for (; r >= 2; r /= 2) {
        p.R = r;
        p.TM = NT_MM / lpr * r;
        p.lds = mm_lds_bytes(q, k, p.srb, p.TM, &p.tb1);
        if (p.lds <= 163840) return p;
    }
    p.srb = 0;
    return p;
}

// count products of one shape in one launch: product p reads A + p * A_stride and
// B + p * B_stride and writes out + p * out_stride (strides in 32-bit words)
struct MMStrides {
    int count;
    size_t A, B, out;
};

// product launches for kernel field Q (explicitly instantiated in gfq_m4rm_<field>.hip)
template <bool STRIDED, int Q>
hipError_t launch_mm_q(const MMArgs &a, const MMPlan &plan, const MMStrides &sd, hipStream_t st);

hipError_t launch_matmul(int q, const MMArgs &a, const MMPlan &plan, hipStream_t st);
hipError_t launch_matmul_strided(int q, const MMArgs &a, const MMPlan &plan, const MMStrides &sd, hipStream_t st);

// Strassen–Winograd levels: the seven signed quadrant sums of every one of `parents`
// packed matrices (stride in_stride words, rows x cols) into 7 * parents matrices (stride
// out_stride, hrows x hcols, hcols a multiple of 32); `left` selects the coefficients of
// the left or the right operand.  merge: quadrants of every parent product (rows x cols)
// from its seven half-size products.
hipError_t launch_sw_split(int q, bool left, const u32 *in, size_t in_stride, u32 *out, size_t out_stride,
                           int parents, int rows, int cols, int hrows, int hcols, hipStream_t st);
hipError_t launch_sw_merge(int q, const u32 *prods, size_t prod_stride, u32 *out, size_t out_stride, int parents,
                           int rows, int cols, int hrows, int hcols, hipStream_t st);
hipError_t launch_reduce(int q, const u32 *part, u32 *C, int m, int n, int Wn, int splits, size_t stride, hipStream_t st);
// One pack (uint8 -> planes) or unpack (planes -> uint8) job of a conversion list.  The
// uint8 side has leading dimension ld; the packed side has W words per plane row.  Jobs are
// ordered by first_block, the first workgroup of the job in the launch (the first job's is
// 0); a job covers ceil(rows * units per row / 256) workgroups.
struct ConvJob {
    const void *src;
    void *dst;
    int64_t ld;
    int rows, cols, W;
    int q, pack, aligned;
    u32 first_block;
    u32 pad;
};
u32 conv_job_blocks(const ConvJob &j);
hipError_t launch_conv_list(const ConvJob *jobs, int njobs, u32 blocks, hipStream_t st);

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st);
hipError_t launch_pack(int q, const uint8_t *src, int64_t ld, u32 *dst, int rows, int cols, int W, hipStream_t st);
hipError_t launch_unpack(int q, const u32 *src, uint8_t *dst, int64_t ld, int rows, int cols, int W, hipStream_t st);

}  // namespace gfq
