/*
 * gfq.h -- C ABI of libgfq: dense matrix products C = A B over F_3, F_5, F_7 and
 * GF(4) = F_2[x]/(x^2 + x + 1) on one AMD Instinct MI355X (gfx950), computed by the
 * Method of Four Russians with an additive basis on bitsliced rows (Boothby and
 * Bradshaw, "Bitslicing and the Method of Four Russians Over Larger Finite Fields":
 * Section 2 for the method, Section 3 for the row-wise bitsliced format, Section 4 for
 * the field encodings).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Field selector q is 3, 5 or 7 for the prime fields and 4 for GF(4).  Any other value
 *    returns GFQ_EFIELD.
 *  - Unpacked matrices are uint8, row-major with a leading dimension in elements, holding
 *    canonical representatives: 0..q-1 for F_q; for F_3 the value 2 stands for -1; for
 *    GF(4) the value c0 + 2 c1 stands for c0 + c1 x.
 *  - Packed matrices use the row-wise bitsliced format of Section 3, the same format for
 *    the left operand, the right operand and the product.  A matrix of R rows and N
 *    columns over a field with P bit-planes (P = 2 for F_3 and GF(4), P = 3 for F_5, F_7)
 *    occupies R * P * W 32-bit words with W = ceil(N / 128) * 4: row r holds plane 0,
 *    then plane 1, ..., each W little-endian words; element j of the row is bit (j mod 32)
 *    of word (j / 32) of each plane.  Element encodings per plane:
 *        F_3 (Section 4.1): plane 0 marks a unit, plane 1 the sign (0 = 00, 1 = 10, -1 = 11)
 *        F_5, F_7 (Section 4.2): plane d is binary digit d of the representative
 *        GF(4) (Section 4.3): plane d is the coefficient c_d
 *    Bits beyond column N-1 ("pad bits") are zero in every buffer this library writes.
 *    Products are written canonical (F_5, F_7: representatives below q), so a packed
 *    product is unique.
 *  - All device buffers are owned by the caller, live in the memory of the current HIP
 *    device, and must be 16-byte aligned when packed.  Calls are asynchronous on the
 *    calling thread's stream (gfq_set_stream); arguments are validated before anything is
 *    launched, and on a validation error no output is touched.
 *  - Every call returns GFQ_OK (0) or a negative status; no call throws.
 */
#ifndef GFQ_H
#define GFQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GFQ_OK = 0,
    GFQ_EINVAL = -1,  /* malformed argument not covered below (e.g. bad config field)  */
    GFQ_EFIELD = -2,  /* q not in {3, 4, 5, 7}                                          */
    GFQ_EDIM = -3,    /* negative or too large dimension, or leading dimension too small */
    GFQ_ENULL = -4,   /* null pointer where data is needed                               */
    GFQ_EALIGN = -5,  /* packed buffer not 16-byte aligned                              */
    GFQ_EALIAS = -6,  /* output overlaps an input                                        */
    GFQ_ENOMEM = -7,  /* the library could not allocate its workspace                    */
    GFQ_EHIP = -8,    /* a HIP runtime call failed (launch or asynchronous error)        */
    GFQ_EBUDGET = -9, /* request larger than the server's memory budget                  */
    GFQ_EAGAIN = -10  /* server queue full or result not ready yet                       */
};

/* Largest inner dimension l accepted by gfq_matmul (keeps every index in 32 bits). */
#define GFQ_MAX_DIM ((int64_t)1 << 24)

/* Bytes of a packed rows x cols matrix over field q (format above); 0 if q or the
 * dimensions are invalid. */
size_t gfq_packed_bytes(int q, int64_t rows, int64_t cols);

/* Pack (Section 3 bitslicing with the encodings of Section 4).
 * src: device, rows x cols uint8, leading dimension ld_src >= cols.  Values are taken as
 *      integers: for F_p the residue mod p is packed; for GF(4) only bits 0 and 1 are used.
 * dst: device, gfq_packed_bytes(q, rows, cols) bytes, 16-byte aligned; pad bits are zeroed.
 * rows == 0 or cols == 0 is a no-op. */
int gfq_pack(int q, int64_t rows, int64_t cols, const uint8_t *src, int64_t ld_src, void *dst);

/* Unpack: inverse of gfq_pack.  src is a packed rows x cols matrix (any representatives);
 * dst (device, leading dimension ld_dst >= cols) receives canonical values. */
int gfq_unpack(int q, int64_t rows, int64_t cols, const void *src, uint8_t *dst, int64_t ld_dst);

/* C = A B (Section 2: row i of C is the combination of the rows of B with coefficients
 * from row i of A; the Method of Four Russians splits it into k-row slabs and the additive
 * basis {alpha_d} with bit maps phi_d reduces each slab to binary combinations of rows).
 * A: packed m x l, B: packed l x n, C: packed m x n, all device pointers in the format
 * above.  C must not overlap A or B.  l must be below GFQ_MAX_DIM.  m == 0 or n == 0 is a
 * no-op; l == 0 writes a zero C.  Pad bits of A and B are ignored. */
int gfq_matmul(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B, void *C);

/* Explicit launch configuration for gfq_matmul_config (used by the autotuner and the k
 * sweep).
 *   k      slab width, 1..10: each slab of k rows of B gets a table of its 2^k binary row
 *          combinations.  Two tables live in LDS at once; up to k = 7 (F_3, GF(4)) or
 *          k = 6 (F_5, F_7) their rows are 256 bytes wide, larger k narrows the rows and
 *          lets 128-bit LDS reads conflict.
 *   rows   requested rows of C per workgroup: 256, 512, 1024 or 2048 (F_5 and F_7 are
 *          capped by their register use; the library covers what fits)
 *   split  number of slices of the inner dimension computed by separate workgroups and
 *          summed afterwards, 1..64 */
typedef struct { int k; int rows; int split; int reserved; } gfq_config;

/* gfq_matmul with an explicit configuration (used by the autotuner and the k sweep).
 * Returns GFQ_EINVAL for a configuration outside the ranges above. */
int gfq_matmul_config(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B,
                      void *C, const gfq_config *cfg);

/* The configuration gfq_matmul would use for this problem shape (no launch). */
int gfq_choose_config(int q, int64_t m, int64_t l, int64_t n, gfq_config *out);

/* One product of a batch: packed device operands as for gfq_matmul. */
typedef struct {
    int q;
    int64_t m, l, n;
    const void *A;
    const void *B;
    void *C;
} gfq_problem;

/* Run count independent products (fields and shapes may differ) as one launch per
 * (field, tile height) whose workgroups take (product, row tile, column tile) items from a
 * longest-first work list.  problems is a host array.  Each product obeys the gfq_matmul
 * rules; a validation error in any product rejects the whole batch before anything is
 * launched.  Equivalent to gfq_batch_create + gfq_batch_launch; the batch's descriptors are
 * released by a later call or gfq_sync once the launch has finished. */
int gfq_matmul_batched(int count, const gfq_problem *problems);

/* A prepared batch: products, launch parameters and work lists on the device.  Create it
 * once for a set of products whose operand pointers stay valid, launch it any number of
 * times.  gfq_batch_create validates every product (any error rejects the batch), chooses
 * each product's slab width and tile height (from the tuning cache when it holds the
 * product's size class), orders each (field, tile height) list of (product, row tile,
 * column tile) items longest first and uploads the descriptors; it synchronises.
 * gfq_batch_launch enqueues, on the calling thread's stream, one launch per list (a
 * workgroup per item) and allocates nothing, so it may be captured into a graph.
 * gfq_batch_times waits for that stream and writes, per product, the microseconds from the
 * start of the most recent launch to the completion of the product's last tile.
 * gfq_batch_destroy waits for the device and frees everything. */
typedef struct gfq_batch gfq_batch;
int gfq_batch_create(int count, const gfq_problem *problems, gfq_batch **out);
int gfq_batch_launch(gfq_batch *batch);
int gfq_batch_times(gfq_batch *batch, double *completion_us);
int gfq_batch_destroy(gfq_batch *batch);

/* Autotuning.  gfq_tune times candidate configurations on scratch operands of the given
 * shape (pseudo-random contents) on the current device and stores the fastest in a cache
 * keyed by (device architecture, mode, field, size class); it synchronises and returns the
 * chosen configuration.  Modes: 0 = single products (k, tile height and split for this
 * shape's size class, where the class rounds m, l, n up to powers of two from 64 to 16384);
 * GFQ_TUNE_BATCH = products inside batches (k and tile height for the class of (m, l); n is
 * ignored).  gfq_choose_config and gfq_batch_create use cached entries when they exist.
 * gfq_tune_lookup returns GFQ_OK and the entry if the class is cached, GFQ_EAGAIN if not.
 * gfq_tune_save / gfq_tune_load write / merge the cache as text, one entry per line.
 * gfq_tune_clear empties it.
 * gfq_tune: each of m, l, n in 1 .. 65536 (else GFQ_EDIM); q in {3,4,5,7} (GFQ_EFIELD);
 * mode 0 or GFQ_TUNE_BATCH (GFQ_EINVAL).  It runs on the calling thread's stream, waits for
 * its own launches, and keeps its scratch operands (one device buffer, filled with
 * pseudo-random words) until the process ends; GFQ_ENOMEM if that buffer cannot be had.
 * Concurrent calls on one device measure each other: tune from one thread at a time.
 * gfq_tune_load returns GFQ_EINVAL if the file cannot be read or holds a malformed or
 * out-of-range entry (the valid entries are merged all the same). */
#define GFQ_TUNE_BATCH 1
int gfq_tune(int q, int64_t m, int64_t l, int64_t n, int mode, gfq_config *out);
int gfq_tune_lookup(int q, int64_t m, int64_t l, int64_t n, int mode, gfq_config *out);
int gfq_tune_save(const char *path);
int gfq_tune_load(const char *path);
int gfq_tune_clear(void);

/* Stream for subsequent calls made by this host thread (a hipStream_t; NULL = default). */
int gfq_set_stream(void *hip_stream);

/* Wait for the calling thread's stream; asynchronous HIP errors surface here as GFQ_EHIP. */
int gfq_sync(void);

/* Kernel timing for measurement tools (off by default).  While on, every launch of the
 * product kernel and of the partial-sum kernel made by this thread is bracketed by HIP
 * events on the launch stream.  gfq_timing_read waits for the recorded events, returns
 * the summed milliseconds and launch counts of both kernels (any pointer may be NULL) and
 * clears the record. */
int gfq_set_timing(int on);
int gfq_timing_read(double *product_ms, int *product_launches, double *reduce_ms, int *reduce_launches);

/* Static description of a status code. */
const char *gfq_strerror(int status);

/* Most recent HIP error text seen by this thread (empty if none). */
const char *gfq_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GFQ_H */
