/*
 * gfq.h -- C ABI of libgfq: dense matrix products C = A B over F_3, F_5, F_7,
 * GF(4) = F_2[x]/(x^2 + x + 1), GF(8) = F_2[x]/(x^3 + x + 1) and F_9 = F_3[i]/(i^2 + 1) on
 * one AMD Instinct MI355X (gfx950), computed by the
 * Method of Four Russians with an additive basis on bitsliced rows (Boothby and
 * Bradshaw, "Bitslicing and the Method of Four Russians Over Larger Finite Fields":
 * Section 2 for the method, Section 3 for the row-wise bitsliced format, Section 4 for
 * the field encodings).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Field selector q is 3, 5 or 7 for the prime fields, 4 for GF(4), 8 for GF(8) and 9
 *    for F_9.  Any other value returns GFQ_EFIELD.
 *  - Unpacked matrices are uint8, row-major with a leading dimension in elements, holding
 *    canonical representatives: 0..q-1 for F_q; for F_3 the value 2 stands for -1; for
 *    GF(4) the value c0 + 2 c1 stands for c0 + c1 x; for GF(8) the value c0 + 2 c1 + 4 c2
 *    stands for c0 + c1 x + c2 x^2; for F_9 the value a0 + 3 a1 (a0, a1 in 0..2, 2 standing
 *    for -1) stands for a0 + a1 i.
 *  - Packed matrices use the row-wise bitsliced format of Section 3, the same format for
 *    the left operand, the right operand and the product.  A matrix of R rows and N
 *    columns over a field with P bit-planes (P = 2 for F_3 and GF(4), P = 3 for F_5, F_7
 *    and GF(8), P = 4 for F_9)
 *    occupies R * P * W 32-bit words with W = ceil(N / 128) * 4: row r holds plane 0,
 *    then plane 1, ..., each W little-endian words; element j of the row is bit (j mod 32)
 *    of word (j / 32) of each plane.  Element encodings per plane:
 *        F_3 (Section 4.1): plane 0 marks a unit, plane 1 the sign (0 = 00, 1 = 10, -1 = 11)
 *        F_5, F_7 (Section 4.2): plane d is binary digit d of the representative
 *        GF(4), GF(8) (Section 4.3): plane d is the coefficient c_d of x^d
 *        F_9 (Section 4.3 over 4.1): planes 0, 1 are the F_3 code of a0, planes 2, 3 of a1
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
    GFQ_EFIELD = -2,  /* q not in {3, 4, 5, 7, 8, 9}                                    */
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
 *      integers: for F_p the residue mod p is packed; for GF(4) only bits 0 and 1 are used,
 *      for GF(8) bits 0 to 2; for F_9 the residue mod 9.
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
 * no-op; l == 0 writes a zero C.  Pad bits of A and B are ignored.
 * When the configuration splits the inner dimension, the partial products go to a device
 * workspace the library keeps per (device, stream) until the process ends (64 MiB or more;
 * GFQ_ENOMEM if it cannot be had); growing it waits for that stream.  Products on different
 * streams may run concurrently. */
int gfq_matmul(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B, void *C);

/* Explicit launch configuration for gfq_matmul_config (used by the autotuner and the k
 * sweep).
 *   k      slab width, 1..10: each slab of k rows of B gets a table of its 2^k binary row
 *          combinations.  Two tables live in LDS at once; up to k = 7 (F_3, GF(4)) or
 *          k = 6 (F_5, F_7, GF(8), F_9) their rows are 256 bytes wide (a 512-column tile,
 *          conflict-free reads), at the next k 128 bytes (a 1024-column tile, two rows of C
 *          per read pass), beyond that narrower (512 columns and less, reads may conflict).
 *   rows   requested rows of C per workgroup: 256, 512, 1024 or 2048; the library takes the
 *          tallest tile up to the request that the field's registers allow (at most 512
 *          rows on 1024-column tiles, 1024 for F_5, F_3, GF(8) and 2048 for GF(4) on
 *          512-column tiles, 512 for F_7 and F_9)
 *   split  number of slices of the inner dimension computed by separate workgroups and
 *          summed afterwards, 1..64
 *   variant how extension-field products are formed (F_3, F_5, F_7: GFQ_VARIANT_ROWWISE
 *          only):
 *          GFQ_VARIANT_ROWWISE  row-wise additive basis (Section 2 with the encodings of
 *                               4.3): GF(4) {1, x}, GF(8) {1, x, x^2}, F_9 {1, -1, i, -i};
 *          GFQ_VARIANT_KARATSUBA matrix-level products over the prime subfield (Section 4.3),
 *                               one plane-table per subfield product:
 *                               GF(4): three F_2 products, C0 = A0 B0 + A1 B1,
 *                                 C1 = (A0 + A1)(B0 + B1) + A0 B0;
 *                               GF(8): six F_2 products by the trinomial formula,
 *                                 P_ii = Ai Bi, P_ij = (Ai + Aj)(Bi + Bj), reduced by
 *                                 x^3 + x + 1: C0 = P00 + P11 + P12 + P22,
 *                                 C1 = P00 + P01 + P12, C2 = P00 + P02 + P11;
 *                               F_9: three F_3 products, C0 = A0 B0 - A1 B1,
 *                                 C1 = (A0 + A1)(B0 + B1) - A0 B0 - A1 B1.
 *          Both give the same packed product; batches use the row-wise form.  The GF(8) and
 *          F_9 matrix routes hold six planes per table entry and take k <= 9. */
#define GFQ_VARIANT_ROWWISE 0
#define GFQ_VARIANT_KARATSUBA 1
typedef struct { int k; int rows; int split; int variant; } gfq_config;

/* gfq_matmul with an explicit configuration (used by the autotuner and the k sweep).
 * Returns GFQ_EINVAL for a configuration outside the ranges above. */
int gfq_matmul_config(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B,
                      void *C, const gfq_config *cfg);

/* gfq_matmul_config for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Where the inner dimension
 * is split, the slices' partial products go to a fixed device array of the library
 * (GFQ_NOALLOC_SCRATCH_BYTES on each device, held from the library's loading until the
 * process ends) instead of the workspace gfq_matmul allocates; the call makes no device
 * allocation and times no launch (gfq_set_timing does not apply).
 * cfg NULL: the configuration gfq_matmul would choose, its split lowered until the partial
 * products (split * gfq_packed_bytes(q, m, n) bytes) fit the array.  An explicit cfg whose
 * partial products do not fit returns GFQ_EBUDGET; one that does not split (split = 1, or
 * l at most k) does not use the array.
 * Every call on a device shares that device's array, which keeps what the last call left in
 * it: calls that overlap in time on one device (different streams or threads) race on it,
 * so issue them on one stream or wait between them.  Nothing in it needs clearing: each
 * partial product is written in full before it is summed.  The first call on a device looks
 * up the array's address on that device (GFQ_EHIP if the lookup fails).
 * Other arguments and return codes as for gfq_matmul_config. */
#define GFQ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int gfq_matmul_noalloc(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B,
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

/* C = A B by Strassen-Winograd recursion with the Four-Russians product as its base case
 * (the paper applies asymptotically faster algorithms above the Four-Russians method for
 * large matrices, Section 2 and Section 5).  Each level splits A, B and C into quadrants
 * and forms C from seven half-size products instead of eight, in Winograd's form:
 *   S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21, S4 = A12 - S2,
 *   T1 = B12 - B11, T2 = B22 - T1, T3 = B22 - B12, T4 = T2 - B21,
 *   P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4, P5 = S1 T1, P6 = S2 T2, P7 = S3 T3,
 *   C11 = P1 + P2, C12 = P1 + P6 + P5 + P3, C21 = P1 + P6 + P7 - P4, C22 = P1 + P6 + P7 + P5.
 * Rows split at ceil(d / 2) and columns (and the inner dimension) at ceil(d / 2) rounded up
 * to a multiple of 32; the missing rows and columns of the second halves are zero.  The
 * arithmetic is exact, so C is the same packed product as gfq_matmul's, byte for byte.
 * levels  0..GFQ_SW_MAX_LEVELS; 0 is gfq_matmul_config(..., leaf).  All 7^levels leaf
 *         products run in one launch of the product kernel.  GFQ_SW_AUTO takes the number
 *         of levels the tuner cached for the product's size class (gfq_tune with
 *         GFQ_TUNE_SW), 0 when there is none.
 * leaf    configuration of the leaf products (NULL: the slab width and route chosen for
 *         one leaf, the tile height and inner-dimension slices fitted to all leaves together);
 *         with more than one slice, the leaves' partial products are summed by one launch.
 * A, B, C and the return codes as for gfq_matmul.  The operand sums and the products of
 * every level live in the per-(device, stream) workspace (about (7/4)^levels times the
 * packed sizes of A, B and C together, summed over the levels). */
#define GFQ_SW_MAX_LEVELS 4
#define GFQ_SW_AUTO (-1)
int gfq_matmul_sw(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B, void *C, int levels,
                  const gfq_config *leaf);

/* Run count independent products (fields and shapes may differ) as one launch per
 * (field, tile shape) whose persistent workgroups take (product, row tile, column tile,
 * slab slice) items from a longest-first list through a device queue head (the method of
 * Section 2 per item), plus one partial-sum launch when products are sliced.  problems is a
 * host array.  Each product obeys the gfq_matmul
 * rules; a validation error in any product rejects the whole batch before anything is
 * launched.  Equivalent to gfq_batch_create + gfq_batch_launch_persistent (the faster drain
 * on mixed batches); the batch's descriptors are released by a later call or gfq_sync once
 * the launch has finished. */
int gfq_matmul_batched(int count, const gfq_problem *problems);

/* A prepared batch: products, launch parameters and work lists on the device.  Create it
 * once for a set of products whose operand pointers stay valid, launch it any number of
 * times.  gfq_batch_create validates every product (any error rejects the batch), chooses
 * each product's slab width and tile height (from the tuning cache when it holds the
 * product's size class; a product taller than 256 rows and at most 256 columns wide gets
 * one column of narrow tiles), cuts the inner dimension of a product into slab slices
 * (at least 8 slabs each, at most 64 slices and 256 MiB of partial products) when each of
 * its tiles would take more than half of a compute unit's share of the whole batch (few
 * tiles and a long inner dimension), orders each (field, tile shape) list of (product, row
 * tile, column tile, slice) items longest first, allocates the descriptors and the sliced
 * products' partial products in one device allocation and uploads the descriptors; it
 * synchronises.
 * gfq_batch_launch enqueues one launch per list (a workgroup per item): the first on the
 * calling thread's stream, the others on side streams of the library (default priority,
 * kept per calling stream until the process ends) that fork from and join back into the
 * calling stream, so the lists overlap.  It allocates nothing, so it may be captured into a
 * graph (the lists become parallel branches); side streams are never created during a
 * capture: if the capturing stream has none yet, the lists are captured one after another
 * (one uncaptured launch on that stream first creates them).  When products are sliced, a
 * partial-sum launch on the calling stream follows the joined lists and writes their C.
 * Launches
 * of one batch must not overlap in time (they share its tile counters, completion stamps
 * and outputs): issue them on one stream, or wait for one before issuing the next.
 * gfq_batch_times waits for that stream and writes, per product, the microseconds from the
 * start of the most recent launch to the completion of the product (its last tile, or the
 * last of its partial sums).
 * gfq_batch_destroy waits for the device and frees everything. */
typedef struct gfq_batch gfq_batch;
int gfq_batch_create(int count, const gfq_problem *problems, gfq_batch **out);
int gfq_batch_launch(gfq_batch *batch);
/* The same batch drained by persistent workgroups: per list, a reset of its queue head, then
 * as many workgroups as the device holds at once (at most one per item), each taking the
 * next item index from the head with an atomic add, publishing it to its threads through
 * workgroup memory between two barriers, and leaving when the index passes the end (Section
 * 2's items, same results as gfq_batch_launch byte for byte).  Streams, side streams,
 * capture, partial sums, completion stamps and the no-overlap rule as for gfq_batch_launch;
 * it allocates nothing.  GFQ_EINVAL if the batch has more than 64 lists. */
int gfq_batch_launch_persistent(gfq_batch *batch);
int gfq_batch_times(gfq_batch *batch, double *completion_us);
/* The slab width k the batch gives each product (host array of count ints; the work the
 * method does per product, Section 2, depends on it). */
int gfq_batch_slab_widths(const gfq_batch *batch, int *k);
/* The number of slab slices the batch cut each product into (host array of count ints; 1:
 * whole tiles). */
int gfq_batch_slices(const gfq_batch *batch, int *slices);
int gfq_batch_destroy(gfq_batch *batch);

/* Autotuning.  gfq_tune times candidate configurations on scratch operands of the given
 * shape (pseudo-random contents) on the current device and stores the fastest in a cache
 * keyed by (device architecture, mode, field, size class); it synchronises and returns the
 * chosen configuration.  Modes: 0 = single products (k, tile height and split for this
 * shape's size class, where the class rounds m, l, n up to powers of two from 64 to 16384);
 * GFQ_TUNE_BATCH = products inside batches (k and tile height for the class of (m, l); n is
 * ignored); GFQ_TUNE_SW = the number of Strassen-Winograd levels, 0 .. GFQ_SW_MAX_LEVELS - 1,
 * for gfq_matmul_sw with GFQ_SW_AUTO (timed with the default leaf choice; the entry holds
 * the levels in its k field, the other fields 0; more levels are chosen only when 2% faster
 * than the fastest with fewer).  gfq_choose_config, gfq_batch_create and gfq_matmul_sw (GFQ_SW_AUTO) use cached
 * entries when they exist.
 * gfq_tune_lookup returns GFQ_OK and the entry if the class is cached, GFQ_EAGAIN if not; a
 * single-product entry keeps the shape it was timed on, and a product of the class with
 * fewer tiles than that shape (so fewer workgroups at the cached split) gets the cached k and
 * tile height with the split chosen again for its own shape by the library's cost model
 * (never fewer slices than cached).
 * gfq_tune_save / gfq_tune_load write / merge the cache as text, one entry per line:
 * "arch mode q m_class l_class n_class k rows split variant", and for mode 0 the rows and
 * columns of the shape timed (absent: the class's largest, 2^m_class x 2^n_class).
 * gfq_tune_clear empties it.
 * gfq_tune: each of m, l, n in 1 .. 65536 (else GFQ_EDIM); q in {3,4,5,7,8,9} (GFQ_EFIELD);
 * mode 0, GFQ_TUNE_BATCH or GFQ_TUNE_SW (GFQ_EINVAL).  It runs on the calling thread's stream, waits for
 * its own launches, and keeps its scratch operands (one device buffer, filled with
 * pseudo-random words) until the process ends; GFQ_ENOMEM if that buffer cannot be had.
 * Concurrent calls on one device measure each other: tune from one thread at a time.
 * gfq_tune_load returns GFQ_EINVAL if the file cannot be read or holds a malformed or
 * out-of-range entry (the valid entries are merged all the same). */
#define GFQ_TUNE_BATCH 1
#define GFQ_TUNE_SW 2
int gfq_tune(int q, int64_t m, int64_t l, int64_t n, int mode, gfq_config *out);
int gfq_tune_lookup(int q, int64_t m, int64_t l, int64_t n, int mode, gfq_config *out);
int gfq_tune_save(const char *path);
int gfq_tune_load(const char *path);
int gfq_tune_clear(void);

/* Product server: continuous batching of products as they arrive (the batched products
 * above, fed by a request queue).  A server owns a worker thread, its own HIP streams (one
 * per in-flight batch, default priority), an arena of device memory for packed operands
 * bounded by a byte budget, and per-slot descriptor buffers; it runs on the device that is
 * current when it is created.
 *
 * Each request is one product C = A B over field q with A m x l, B l x n.  Operands are
 * device pointers owned by the caller and must stay valid, and C untouched by others, until
 * the request's completion has been returned by gfq_server_poll.  By default A and B are
 * uint8 matrices (canonical values, leading dimensions lda >= l, ldb >= n) and C receives a
 * uint8 matrix (ldc >= n); the flags GFQ_REQ_A_PACKED, GFQ_REQ_B_PACKED, GFQ_REQ_C_PACKED
 * mark an operand as already packed (format above, 16-byte aligned; its ld is ignored), so
 * operands kept packed in device memory are used in place.  Every packed operand the server
 * makes (the packed forms of uint8 A and B, and the packed product before it is unpacked) is
 * held in the arena from admission to completion.
 *
 * The worker admits requests in order of arrival (not_before_us, or the submission time
 * when that is earlier or 0) while the arena has room for a request's packed operands and a
 * batch has room (max_batch requests, max_items tiles); the first request that does not
 * fit waits for memory released by completing batches, so no request is overtaken.  An
 * admitted batch is launched at once on a free slot's stream: one conversion launch packs
 * every uint8 operand, one work-list launch per (field, tile height) computes the
 * products, one conversion launch unpacks every uint8 product.  Batches on different slots
 * overlap on the device; requests that arrive meanwhile form the next batch as soon as a
 * slot is free.  In GFQ_SERVE_SERIAL mode the server instead runs one request at a time
 * with the single-product calls (gfq_pack, gfq_matmul, gfq_unpack) - the baseline of
 * plain launches, measured by the same clocks.
 *
 * Times are microseconds of the server clock (gfq_server_now_us, monotonic, 0 at creation).
 */
typedef struct gfq_server gfq_server;

#define GFQ_SERVE_BATCHED 0
#define GFQ_SERVE_SERIAL 1

typedef struct {
    size_t budget_bytes; /* arena limit for packed operands (0 = 1 GiB)                     */
    int slots;           /* batches in flight, 1..8 (0 = 3; serial mode uses 1)             */
    int max_batch;       /* requests per batch, 1..4096 (0 = 256; serial mode uses 1)       */
    int max_items;       /* tiles per batch, 32768..1048576 (0 = 65536)                     */
    int mode;            /* GFQ_SERVE_BATCHED or GFQ_SERVE_SERIAL                           */
    double watchdog_s;   /* a batch not complete this many seconds after its launch fails:   *
                          * its requests complete with GFQ_EHIP, its slot and arena ranges   *
                          * are never reused, the server is marked failed (0 = no watchdog) */
} gfq_server_opts;

#define GFQ_REQ_A_PACKED 1
#define GFQ_REQ_B_PACKED 2
#define GFQ_REQ_C_PACKED 4

typedef struct {
    int q;
    int64_t m, l, n;        /* each in 0 .. 65535 (m == 0, n == 0 or l == 0 are allowed)  */
    const void *A;
    int64_t lda;
    const void *B;
    int64_t ldb;
    void *C;
    int64_t ldc;
    int flags;              /* GFQ_REQ_* bits                                             */
    uint64_t tag;           /* returned with the completion                               */
    double not_before_us;   /* arrival time on the server clock; 0 = at submission        */
    void *C_host;           /* NULL, or host memory (pinned for speed) that receives a copy  *
                             * of the product before the completion is reported: the span of *
                             * C, (m - 1) ldc + n bytes (packed: gfq_packed_bytes)            */
} gfq_request;

typedef struct {
    uint64_t tag;
    int status;             /* GFQ_OK, or GFQ_EHIP if the device work failed              */
    int batch_size;         /* requests in the batch that carried this one                */
    double arrival_us;      /* max(submission, not_before_us)                             */
    double launch_us;       /* batch launched                                             */
    double done_us;         /* completion observed by the worker                          */
} gfq_completion;

typedef struct {
    int64_t submitted, completed, batches;
    int64_t queued;              /* submitted, not yet admitted                             */
    int64_t max_batch_seen;
    size_t arena_in_use, arena_held, arena_peak_in_use;
} gfq_server_stats;

/* Create a server (opts may be NULL for defaults).  GFQ_EINVAL for options out of range,
 * GFQ_ENOMEM / GFQ_EHIP if its streams or descriptor buffers cannot be had. */
int gfq_server_create(const gfq_server_opts *opts, gfq_server **out);
/* Queue count requests (host array, copied).  All are validated first (field, dimensions,
 * null or misaligned pointers, leading dimensions, C overlapping A or B); the first error
 * rejects them all.  GFQ_EBUDGET if a request's packed operands alone exceed the budget;
 * GFQ_EHIP if the server has failed.  Returns without waiting. */
int gfq_server_submit(gfq_server *srv, const gfq_request *reqs, int count);
/* Move up to max completions into out (*got of them), waiting up to timeout_us for the
 * first (0 = do not wait, negative = wait indefinitely).  GFQ_OK even when *got is 0. */
int gfq_server_poll(gfq_server *srv, gfq_completion *out, int max, int *got, double timeout_us);
double gfq_server_now_us(const gfq_server *srv);
int gfq_server_stats_read(const gfq_server *srv, gfq_server_stats *out);
/* Wait for the batches in flight, drop requests not yet admitted (their completions are
 * never reported), stop the worker and free everything. */
int gfq_server_destroy(gfq_server *srv);

/* Stream for subsequent calls made by this host thread (a hipStream_t; NULL = default). */
int gfq_set_stream(void *hip_stream);

/* Wait for the calling thread's stream; asynchronous HIP errors surface here as GFQ_EHIP. */
int gfq_sync(void);

/* Kernel timing for measurement tools (off by default).  While on, every launch of the
 * product kernel and of the elementwise kernels around it (partial sums of split products,
 * the splits and merges of gfq_matmul_sw) made by this thread is bracketed by HIP events
 * on the launch stream.  gfq_timing_read waits for the recorded events, returns the summed
 * milliseconds and launch counts of the product kernel and of the elementwise kernels
 * (reduce_*; any pointer may be NULL) and clears the record. */
int gfq_set_timing(int on);
int gfq_timing_read(double *product_ms, int *product_launches, double *reduce_ms, int *reduce_launches);

/* Static description of a status code. */
const char *gfq_strerror(int status);

/* Most recent HIP error text seen by this thread (empty if none). */
const char *gfq_last_hip_error(void);

/* Measurement helpers (no part of the paper's method): the machine rates that the product
 * kernels' roofline fractions are quoted against, each run once and timed with HIP events on
 * the calling thread's stream (the call waits for it).
 * gfq_probe_valu: blocks workgroups of 512 lanes, each lane iters x 17 dependent-free
 *   v_bitop3_b32 instructions (the product's only arithmetic); *lane_ops = total lane
 *   operations.  sink: device scratch of blocks x 512 words (written only by a value no
 *   run produces).
 * gfq_probe_lds: blocks workgroups of 512 lanes reading 128-bit LDS words, every 16-lane group
 *   one 256-byte row per read (the access shape of the product's gathers), iters x 16 reads
 *   per lane; *bytes = total bytes read.  sink as above.
 * gfq_probe_copy: copies bytes (a multiple of 16, 16-byte aligned device buffers) in 128-bit
 *   words; HBM traffic is 2 x bytes.
 * Return GFQ_EINVAL for bad arguments, GFQ_EHIP for a failed launch. */
int gfq_probe_valu(int blocks, int iters, uint32_t *sink, double *lane_ops, float *ms);
int gfq_probe_lds(int blocks, int iters, uint32_t *sink, double *bytes, float *ms);
int gfq_probe_copy(const void *src, void *dst, size_t bytes, float *ms);

#ifdef __cplusplus
}
#endif

#endif /* GFQ_H */
