// gfq_internal.h -- declarations shared by the C-ABI layer and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gfq {

typedef uint32_t u32;

constexpr int KMAX = 10;   // largest slab width
constexpr int GMAX = 4;    // longest Gray walk kept in registers during the table build

constexpr int log2_floor(int x) { return x <= 1 ? 0 : 1 + log2_floor(x / 2); }

// LDS table layouts: tile width in 32-bit words (per plane) and copies per super-row.
enum Layout { LAYOUT_W32_R2 = 0, LAYOUT_W32_R1 = 1, LAYOUT_W16_R1 = 2, LAYOUT_W8_R1 = 3 };
inline int layout_twd(int lay) { return lay <= LAYOUT_W32_R1 ? 32 : (lay == LAYOUT_W16_R1 ? 16 : 8); }
inline int layout_srb(int lay) { return lay == LAYOUT_W32_R2 ? 256 : layout_twd(lay) * 4; }

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
    int canon;             // 1: write canonical C; 0: write a raw partial product
};

inline int planes_of(int q) { return (q == 3 || q == 4) ? 2 : 3; }
inline int words_of(int64_t cols) { return (int)(((cols + 127) / 128) * 4); }

hipError_t launch_matmul(int q, const MMArgs &a, int layout, int rowsTile, hipStream_t st);
hipError_t launch_reduce(int q, const u32 *part, u32 *C, int m, int n, int Wn, int splits, size_t stride, hipStream_t st);
hipError_t launch_pack(int q, const uint8_t *src, int64_t ld, u32 *dst, int rows, int cols, int W, hipStream_t st);
hipError_t launch_unpack(int q, const u32 *src, uint8_t *dst, int64_t ld, int rows, int cols, int W, hipStream_t st);
int rows_tile_of(int layout, int rowsTile);   // rows of C one workgroup really covers

}  // namespace gfq
