// gfq_kernels.hip -- HIP kernels for gfx950: pack, unpack, the Four-Russians product and
// the reduction of split-l partial products.
//
// Method (paper, Section 2): row i of C is sum_j a_ij B_j.  The inner dimension is cut
// into slabs of k rows of B; for each slab a table of all 2^k binary combinations of its
// rows is built once and shared by every row of C.  With an additive basis {alpha_d} and
// bit maps phi_d (a = sum_d alpha_d phi_d(a)), the slab's contribution to row i is
// sum_d alpha_d T[phi_d(a_i, slab)], so only binary combinations are ever tabulated.
//
// Work decomposition on the GPU
//   grid.x  column tile: TWD 32-bit words of every plane (32*TWD columns of C)
//   grid.y  row tile: TM rows of C
//   grid.z  slice of the slabs ("split-l"); slices > 1 write partial products that
//           gfq_reduce_partials sums.
// Per workgroup and slab: stage the slab's k rows of B and the phi_d indices of the tile's
// rows into LDS, build the table in LDS (Gray-code order), then every lane gathers table
// rows and accumulates alpha_d-scaled rows into registers with bitwise VALU operations.
//
// LDS table layout.  A table row (one entry, one plane) is a "super-row" of SRB bytes
// holding REP copies of the TWD-word tile row.  gfx950 serves a 128-bit LDS read of 16
// lanes from 64 four-byte banks in one pass, so a 16-lane group is conflict-free exactly
// when it reads 256 distinct consecutive bytes.  With SRB = 256 the lanes of one 16-lane
// group that gather different rows of C read different copies and never conflict.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GFQ_HD __host__ __device__ __forceinline__
#include "gfq_field.h"
#include "gfq_internal.h"

namespace gfq {

// ---------------------------------------------------------------------------------------
// Field traits used by the kernels.  Values travel as P planes of 4 words (one 128-bit
// load per plane); V is that bundle.
// ---------------------------------------------------------------------------------------
template <int P> struct Vec { uint4 p[P]; };

__device__ __forceinline__ u32 comp(const uint4 &v, int i) {
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}
__device__ __forceinline__ void setc(uint4 &v, int i, u32 x) {
    if (i == 0) v.x = x; else if (i == 1) v.y = x; else if (i == 2) v.z = x; else v.w = x;
}

template <int Q> struct FT;

// F_3: storage planes (unit, sign); basis {1, -1} with phi_0 = [a = 1] = x0 ^ x1 and
// phi_1 = [a = -1] = x1 (Section 4.1).  Accumulation: acc + T[phi_0] - T[phi_1].
template <> struct FT<3> {
    static constexpr int P = 2, D = 2, PA = 2;   // PA: accumulator planes
    typedef Vec<2> V;
    typedef Vec<2> Acc;
    __device__ static void phis(const u32 *x, u32 *f) { f[0] = x[0] ^ x[1]; f[1] = x[1]; }
    __device__ static V add(const V &a, const V &b) {
        V r;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            F3v x = {comp(a.p[0], i), comp(a.p[1], i)}, y = {comp(b.p[0], i), comp(b.p[1], i)};
            F3v z = f3_add(x, y);
            setc(r.p[0], i, z.u); setc(r.p[1], i, z.s);
        }
        return r;
    }
    __device__ static V sub(const V &a, const V &b) {
        V r;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            F3v x = {comp(a.p[0], i), comp(a.p[1], i)}, y = {comp(b.p[0], i), comp(b.p[1], i)};
            F3v z = f3_sub(x, y);
            setc(r.p[0], i, z.u); setc(r.p[1], i, z.s);
        }
        return r;
    }
    __device__ static V neg_row(const V &b) { return b; }   // unused: F_3 subtracts directly
    __device__ static Acc acc_zero() { Acc a; a.p[0] = a.p[1] = make_uint4(0, 0, 0, 0); return a; }
    __device__ static void accumulate(Acc &acc, const V *t) { acc = sub(add(acc, t[0]), t[1]); }
    __device__ static V finish(const Acc &a) { return a; }
    __device__ static V canon(const V &a) { return a; }
};

// F_7: binary digits, basis {1, 2, 4}; doubling is a plane rotation (Section 4.2).
template <> struct FT<7> {
    static constexpr int P = 3, D = 3, PA = 3;
    typedef Vec<3> V;
    typedef Vec<3> Acc;
    __device__ static void phis(const u32 *x, u32 *f) { f[0] = x[0]; f[1] = x[1]; f[2] = x[2]; }
    template <typename F> __device__ static V map2(const V &a, const V &b, F f) {
        V r;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            P3v x = {comp(a.p[0], i), comp(a.p[1], i), comp(a.p[2], i)};
            P3v y = {comp(b.p[0], i), comp(b.p[1], i), comp(b.p[2], i)};
            P3v z = f(x, y);
            setc(r.p[0], i, z.b0); setc(r.p[1], i, z.b1); setc(r.p[2], i, z.b2);
        }
        return r;
    }
    __device__ static V add(const V &a, const V &b) { return map2(a, b, [](P3v x, P3v y) { return f7_add(x, y); }); }
    __device__ static V neg_row(const V &b) {
        V r;
#pragma unroll
        for (int p = 0; p < 3; p++) r.p[p] = make_uint4(~b.p[p].x, ~b.p[p].y, ~b.p[p].z, ~b.p[p].w);
        return r;
    }
    __device__ static V sub(const V &a, const V &b) { return add(a, neg_row(b)); }
    __device__ static V dbl(const V &a) { V r; r.p[0] = a.p[2]; r.p[1] = a.p[0]; r.p[2] = a.p[1]; return r; }
    __device__ static Acc acc_zero() { Acc a; a.p[0] = a.p[1] = a.p[2] = make_uint4(0, 0, 0, 0); return a; }
    __device__ static void accumulate(Acc &acc, const V *t) {
        acc = add(acc, t[0]);
        acc = add(acc, dbl(t[1]));
        acc = add(acc, dbl(dbl(t[2])));
    }
    __device__ static V finish(const Acc &a) { return a; }
    __device__ static V canon(const V &a) {
        V r;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            P3v x = {comp(a.p[0], i), comp(a.p[1], i), comp(a.p[2], i)};
            P3v z = f7_reduce(x);
            setc(r.p[0], i, z.b0); setc(r.p[1], i, z.b1); setc(r.p[2], i, z.b2);
        }
        return r;
    }
};

// F_5: binary digits, basis {1, 2, 4} = {1, 2, -1}; add = 4-bit sum then fold5 (Section 4.2).
template <> struct FT<5> {
    static constexpr int P = 3, D = 3, PA = 3;
    typedef Vec<3> V;
    typedef Vec<3> Acc;
    __device__ static void phis(const u32 *x, u32 *f) { f[0] = x[0]; f[1] = x[1]; f[2] = x[2]; }
    template <typename F> __device__ static V map1(const V &a, F f) {
        V r;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            P3v x = {comp(a.p[0], i), comp(a.p[1], i), comp(a.p[2], i)};
            P3v z = f(x);
            setc(r.p[0], i, z.b0); setc(r.p[1], i, z.b1); setc(r.p[2], i, z.b2);
        }
        return r;
    }
    __device__ static V add(const V &a, const V &b) {
        V r;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            P3v x = {comp(a.p[0], i), comp(a.p[1], i), comp(a.p[2], i)};
            P3v y = {comp(b.p[0], i), comp(b.p[1], i), comp(b.p[2], i)};
            P3v z = f5_add(x, y);
            setc(r.p[0], i, z.b0); setc(r.p[1], i, z.b1); setc(r.p[2], i, z.b2);
        }
        return r;
    }
    __device__ static V neg_row(const V &b) { return map1(b, [](P3v x) { return f5_neg(x); }); }
    __device__ static V sub(const V &a, const V &b) { return add(a, neg_row(b)); }
    __device__ static Acc acc_zero() { Acc a; a.p[0] = a.p[1] = a.p[2] = make_uint4(0, 0, 0, 0); return a; }
    __device__ static void accumulate(Acc &acc, const V *t) {
        acc = add(acc, t[0]);
        acc = add(acc, map1(t[1], [](P3v x) { return f5_dbl(x); }));
        acc = add(acc, neg_row(t[2]));          // 4 = -1 mod 5
    }
    __device__ static V finish(const Acc &a) { return a; }
    __device__ static V canon(const V &a) { return map1(a, [](P3v x) { return f5_reduce(x); }); }
};

// GF(4): planes (c0, c1), basis {1, x}, phi_d = c_d.  Two XOR accumulators, combined as
// acc_0 + x * acc_1 at the end (Section 4.3).
template <> struct FT<4> {
    static constexpr int P = 2, D = 2, PA = 4;
    typedef Vec<2> V;
    typedef Vec<4> Acc;
    __device__ static void phis(const u32 *x, u32 *f) { f[0] = x[0]; f[1] = x[1]; }
    __device__ static uint4 x4(const uint4 &a, const uint4 &b) {
        return make_uint4(a.x ^ b.x, a.y ^ b.y, a.z ^ b.z, a.w ^ b.w);
    }
    __device__ static V add(const V &a, const V &b) { V r; r.p[0] = x4(a.p[0], b.p[0]); r.p[1] = x4(a.p[1], b.p[1]); return r; }
    __device__ static V sub(const V &a, const V &b) { return add(a, b); }
    __device__ static V neg_row(const V &b) { return b; }
    __device__ static Acc acc_zero() { Acc a; for (int p = 0; p < 4; p++) a.p[p] = make_uint4(0, 0, 0, 0); return a; }
    __device__ static void accumulate(Acc &acc, const V *t) {
        acc.p[0] = x4(acc.p[0], t[0].p[0]); acc.p[1] = x4(acc.p[1], t[0].p[1]);
        acc.p[2] = x4(acc.p[2], t[1].p[0]); acc.p[3] = x4(acc.p[3], t[1].p[1]);
    }
    __device__ static V finish(const Acc &a) {
        // acc_0 + x * acc_1 with x (b0 + b1 x) = b1 + (b0 + b1) x
        V r;
        r.p[0] = x4(a.p[0], a.p[3]);
        r.p[1] = x4(x4(a.p[1], a.p[2]), a.p[3]);
        return r;
    }
    __device__ static V canon(const V &a) { return a; }
};

template <int P> __device__ __forceinline__ Vec<P> vzero() {
    Vec<P> v;
#pragma unroll
    for (int p = 0; p < P; p++) v.p[p] = make_uint4(0, 0, 0, 0);
    return v;
}

// Mask for the 4 words starting at word w0 of a row with n valid columns.
__device__ __forceinline__ uint4 colmask(int w0, int n) {
    u32 m[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        int c = (w0 + i) * 32;
        int v = n - c;
        m[i] = v >= 32 ? 0xffffffffu : (v <= 0 ? 0u : ((1u << v) - 1u));
    }
    return make_uint4(m[0], m[1], m[2], m[3]);
}
__device__ __forceinline__ uint4 and4(const uint4 &a, const uint4 &b) {
    return make_uint4(a.x & b.x, a.y & b.y, a.z & b.z, a.w & b.w);
}

// ---------------------------------------------------------------------------------------
// The Four-Russians product kernel.
// ---------------------------------------------------------------------------------------
template <int Q, int TWD, int REP, int R, int NT>
__global__ __launch_bounds__(NT) void m4rm_kernel(MMArgs a) {
    typedef FT<Q> F;
    constexpr int P = F::P, D = F::D;
    constexpr int LPR = TWD / 4;                 // lanes per row of C (4 words each)
    constexpr int SRB = REP * TWD * 4;           // bytes per (entry, plane) super-row
    constexpr int RS = NT / LPR;                 // rows of C per pass of the workgroup
    constexpr int TM = RS * R;                   // rows of C per workgroup
    constexpr int CG = TWD / 4;                  // 4-word column groups per tile
    constexpr int NCHUNK = KMAX * P * CG;        // staging chunks of one slab of B
    static_assert(NCHUNK <= NT, "one staging chunk per thread");
    static_assert(REP * LPR <= 16, "super-row wider than a 16-lane read group");

    extern __shared__ __align__(16) unsigned char smem[];
    const int k = a.k;
    const int E = 1 << k;
    unsigned char *T = smem;
    u32 *Bst = reinterpret_cast<u32 *>(smem + (size_t)E * P * SRB);       // [2][KMAX][P][TWD]
    u32 *Ibuf = Bst + 2 * KMAX * P * TWD;                                  // [2][TM][4]

    const int tid = threadIdx.x;
    const int colw0 = blockIdx.x * TWD;          // first word column of this tile
    const int row0 = blockIdx.y * TM;
    const int s_begin = blockIdx.z * a.slabs_per_split;
    const int s_end = min(a.S, s_begin + a.slabs_per_split);
    const u32 kmask = (1u << k) - 1u;

    // Build split: entries = (high part h, low part) with G low bits walked in Gray order.
    constexpr int HB = log2_floor(NT / CG);      // high bits: one phase-2 task per thread
    static_assert(KMAX - HB <= GMAX, "Gray walk longer than the rows kept in registers");
    const int G = k > HB ? k - HB : 0;
    const int NH = 1 << (k - G);                 // number of high parts

    // --- staging roles -----------------------------------------------------------------
    // B chunk: (t, p, c): row t of the slab, plane p, column group c.
    const int bt = tid / (P * CG), bp = (tid / CG) % P, bc = tid % CG;
    const bool b_active = tid < k * P * CG;
    const int bcol = colw0 + bc * 4;
    // A: rows r = tid, tid + NT, ... of the tile; P planes x (lo, hi) words each.
    constexpr int ARPT = (TM + NT - 1) / NT;     // tile rows staged per thread

    uint4 bpre = make_uint4(0, 0, 0, 0);
    u32 apre[ARPT][P][2];

    auto prefetch = [&](int s) {
        if (b_active) {
            const int brow = s * k + bt;
            if (brow < a.l && bcol < a.Wn) {
                bpre = *reinterpret_cast<const uint4 *>(a.B + ((size_t)brow * P + bp) * a.Wn + bcol);
            } else {
                bpre = make_uint4(0, 0, 0, 0);
            }
        }
        const int bit0 = s * k;
        const int w0 = bit0 >> 5;
        const bool need_hi = (bit0 & 31) + k > 32;
#pragma unroll
        for (int j = 0; j < ARPT; j++) {
            const int lr = tid + j * NT;
            const int row = row0 + lr;
            const bool ok = lr < TM && row < a.m;
#pragma unroll
            for (int p = 0; p < P; p++) {
                const u32 *arow = a.A + ((size_t)row * P + p) * a.Wl;
                apre[j][p][0] = ok ? arow[w0] : 0u;
                apre[j][p][1] = (ok && need_hi && w0 + 1 < a.Wl) ? arow[w0 + 1] : 0u;
            }
        }
    };

    typename F::Acc acc[R];
#pragma unroll
    for (int r = 0; r < R; r++) acc[r] = F::acc_zero();

    const int rs = tid / LPR;                    // row slot
    const int cg = tid % LPR;                    // column group of this lane
    const u32 laneoff = (u32)(tid % (REP * LPR)) * 16u;

    if (s_begin < s_end) prefetch(s_begin);

    for (int s = s_begin; s < s_end; s++) {
        const int buf = s & 1;
        u32 *Bs = Bst + buf * KMAX * P * TWD;
        u32 *Ib = Ibuf + buf * TM * 4;
        // (a) stage this slab: B chunk and phi_d indices (pre-multiplied LDS offsets)
        if (b_active) *reinterpret_cast<uint4 *>(Bs + (bt * P + bp) * TWD + bc * 4) = bpre;
        {
            const int sh = (s * k) & 31;
#pragma unroll
            for (int j = 0; j < ARPT; j++) {
                const int lr = tid + j * NT;
                if (lr < TM) {
                    u32 x[P], f[D];
#pragma unroll
                    for (int p = 0; p < P; p++)
                        x[p] = __builtin_amdgcn_alignbit(apre[j][p][1], apre[j][p][0], sh) & kmask;
                    F::phis(x, f);
                    uint4 o;
                    o.x = f[0] * (u32)(P * SRB);
                    o.y = D > 1 ? f[1] * (u32)(P * SRB) : 0u;
                    o.z = D > 2 ? f[D > 2 ? 2 : 0] * (u32)(P * SRB) : 0u;
                    o.w = 0u;
                    *reinterpret_cast<uint4 *>(Ib + lr * 4) = o;
                }
            }
        }
        // (b) prefetch the next slab while this one is processed
        if (s + 1 < s_end) prefetch(s + 1);
        __syncthreads();

        // (c) build phase 1: entries h << G, direct sums of rows G..k-1
        for (int task = tid; task < CG * NH; task += NT) {
            const int c = task % CG, h = task / CG;
            typename F::V v = vzero<P>();
            bool first = true;
            for (int t = 0; t < k - G; t++) {
                if ((h >> t) & 1) {
                    typename F::V b;
#pragma unroll
                    for (int p = 0; p < P; p++)
                        b.p[p] = *reinterpret_cast<const uint4 *>(Bs + ((G + t) * P + p) * TWD + c * 4);
                    v = first ? b : F::add(v, b);
                    first = false;
                }
            }
            unsigned char *dst = T + (size_t)(h << G) * P * SRB + c * 16;
            const int rot = (tid / CG) % REP;
#pragma unroll
            for (int i = 0; i < REP; i++) {
                const int rho = (i + rot) % REP;
#pragma unroll
                for (int p = 0; p < P; p++)
                    *reinterpret_cast<uint4 *>(dst + p * SRB + rho * TWD * 4) = v.p[p];
            }
        }
        __syncthreads();

        // (d) build phase 2: walk the low G bits of each high part in Gray-code order
        if (G > 0) {
            for (int task = tid; task < CG * NH; task += NT) {
                const int c = task % CG, cc = task / CG;
                const int rot = (tid / CG) % REP;
                // row t of the slab for this column group, read from the LDS staging area
                auto brow = [&](int t) {
                    typename F::V b;
#pragma unroll
                    for (int p = 0; p < P; p++)
                        b.p[p] = *reinterpret_cast<const uint4 *>(Bs + (t * P + p) * TWD + c * 4);
                    return b;
                };
                const int hg = cc ^ (cc >> 1);
                typename F::V v;
                const unsigned char *src = T + (size_t)(hg << G) * P * SRB + c * 16;
#pragma unroll
                for (int p = 0; p < P; p++) v.p[p] = *reinterpret_cast<const uint4 *>(src + p * SRB);
                auto store = [&](int e, const typename F::V &x) {
                    unsigned char *dst = T + (size_t)e * P * SRB + c * 16;
#pragma unroll
                    for (int i = 0; i < REP; i++) {
                        const int rho = (i + rot) % REP;
#pragma unroll
                        for (int p = 0; p < P; p++)
                            *reinterpret_cast<uint4 *>(dst + p * SRB + rho * TWD * 4) = x.p[p];
                    }
                };
                if (cc & 1) {
                    v = F::add(v, brow(G - 1));
                    store((hg << G) | (1 << (G - 1)), v);
                }
                const int jb = cc << G;
                for (int j = 1; j < (1 << G); j++) {
                    const int jj = jb + j;
                    const int b = __builtin_ctz(jj);
                    const int e = jj ^ (jj >> 1);
                    const typename F::V rb = brow(b);
                    // a bit switched on adds its row, a bit switched off subtracts it
                    if ((e >> b) & 1) v = F::add(v, rb);
                    else v = F::sub(v, rb);
                    store(e, v);
                }
            }
            __syncthreads();
        }

        // (e) accumulate: every row of the tile gathers D table rows per slab
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int lr = rs + r * RS;
            const uint4 o = *reinterpret_cast<const uint4 *>(Ib + lr * 4);
            const u32 off[3] = {o.x, o.y, o.z};
            typename F::V t[D];
#pragma unroll
            for (int d = 0; d < D; d++) {
                const unsigned char *src = T + off[d] + laneoff;
#pragma unroll
                for (int p = 0; p < P; p++) t[d].p[p] = *reinterpret_cast<const uint4 *>(src + p * SRB);
            }
            F::accumulate(acc[r], t);
        }
    }

    // store: combine, canonicalise (single slice) and zero the pad columns
    const int w = colw0 + cg * 4;
    if (w < a.Wn) {
        const uint4 msk = colmask(w, a.n);
        u32 *out = a.out + (size_t)blockIdx.z * a.split_stride;
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int row = row0 + rs + r * RS;
            if (row < a.m) {
                typename F::V v = F::finish(acc[r]);
                if (a.canon) v = F::canon(v);
#pragma unroll
                for (int p = 0; p < P; p++)
                    *reinterpret_cast<uint4 *>(out + ((size_t)row * P + p) * a.Wn + w) = and4(v.p[p], msk);
            }
        }
    }
}

// Sum of `splits` partial products (same packed layout, split_stride words apart), then
// canonicalise and zero the pad columns.  One thread per (row, 4-word group).
template <int Q>
__global__ __launch_bounds__(256) void reduce_partials_kernel(const u32 *part, u32 *C, int m, int n, int Wn,
                                                              int splits, size_t split_stride) {
    typedef FT<Q> F;
    constexpr int P = F::P;
    const int groups = Wn / 4;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)m * groups) return;
    const int row = (int)(idx / groups), w = (int)(idx % groups) * 4;
    typename F::V v;
#pragma unroll
    for (int p = 0; p < P; p++) v.p[p] = *reinterpret_cast<const uint4 *>(part + ((size_t)row * P + p) * Wn + w);
    for (int z = 1; z < splits; z++) {
        typename F::V x;
        const u32 *pz = part + z * split_stride;
#pragma unroll
        for (int p = 0; p < P; p++) x.p[p] = *reinterpret_cast<const uint4 *>(pz + ((size_t)row * P + p) * Wn + w);
        v = F::add(v, x);
    }
    v = F::canon(v);
    const uint4 msk = colmask(w, n);
#pragma unroll
    for (int p = 0; p < P; p++) *reinterpret_cast<uint4 *>(C + ((size_t)row * P + p) * Wn + w) = and4(v.p[p], msk);
}

// ---------------------------------------------------------------------------------------
// Pack / unpack.  One wave per (row, 64 columns): each lane takes one element, and a
// wave-wide ballot of one plane bit yields that plane's 64-bit word pair.
// ---------------------------------------------------------------------------------------
template <int Q>
__device__ __forceinline__ void encode(u32 v, u32 *bits) {
    if (Q == 3) {
        v %= 3u;
        bits[0] = v != 0u;
        bits[1] = v == 2u;
    } else if (Q == 4) {
        bits[0] = v & 1u;
        bits[1] = (v >> 1) & 1u;
    } else {
        v %= (u32)Q;
        bits[0] = v & 1u; bits[1] = (v >> 1) & 1u; bits[2] = (v >> 2) & 1u;
    }
}

template <int Q>
__global__ __launch_bounds__(256) void pack_kernel(const uint8_t *src, int64_t ld, u32 *dst, int rows, int cols, int W) {
    constexpr int P = FT<Q>::P;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int chunks = W / 2;                    // 64-column chunks per row
    const int64_t items = (int64_t)rows * chunks;
    for (int64_t it = wave; it < items; it += nwaves) {
        const int row = (int)(it / chunks), ch = (int)(it % chunks);
        const int col = ch * 64 + lane;
        u32 v = col < cols ? src[(int64_t)row * ld + col] : 0u;
        u32 bits[P];
        encode<Q>(v, bits);
        if (col >= cols) {
#pragma unroll
            for (int p = 0; p < P; p++) bits[p] = 0u;
        }
#pragma unroll
        for (int p = 0; p < P; p++) {
            const uint64_t b = __ballot(bits[p] != 0u);
            if (lane == 0) {
                uint2 wv = make_uint2((u32)b, (u32)(b >> 32));
                *reinterpret_cast<uint2 *>(dst + ((size_t)row * P + p) * W + ch * 2) = wv;
            }
        }
    }
}

template <int Q>
__global__ __launch_bounds__(256) void unpack_kernel(const u32 *src, uint8_t *dst, int64_t ld, int rows, int cols, int W) {
    constexpr int P = FT<Q>::P;
    const int64_t total = (int64_t)rows * cols;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int row = (int)(idx / cols), col = (int)(idx % cols);
        u32 b[P];
#pragma unroll
        for (int p = 0; p < P; p++) b[p] = (src[((size_t)row * P + p) * W + (col >> 5)] >> (col & 31)) & 1u;
        u32 v;
        if (Q == 3) v = b[0] ? (b[1] ? 2u : 1u) : 0u;
        else if (Q == 4) v = b[0] | (b[1] << 1);
        else v = (b[0] | (b[1] << 1) | (b[2] << 2)) % (u32)Q;
        dst[(int64_t)row * ld + col] = (uint8_t)v;
    }
}

// ---------------------------------------------------------------------------------------
// Host-side launchers (called from gfq_api.cpp).
// ---------------------------------------------------------------------------------------
template <int Q, int TWD, int REP, int R>
static hipError_t launch_mm(const MMArgs &a, int rowsTile, hipStream_t st) {
    constexpr int NT = 512;
    constexpr int P = FT<Q>::P;
    constexpr int LPR = TWD / 4;
    constexpr int TM = (NT / LPR) * R;
    (void)rowsTile;
    const size_t lds = (size_t)(1u << a.k) * P * (REP * TWD * 4) + 2 * KMAX * P * TWD * 4 + 2 * TM * 16;
    dim3 grid((a.Wn + TWD - 1) / TWD, (a.m + TM - 1) / TM, (a.S + a.slabs_per_split - 1) / a.slabs_per_split);
    auto kern = m4rm_kernel<Q, TWD, REP, R, NT>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, st, a);
    return hipGetLastError();
}

template <int Q, int TWD, int REP>
static hipError_t launch_mm_rows(const MMArgs &a, int rowsTile, hipStream_t st) {
    constexpr int LPR = TWD / 4;
    const int R = rowsTile * LPR / 512;
    if (R <= 1) return launch_mm<Q, TWD, REP, 1>(a, rowsTile, st);
    if (R == 2) return launch_mm<Q, TWD, REP, 2>(a, rowsTile, st);
    if (R <= 4) return launch_mm<Q, TWD, REP, 4>(a, rowsTile, st);
    return launch_mm<Q, TWD, REP, 8>(a, rowsTile, st);
}

template <int Q>
static hipError_t launch_mm_q(const MMArgs &a, int variant, int rowsTile, hipStream_t st) {
    switch (variant) {
    case LAYOUT_W32_R2: return launch_mm_rows<Q, 32, 2>(a, rowsTile, st);
    case LAYOUT_W32_R1: return launch_mm_rows<Q, 32, 1>(a, rowsTile, st);
    case LAYOUT_W16_R1: return launch_mm_rows<Q, 16, 1>(a, rowsTile, st);
    default: return launch_mm_rows<Q, 8, 1>(a, rowsTile, st);
    }
}

hipError_t launch_matmul(int q, const MMArgs &a, int variant, int rowsTile, hipStream_t st) {
    switch (q) {
    case 3: return launch_mm_q<3>(a, variant, rowsTile, st);
    case 4: return launch_mm_q<4>(a, variant, rowsTile, st);
    case 5: return launch_mm_q<5>(a, variant, rowsTile, st);
    default: return launch_mm_q<7>(a, variant, rowsTile, st);
    }
}

hipError_t launch_reduce(int q, const u32 *part, u32 *C, int m, int n, int Wn, int splits, size_t stride, hipStream_t st) {
    const size_t threads = (size_t)m * (Wn / 4);
    dim3 grid((unsigned)((threads + 255) / 256));
    switch (q) {
    case 3: hipLaunchKernelGGL(reduce_partials_kernel<3>, grid, dim3(256), 0, st, part, C, m, n, Wn, splits, stride); break;
    case 4: hipLaunchKernelGGL(reduce_partials_kernel<4>, grid, dim3(256), 0, st, part, C, m, n, Wn, splits, stride); break;
    case 5: hipLaunchKernelGGL(reduce_partials_kernel<5>, grid, dim3(256), 0, st, part, C, m, n, Wn, splits, stride); break;
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
    const int64_t items = (int64_t)rows * (W / 2);
    dim3 grid(grid_for(items, 4));
    switch (q) {
    case 3: hipLaunchKernelGGL(pack_kernel<3>, grid, dim3(256), 0, st, src, ld, dst, rows, cols, W); break;
    case 4: hipLaunchKernelGGL(pack_kernel<4>, grid, dim3(256), 0, st, src, ld, dst, rows, cols, W); break;
    case 5: hipLaunchKernelGGL(pack_kernel<5>, grid, dim3(256), 0, st, src, ld, dst, rows, cols, W); break;
    default: hipLaunchKernelGGL(pack_kernel<7>, grid, dim3(256), 0, st, src, ld, dst, rows, cols, W); break;
    }
    return hipGetLastError();
}

hipError_t launch_unpack(int q, const u32 *src, uint8_t *dst, int64_t ld, int rows, int cols, int W, hipStream_t st) {
    dim3 grid(grid_for((int64_t)rows * cols, 256));
    switch (q) {
    case 3: hipLaunchKernelGGL(unpack_kernel<3>, grid, dim3(256), 0, st, src, dst, ld, rows, cols, W); break;
    case 4: hipLaunchKernelGGL(unpack_kernel<4>, grid, dim3(256), 0, st, src, dst, ld, rows, cols, W); break;
    case 5: hipLaunchKernelGGL(unpack_kernel<5>, grid, dim3(256), 0, st, src, dst, ld, rows, cols, W); break;
    default: hipLaunchKernelGGL(unpack_kernel<7>, grid, dim3(256), 0, st, src, dst, ld, rows, cols, W); break;
    }
    return hipGetLastError();
}

}  // namespace gfq
