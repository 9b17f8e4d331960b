// gfq_m4rm_tile.h -- the Four-Russians product on one tile, shared by the plain kernel
// and the work-list kernel of batches.
//
// Method (paper, Section 2): row i of C is sum_j a_ij B_j.  The inner dimension is cut
// into slabs of k rows of B; for each slab a table of all 2^k binary combinations of its
// rows is built once and shared by every row of C.  With an additive basis {alpha_d} and
// bit maps phi_d (a = sum_d alpha_d phi_d(a)), the slab adds sum_d alpha_d T[phi_d(a_i)]
// to row i, so only binary combinations are ever tabulated.
//
// Work decomposition
//   grid.x  column tile: TWD 32-bit words of every plane (32 * TWD columns of C)
//   grid.y  row tile: TM = R * NT / (TWD / 4) rows of C
//   grid.z  slice of the slabs ("split-l"); more than one slice writes partial products
//           that the reduce kernel sums.
// Each lane owns 4 consecutive words of R rows of C and keeps their accumulators in VGPRs.
//
// Pipeline per workgroup (one barrier per slab).  Iteration s:
//   stage   write slab s+3's rows of B (loaded into registers one iteration earlier) and
//           the phi_d table offsets of every row of the tile for slab s+2 into LDS;
//   prefix  (F_5, F_7) the chunk prefixes of slab s+2's table;
//   build   the table of slab s+1 into the idle table buffer, in Gray-code order;
//   gather  for every row, D table rows of slab s, alpha_d-scaled into the accumulator;
//   barrier.
// The build of slab s+1 and the gathers of slab s are independent: half of the waves
// build first, the other half gather first, so every SIMD overlaps the two.  Where a
// tile's gathers outweigh its build (F::HALF_BUILD_ROWS rows per lane or more) only the
// first half of the waves builds, each thread walking twice as many entries.
//
// LDS table layout.  One (entry, plane) "super-row" is SRB bytes holding REP copies of
// the TWD-word tile row.  gfx950 serves a 128-bit LDS read of 16 lanes from 64 four-byte
// banks in one pass, so a 16-lane group is conflict-free exactly when its 16 reads cover
// 256 distinct consecutive bytes: with SRB = 256 the REP rows of C gathered by one 16-lane
// group come from different copies.  With SRB = 128 a super-row is one 32-word row and a
// group serves two rows of C, each in one half of the banks (planes swapped on odd entries
// when their number is even, so that the half follows the entry; for F_3, F_9 and GF(4), whose
// accumulation survives exchanged planes, the second row reads them exchanged and never meets
// the first); with SRB = 64 and less,
// four or more rows of C share a group and conflict as their entries fall.  Table 0 sits
// at LDS offset 0 and table 1 at TB1, a power of two not below the table size, so an
// address is (offset | lane offset | base).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gfq_device.h"
#include "gfq_internal.h"

namespace gfq {

__device__ __forceinline__ u32 comp4(const uint4 &v, int i) {
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

template <int H> struct half_tag { static constexpr int value = H; };

// Tiles whose rows of C, two to a 16-lane read pass, read their table planes in opposite
// orders (see m4rm_tile, GSW): fields negated by exchanging planes 2j and 2j + 1, 128-byte
// super-rows.  With two table planes an entry takes 256 bytes, so its offset is the entry
// index times 256: one byte, and every gathered address is put together by one byte
// permutation (lane byte, entry byte, table-base bytes).  That needs the second table at a
// multiple of 65536 bytes (the launcher checks it).
template <int Q, int TWD, int REP> constexpr bool gsw_tile() {
    return FT<Q>::EXCHANGE_READS && REP == 1 && TWD == 32;
}
// Three-plane fields with a front slot (F_7, GF(8); F::FRONT_SLOT) at 128-byte super-rows:
// each entry gets a fourth slot in front, so that the second row of a read pass reads
// lam * t (F_7: the doubled entry, GF(8): x t) from slots 0, 1, 2 while the first reads t
// from slots 1, 2, 3, each plane at the same offset from its row's base.  Entries are 512
// bytes, so slot j sits in half j mod 2 of the banks and the two rows never meet; the second
// row accumulates lam C, mapped back before the store.
template <class F, class = void> struct has_front_slot : std::false_type {};
template <class F> struct has_front_slot<F, std::void_t<decltype(F::FRONT_SLOT)>> : std::bool_constant<F::FRONT_SLOT> {};
template <int Q, int TWD, int REP> constexpr bool dbl_copy_tile() {
    return has_front_slot<FT<Q>>::value && REP == 1 && TWD == 32;
}
// the slot of plane p relative to the row's base slot (front-slot tiles), else p
template <class F, bool DCP> constexpr int plane_slot(int p) {
    if constexpr (DCP) return F::front_slot(p) - 1;
    else return p;
}
// fields whose exchanged reads also exchange the two gathers' table rows (GF(4))
template <class F> constexpr bool exchange_slots() {
    if constexpr (F::EXCHANGE_READS) return F::EXCHANGE_SLOTS;
    else return false;
}
template <int Q, int TWD, int REP> constexpr bool perm_addr_tile() {
    return gsw_tile<Q, TWD, REP>() && FT<Q>::PT == 2 && !FT<Q>::HALF_ROWS;
}

// The tile of the product `a` whose first row is row0 (R * NT / (TWD / 4) rows, fewer where
// the product ends) and whose first column word is colw0 (TWD words), over slab slice bz.
// Called by every thread of an NT-thread workgroup; uses the workgroup's dynamic LDS.  ITEM:
// the tile is one item of a batch (see the thread index below).
template <int Q, int TWD, int REP, int R, int NT, bool ITEM = false>
__device__ __forceinline__ void m4rm_tile_rows(const MMArgs &a, int colw0, int row0, int bz) {
    typedef FT<Q> F;
    // P planes per row in the packed operands, PT planes per table entry, D table rows
    // gathered per slab (GP planes of each), PA accumulator planes per word
    constexpr int P = F::P, PT = F::PT, D = F::D, GP = F::GP, PA = F::PA;
    constexpr int LPR = TWD / 4;                 // lanes per row of C
    constexpr int SRB = REP * TWD * 4;           // bytes per (entry, plane) super-row
    constexpr int RS = NT / LPR;                 // row slots per pass
    constexpr int TM = RS * R;                   // rows of C per workgroup
    constexpr int CG = TWD / 4;                  // 4-word column groups per tile
    constexpr int ARPT = (TM + NT - 1) / NT;     // tile rows staged per thread
    constexpr int NCH = NT / TWD;                // build chunks per column word
    constexpr int LOG_NCH = log2_floor(NCH);
    constexpr int IBW = (D + 1) / 2;             // u32 words per row of the offset buffer
    // 128-byte super-rows hold one 32-word tile row: a 16-lane read pass serves two rows of C,
    // each reading one half of the 64 banks.  With an even number of table planes every
    // entry starts on a 256-byte boundary, so plane p of every entry would sit in the same
    // half and the two rows of a pass would always meet there: planes swap in pairs on odd
    // entries (plane p of entry e at (p ^ (e & 1)) * SRB), so the halves follow the entries.
    //
    // Fields whose accumulation survives exchanged planes (F::EXCHANGE_READS: F_3 and F_9,
    // whose entries exchanging planes 2j and 2j + 1 negates, and GF(4)) avoid the meetings
    // altogether: the second row of every pass (lanes 8-15 of each 16) reads plane p ^ 1 where
    // the first reads plane p, so the two rows are always in opposite halves; that row
    // accumulates a fixed linear image of C (-C; GF(4), whose second row also takes its two
    // gathers' table rows in exchanged order: x^2 C^2), mapped back before it is stored.
    constexpr bool GSW = gsw_tile<Q, TWD, REP>();
    constexpr bool PERM = perm_addr_tile<Q, TWD, REP>();
    static_assert(!GSW || (SRB == 128 && LPR == 8), "two rows of C per 16-lane pass");
    constexpr bool SWZ = (PT % 2 == 0) && SRB == 128 && !GSW;
    constexpr bool XSW = SWZ || GSW;             // odd planes read at the row's address ^ SRB
    // gathers of three rows ahead where the accumulate per row is short (F_3: 32 instructions
    // per row against four 128-bit reads) and the registers allow it (250 VGPRs at 16 rows per
    // lane; two rows ahead measured 3% slower on the F_3 8192^3 product)
    constexpr bool PF3 = GSW && R == 16;
    constexpr bool DCP = dbl_copy_tile<Q, TWD, REP>();
    static_assert(!DCP || (PT == 3 && SRB == 128 && !GSW && !SWZ), "doubled copy: three planes, 128-byte super-rows");
    constexpr int ES = (PT + (DCP ? 1 : 0)) * SRB;   // bytes per table entry
    static_assert(KMAX * P * CG <= NT, "one B staging chunk per thread");
    static_assert(REP * LPR <= 16, "super-row wider than a 16-lane read group");
    static_assert(NCH % REP == 0 || REP % NCH == 0, "replica rotation");

    extern __shared__ __align__(16) unsigned char smem[];
    const int k = a.k;
    const u32 tbytes = (u32)(1u << k) * ES;
    const u32 TB1 = a.tb1;                       // power of two >= tbytes, <= 65536
    u32 *Bst = reinterpret_cast<u32 *>(smem + TB1 + tbytes);   // [3][KMAX][P][TWD]
    u32 *PB = Bst + 3 * KMAX * P * TWD;                         // [2][NCH][PT][TWD] (split prefixes)
    u32 *Ib = PB + (F::SPLIT_PREFIX ? 2 * NCH * PT * TWD : 0);  // [3][TM][IBW]

    // In a batch item the thread index passes through an empty asm statement, so that nothing
    // derived from it is hoisted out of the tile: in a persistent workgroup's loop over items
    // such values stay live across every tile variant of the loop and crowd the registers
    // (15-25 VGPRs per batch kernel).  The single-product kernels keep the plain index: the
    // opaque one ran the F_5 8192^3 product 3% slower.
    int tid = threadIdx.x;
    if constexpr (ITEM) asm volatile("" : "+v"(tid));
    const int s_begin = bz * a.slabs_per_split;
    const int s_end = min(a.S, s_begin + a.slabs_per_split);
    const u32 kmask = (1u << k) - 1u;

    // ---- staging of B: chunk (row t of the slab, plane p, 4-word group c) per thread ----
    const int bt = tid / (P * CG), bp = (tid / CG) % P, bc = tid % CG;
    const bool b_active = tid < k * P * CG;
    const int bcol = colw0 + bc * 4;
    // Global loads inside the slab loop read addresses clamped into the operand (a slab
    // exists, so l >= 1, and the tile exists, so m, n >= 1) and the values of out-of-range
    // positions are masked where they are used.  No load has a path that writes its
    // destination register otherwise: such a write (a zero for an out-of-range position)
    // would have to wait for every load in flight, including the prefetches just issued.
    auto load_b = [&](int s) -> uint4 {
        const int brow = min(s * k + bt, a.l - 1);
        const int col = min(bcol, a.Wn - 4);
        return *reinterpret_cast<const uint4 *>(a.B + ((size_t)brow * P + bp) * a.Wn + col);
    };
    auto store_b = [&](int s, const uint4 &v) {
        const u32 m = (s * k + bt < a.l && bcol < a.Wn) ? 0xffffffffu : 0u;
        if (b_active)
            *reinterpret_cast<uint4 *>(Bst + (((s % 3) * KMAX + bt) * P + bp) * TWD + bc * 4) =
                make_uint4(v.x & m, v.y & m, v.z & m, v.w & m);
    };

    // ---- staging of A: a window of words (w, w+1, w+2) per staged row and plane ----
    // Staging slot j of this thread is position i = tid + j NT of the offset buffer, which
    // holds the rows of one row slot together (position rs R + r for row rs + r RS, so that a
    // lane fetches its R rows' offsets with 128-bit reads); slot j therefore stages that
    // row, and the offsets of a wave's 64 lanes land in consecutive words (no bank conflict).
    auto srow = [&](int j) -> int {
        const int i = min(tid + j * NT, TM - 1);
        return (i % R) * RS + i / R;
    };
    u32 aw[ARPT][P][3], apre[ARPT][P];
    int aw_w = (s_begin * k) >> 5;
    // One staged row per thread and at most three planes: the words entering the window come
    // from a 16-byte quad per plane (one load per four moves, a quarter of the cache misses
    // of single-word loads; the rows are far apart, so their lines rarely last between two
    // moves).  Elsewhere the registers are short and the next word is loaded alone.
    constexpr bool AQ = ARPT == 1 && P <= 3;
    uint4 aq[AQ ? P : 1];
    // the quad holding word wn of this thread's row (clamped into the operand; the words
    // outside it are masked where they enter the window).  Called only when the slice has
    // slabs, so l >= 1, Wl >= 4 and m >= 1 (a tile exists).
    auto load_quad = [&](int wn) {
        const int qw = min(wn & ~3, a.Wl - 4);
        const int row = min(row0 + srow(0), a.m - 1);
#pragma unroll
        for (int p = 0; p < (AQ ? P : 0); p++)
            aq[p] = *reinterpret_cast<const uint4 *>(a.A + ((size_t)row * P + p) * a.Wl + qw);
    };
    auto quad_word = [](const uint4 &q, int c) -> u32 { return c == 0 ? q.x : (c == 1 ? q.y : (c == 2 ? q.z : q.w)); };
    auto a_word = [&](int j, int p, int w) -> u32 {
        const int row = row0 + srow(j);
        if (tid + j * NT < TM && row < a.m && w < a.Wl) return a.A[((size_t)row * P + p) * a.Wl + w];
        return 0u;
    };
#pragma unroll
    for (int j = 0; j < ARPT; j++)
#pragma unroll
        for (int p = 0; p < P; p++) {
            aw[j][p][0] = a_word(j, p, aw_w);
            aw[j][p][1] = a_word(j, p, aw_w + 1);
            aw[j][p][2] = a_word(j, p, aw_w + 2);
            apre[j][p] = AQ ? 0u : a_word(j, p, aw_w + 3);
        }
    // (only with slabs to walk: a tile of an l = 0 product has none, and then Wl = 0)
    if constexpr (AQ) {
        if (s_begin < s_end) load_quad(aw_w + 3);
    }
    auto apre_mask = [&](int j, int w) -> u32 {
        return (tid + j * NT < TM && row0 + srow(j) < a.m && w < a.Wl) ? 0xffffffffu : 0u;
    };
    // offsets (u16, entry * ES) of the D table rows for slab s, for every tile row
    auto stage_idx = [&](int s) {
        const int sh = (s * k) & 31;
        u32 *ib = Ib + (s % 3) * TM * IBW;
#pragma unroll
        for (int j = 0; j < ARPT; j++) {
            const int pos = tid + j * NT;           // row srow(j)
            if (pos < TM) {
                u32 x[P], f[D];
#pragma unroll
                for (int p = 0; p < P; p++) x[p] = __builtin_amdgcn_alignbit(aw[j][p][1], aw[j][p][0], sh) & kmask;
                F::phis(x, f);
                u32 o[IBW * 2];
#pragma unroll
                for (int d = 0; d < IBW * 2; d++) {
                    const u32 e = d < D ? f[d < D ? d : 0] : 0u;
                    o[d] = e * (u32)ES + (SWZ ? (e & 1u) * (u32)SRB : 0u);   // slot 0's place
                }
                // the row is gathered by the lanes at row slot pos / R: the second row of a
                // read pass takes the two table rows in exchanged order (GF(4))
                if constexpr (GSW && exchange_slots<F>()) {
                    static_assert(D == 2, "two gathers");
                    if ((pos / R) & 1) {
                        const u32 t = o[0];
                        o[0] = o[1];
                        o[1] = t;
                    }
                }
#pragma unroll
                for (int w = 0; w < IBW; w++) ib[pos * IBW + w] = o[2 * w] | (o[2 * w + 1] << 16);
            }
        }
    };
    // the word the next move brings in: a load from a clamped address, masked when it
    // enters the window
    auto prefetch_a = [&]() {
        if constexpr (AQ) {
            if (((aw_w + 3) & 3) == 0) load_quad(aw_w + 3);     // else the held quad has it
            return;
        }
        const int w = min(aw_w + 3, a.Wl - 1);
#pragma unroll
        for (int j = 0; j < ARPT; j++) {
            const int row = min(row0 + srow(j), a.m - 1);
#pragma unroll
            for (int p = 0; p < P; p++) apre[j][p] = a.A[((size_t)row * P + p) * a.Wl + w];
        }
    };
    // move the window to the words of slab s (called in slab order; k < 32 so it moves by
    // at most one word); true if it moved.  The word entering the window was prefetched
    // after the previous move (at least three slabs earlier); the caller prefetches the
    // next one after its other loads.
    auto advance = [&](int s) -> bool {
        const int w = (s * k) >> 5;
        if (w == aw_w) return false;
#pragma unroll
        for (int j = 0; j < ARPT; j++)
#pragma unroll
            for (int p = 0; p < P; p++) {
                aw[j][p][0] = aw[j][p][1];
                aw[j][p][1] = aw[j][p][2];
                aw[j][p][2] = (AQ ? quad_word(aq[p], (w + 2) & 3) : apre[j][p]) & apre_mask(j, w + 2);
            }
        aw_w = w;
        return true;
    };

    // ---- table build.  Entry e of a slab's table is split as e = (c << G) | g: chunk c
    // (C = k - G high bits, at most NCH chunks) and walk index g.  Thread (word dw, chunk c)
    // starts from the chunk prefix T[c << G], the sum of rows G + t over the bits t of c,
    // and walks the G low bits in Gray-code order, adding row b when bit b switches on and
    // subtracting it when it switches off.  For three-plane fields the prefixes come from
    // a stage one slab earlier (prefix): NCH/4 threads per word each take four consecutive
    // chunks (a masked sum over the bits above the lowest two, then a Gray walk over those
    // two) and leave them in a small buffer.  Where a table addition is short (F_3: 4
    // instructions; GF(4), GF(8): one XOR per plane) each thread sums its own prefix (a
    // masked sum).  The rows a stage needs are read from LDS in one batch before its chain
    // of additions. ----
    constexpr bool SPLIT_PREFIX = F::SPLIT_PREFIX;
    // HALF_BUILD: only the first half of the waves build (one per SIMD), each walking twice
    // as far, so that half as many chunk prefixes are summed (F::HALF_BUILD_ROWS)
    constexpr bool HALF_BUILD = NCH >= 8 && R >= F::HALF_BUILD_ROWS;
    constexpr int LOG_NB = LOG_NCH - (HALF_BUILD ? 1 : 0);     // log2 of the building chunks
    constexpr int NB = 1 << LOG_NB;
    // the widest slab whose two tables fit 128 KiB at this super-row width
    constexpr int KT = log2_floor(65536 / ES) < KMAX ? log2_floor(65536 / ES) : KMAX;
    constexpr int GMAX = KT > LOG_NB ? KT - LOG_NB : 0;         // longest walk: 2^GMAX entries
    constexpr int PFW = NB / 4;                                 // prefix threads per word
    constexpr int PFB = LOG_NB > 2 ? LOG_NB - 2 : 0;           // masked bits per prefix thread
    static_assert(NB >= 4, "four chunks per prefix thread");
    const int dw = tid % TWD, ch = tid / TWD;
    const int C = k > LOG_NB ? LOG_NB : k;       // chunk bits
    const int G = k - C;                         // walk bits
    const int nchunks = 1 << C;
    u32 rep_off[REP];                            // this chunk's copy rotation
#pragma unroll
    for (int i = 0; i < REP; i++) rep_off[i] = (u32)(((i + ch) % REP) * TWD * 4);
    auto step = [&](u32 *v, const u32 *r, bool on) {
        u32 z[PT];
        if (on) F::tadd(v, r, z);
        else F::tsub(v, r, z);
#pragma unroll
        for (int p = 0; p < PT; p++) v[p] = z[p];
    };
    // Every staged row index read below is below KMAX, inside the staging buffer, so the
    // reads are unconditional (rows at or beyond k hold stale data and are masked or never
    // enter a stored value).
    auto prefix = [&](int s) {
        if (!SPLIT_PREFIX || ch >= PFW) return;  // thread (dw, g = ch) of the first NT/4
        const u32 *bs = Bst + (s % 3) * KMAX * P * TWD + dw;
        u32 *pb = PB + (s & 1) * NCH * PT * TWD + dw;
        u32 hr[PFB > 0 ? PFB : 1][PT], lo0[PT], lo1[PT];
#pragma unroll
        for (int t = 0; t < PFB; t++) {
            u32 x[P];
#pragma unroll
            for (int p = 0; p < P; p++) x[p] = bs[((G + 2 + t) * P + p) * TWD];
            F::to_table(x, hr[t]);
        }
        {
            u32 x[P], y[P];
#pragma unroll
            for (int p = 0; p < P; p++) {
                x[p] = bs[(G * P + p) * TWD];
                y[p] = bs[((G + 1) * P + p) * TWD];
            }
            F::to_table(x, lo0);
            F::to_table(y, lo1);
        }
        u32 v[PT];
#pragma unroll
        for (int p = 0; p < PT; p++) v[p] = 0u;
#pragma unroll
        for (int t = 0; t < PFB; t++) {
            const u32 m = (2 + t < C) ? 0u - (u32)((ch >> t) & 1) : 0u;
            u32 r[PT];
#pragma unroll
            for (int p = 0; p < PT; p++) r[p] = hr[t][p] & m;        // the zero row adds nothing
            step(v, r, true);
        }
        const int c0 = ch * 4;
        auto put = [&](int c, const u32 *x) {
            if (c < nchunks)
#pragma unroll
                for (int p = 0; p < PT; p++) pb[(c * PT + p) * TWD] = x[p];
        };
        put(c0, v);
        step(v, lo0, true);
        put(c0 + 1, v);
        step(v, lo1, true);
        put(c0 + 3, v);
        step(v, lo0, false);
        put(c0 + 2, v);
    };
    auto build = [&](int s) {
        if (ch >= nchunks) return;
        const u32 *bs = Bst + (s % 3) * KMAX * P * TWD + dw;
        unsigned char *T = smem + ((s & 1) ? TB1 : 0u) + dw * 4;
        // entry of parity b at dst (plane order swapped in pairs on odd entries when SWZ)
        auto store = [&](unsigned char *dst, const u32 *v, u32 b) {
            if constexpr (DCP) {
                // slot 0: the front value; plane p at slot F::front_slot(p)
                *reinterpret_cast<u32 *>(dst) = F::front(v);
#pragma unroll
                for (int p = 0; p < PT; p++) *reinterpret_cast<u32 *>(dst + F::front_slot(p) * SRB) = v[p];
                return;
            }
#pragma unroll
            for (int i = 0; i < REP; i++)
#pragma unroll
                for (int p = 0; p < PT; p++)
                    *reinterpret_cast<u32 *>(dst + (SWZ ? ((u32)p ^ b) : (u32)p) * SRB + rep_off[i]) = v[p];
        };
        u32 v[PT];
        if constexpr (SPLIT_PREFIX) {
            const u32 *pb = PB + (s & 1) * NCH * PT * TWD + dw;
#pragma unroll
            for (int p = 0; p < PT; p++) v[p] = pb[(ch * PT + p) * TWD];
        } else {
            // the chunk's prefix here: the sum of its rows G + t over the bits t of ch.  A wave
            // holds 64 / TWD consecutive chunks, so only the low LOWB bits of ch differ
            // between its lanes: those rows enter masked (the zero row adds nothing, and the
            // first one is the prefix itself), the others only where the wave's bit is set
            // (a branch on a value every lane shares).
            constexpr int LOWB = TWD >= 64 ? 0 : log2_floor(64 / TWD);
            const int chw = __builtin_amdgcn_readfirstlane(ch);
#pragma unroll
            for (int p = 0; p < PT; p++) v[p] = 0u;
#pragma unroll
            for (int t = 0; t < LOG_NCH; t++) {
                if (t >= C) break;
                if (t >= LOWB && !((chw >> t) & 1)) continue;
                u32 pr[P], x[PT];
#pragma unroll
                for (int p = 0; p < P; p++) pr[p] = bs[((G + t) * P + p) * TWD];
                F::to_table(pr, x);
                if (t < LOWB) {
                    const u32 m = 0u - (u32)((ch >> t) & 1);
#pragma unroll
                    for (int p = 0; p < PT; p++) x[p] &= m;
                }
                if (t == 0) {
#pragma unroll
                    for (int p = 0; p < PT; p++) v[p] = x[p];
                } else {
                    step(v, x, true);
                }
            }
        }
        unsigned char *eb = T + (u32)(ch << G) * ES;
        store(eb, v, G == 0 ? (u32)(ch & 1) : 0u);
        if constexpr (GMAX > 0) {
            u32 wr[GMAX > 0 ? GMAX : 1][PT];
#pragma unroll
            for (int b = 0; b < GMAX; b++) {
                u32 x[P];
#pragma unroll
                for (int p = 0; p < P; p++) x[p] = bs[(b * P + p) * TWD];
                F::to_table(x, wr[b]);
            }
#pragma unroll
            for (int j = 1; j < (1 << GMAX); j++) {
                if (j >= (1 << G)) break;
                const int b = __builtin_ctz(j);
                const int g = j ^ (j >> 1);
                step(v, wr[b], (g >> b) & 1);
                store(eb + g * ES, v, (u32)(g & 1));             // j < 2^G: G >= 1, parity of g
            }
        }
    };

    // ---- accumulators: R rows x 4 words x PA planes per lane ----
    u32 acc[R][4][PA];
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int i = 0; i < 4; i++) F::acc_init(acc[r][i], s_end - s_begin);

    const int rs = tid / LPR, cg = tid % LPR;
    const bool neg_row = GSW && ((tid / LPR) & 1);   // reads planes exchanged, accumulates -C
    // the first row of a doubled-copy pass reads slots 1, 2, 3, the second slots 0, 1, 2
    const bool dbl_row = DCP && ((tid / LPR) & 1);
    const u32 laneoff = (u32)(tid % (REP * LPR)) * 16u + (neg_row ? (u32)SRB : 0u) + ((DCP && !dbl_row) ? (u32)SRB : 0u);

    // gathers of one row: D table rows, GP planes each (plane F::gplane(d, p) of row d), 4 words
    // per lane
    // The kernels allocate no static LDS, so the dynamic buffer starts at LDS address 0 and
    // an offset into it is its LDS address: the reads go through an LDS pointer made from
    // the offset, which spares an addition of the buffer's base per table row.
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(3))) const u32x4 lds_u32x4;
    auto fetch = [&](const u32 *iw, int r, u32 lo, uint4 (&t)[D][GP]) {
#pragma unroll
        for (int d = 0; d < D; d++) {
            const u32 x = iw[r * IBW + (d >> 1)];
            u32 off, offx;
            if constexpr (PERM) {
                // offsets are entry * 256 (byte 1 of each 16-bit half); lo holds the lane's
                // byte offset (byte 0) and the table base (bytes 2, 3)
                const u32 sel = (d & 1) ? 0x03020700u : 0x03020500u;
                off = __builtin_amdgcn_perm(x, lo, sel);
                offx = __builtin_amdgcn_perm(x, lo ^ (u32)SRB, sel);
            } else {
                off = ((d & 1) ? (x >> 16) : (x & 0xffffu)) | lo;
                offx = XSW ? off ^ (u32)SRB : off;
            }
            lds_u32x4 *row = (lds_u32x4 *)(uintptr_t)off;
            lds_u32x4 *rowx = (lds_u32x4 *)(uintptr_t)offx;   // odd planes
#pragma unroll
            for (int p = 0; p < GP; p++) {
                const int pl = F::gplane(d, p);
                const u32x4 v = (XSW && (pl & 1)) ? rowx[(pl & ~1) * (SRB / 16)]
                                                  : row[(XSW ? (pl & ~1) : plane_slot<F, DCP>(pl)) * (SRB / 16)];
                t[d][p] = make_uint4(v.x, v.y, v.z, v.w);
            }
        }
    };
    auto consume = [&](int r, const uint4 (&t)[D][GP]) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            u32 ti[D][GP];
#pragma unroll
            for (int d = 0; d < D; d++)
#pragma unroll
                for (int p = 0; p < GP; p++) ti[d][p] = comp4(t[d][p], i);
            F::accumulate(acc[r][i], ti);
        }
    };
    // half a row's gathers (HALF_ROWS fields): D / 2 table rows starting at d = h * D / 2
    constexpr int DH = D / 2 > 0 ? D / 2 : 1;
    auto fetch_half = [&](const u32 *iw, int r, int h, u32 lo, uint4 (&t)[DH][GP]) {
#pragma unroll
        for (int dd = 0; dd < DH; dd++) {
            const int d = h * DH + dd;
            const u32 x = iw[r * IBW + (d >> 1)];
            const u32 off = ((d & 1) ? (x >> 16) : (x & 0xffffu)) | lo;
            lds_u32x4 *row = (lds_u32x4 *)(uintptr_t)off;
            lds_u32x4 *rowx = (lds_u32x4 *)(uintptr_t)(XSW ? off ^ (u32)SRB : off);   // odd planes
#pragma unroll
            for (int p = 0; p < GP; p++) {
                const int pl = F::gplane(d, p);
                const u32x4 v = (XSW && (pl & 1)) ? rowx[(pl & ~1) * (SRB / 16)]
                                                  : row[(XSW ? (pl & ~1) : plane_slot<F, DCP>(pl)) * (SRB / 16)];
                t[dd][p] = make_uint4(v.x, v.y, v.z, v.w);
            }
        }
    };
    auto consume_half_impl = [&](auto hc, int r, const uint4 (&t)[DH][GP]) {
        constexpr int H = decltype(hc)::value;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            u32 ti[DH][GP];
#pragma unroll
            for (int dd = 0; dd < DH; dd++)
#pragma unroll
                for (int p = 0; p < GP; p++) ti[dd][p] = comp4(t[dd][p], i);
            if constexpr (F::HALF_ROWS) F::template accumulate_half<H>(acc[r][i], ti);
        }
    };
    auto consume_half0 = [&](int r, const uint4 (&t)[DH][GP]) { consume_half_impl(half_tag<0>{}, r, t); };
    auto consume_half1 = [&](int r, const uint4 (&t)[DH][GP]) { consume_half_impl(half_tag<1>{}, r, t); };

    // software-pipelined: the reads of row r+1 are issued before row r is accumulated
    auto gather = [&](int s) {
        const u32 lo = laneoff | ((s & 1) ? TB1 : 0u);
        const u32 *ib = Ib + (s % 3) * TM * IBW + rs * R * IBW;
        u32 iw[R * IBW];
        if constexpr (R * IBW == 1) {
            iw[0] = ib[0];
        } else if constexpr ((R * IBW) % 4 == 0) {
#pragma unroll
            for (int w = 0; w < R * IBW; w += 4) {
                const uint4 v = *reinterpret_cast<const uint4 *>(ib + w);
                iw[w] = v.x; iw[w + 1] = v.y; iw[w + 2] = v.z; iw[w + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int w = 0; w < R * IBW; w += 2) {
                const uint2 v = *reinterpret_cast<const uint2 *>(ib + w);
                iw[w] = v.x; iw[w + 1] = v.y;
            }
        }
        if constexpr (F::HALF_ROWS) {
            // half rows: the second half of row r is read while the first is added, and the
            // first half of row r+1 while the second is added
            uint4 h0[D / 2][GP], h1[D / 2][GP];
            fetch_half(iw, 0, 0, lo, h0);
#pragma unroll
            for (int r = 0; r < R; r++) {
                fetch_half(iw, r, 1, lo, h1);
                consume_half0(r, h0);
                if (r + 1 < R) fetch_half(iw, r + 1, 0, lo, h0);
                consume_half1(r, h1);
            }
        } else if constexpr (PF3) {
            // three rows of reads in flight: row r+3's are issued before row r is added
            uint4 tq[4][D][GP];
            fetch(iw, 0, lo, tq[0]);
            if (R > 1) fetch(iw, 1, lo, tq[1]);
            if (R > 2) fetch(iw, 2, lo, tq[2]);
#pragma unroll
            for (int r = 0; r < R; r++) {
                if (r + 3 < R) fetch(iw, r + 3, lo, tq[(r + 3) % 4]);
                consume(r, tq[r % 4]);
            }
        } else {
            uint4 ta[D][GP], tb[D][GP];
            fetch(iw, 0, lo, ta);
#pragma unroll
            for (int r = 0; r < R; r += 2) {
                if (r + 1 < R) fetch(iw, r + 1, lo, tb);
                consume(r, ta);
                if (r + 2 < R) fetch(iw, r + 2, lo, ta);
                if (r + 1 < R) consume(r + 1, tb);
            }
        }
    };

    const bool build_first = (tid / 64) < (NT / 128);   // first half of the waves

    // ---- prologue: stage slabs s0 .. s0+2 (B rows) and s0, s0+1 (table offsets), the
    // prefixes of s0 and s0+1, then the table of s0 ----
    uint4 bpre = make_uint4(0u, 0u, 0u, 0u);
    if (s_begin < s_end) {
        store_b(s_begin, load_b(s_begin));
        stage_idx(s_begin);
        if (advance(s_begin + 1)) prefetch_a();
        if (s_begin + 1 < s_end) {
            store_b(s_begin + 1, load_b(s_begin + 1));
            stage_idx(s_begin + 1);
            if (advance(s_begin + 2)) prefetch_a();
        }
        if (s_begin + 2 < s_end) store_b(s_begin + 2, load_b(s_begin + 2));
        if (s_begin + 3 < s_end && b_active) bpre = load_b(s_begin + 3);
        __syncthreads();
        prefix(s_begin);
        if (s_begin + 1 < s_end) prefix(s_begin + 1);
        __syncthreads();
        build(s_begin);
        __syncthreads();
    }

    for (int s = s_begin; s < s_end; s++) {
        // Iteration s stages the B rows of slab s+3 and the table offsets of slab s+2,
        // computes the chunk prefixes of slab s+2, builds the table of slab s+1 and
        // gathers slab s.  Every register filled by an earlier load is consumed before
        // this iteration's loads are issued (B rows of slab s+4, then the next A word);
        // those are used at least an iteration later, so no wait in the loop covers a load
        // of the same iteration.
        bool moved = false;
        if (s + 3 < s_end) store_b(s + 3, bpre);
        if (s + 2 < s_end) {
            stage_idx(s + 2);
            moved = advance(s + 3);
        }
        if (s + 4 < s_end && b_active) bpre = load_b(s + 4);
        if (moved) prefetch_a();
        // The two waves sharing a SIMD (w and w + NT/256) run the independent build and
        // gather phases in opposite orders, so one wave's VALU-heavy gathers fill the other
        // wave's waits on the table build's LDS round trips.
#pragma unroll 1
        for (int phase = 0; phase < 2; phase++) {
            if ((phase == 0) == build_first) {
                if (s + 2 < s_end) prefix(s + 2);
                if (s + 1 < s_end) build(s + 1);
            } else {
                gather(s);
            }
        }
        __syncthreads();
    }

    // ---- store: finish (resolve, canonicalise), zero the pad columns ----
    const int w = colw0 + cg * 4;
    if (w < a.Wn) {
        u32 msk[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int v = a.n - (w + i) * 32;
            msk[i] = v >= 32 ? 0xffffffffu : (v <= 0 ? 0u : ((1u << v) - 1u));
        }
        u32 *out = a.out + (size_t)bz * a.split_stride;
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int row = row0 + rs + r * RS;
            if (row < a.m) {
                u32 o[4][P];
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    if constexpr (GSW) F::exchange_fix(acc[r][i], neg_row ? 0xffffffffu : 0u);
                    F::finish(acc[r][i], o[i]);
                    if constexpr (DCP) F::front_fix(o[i], dbl_row ? 0xffffffffu : 0u);
                }
#pragma unroll
                for (int p = 0; p < P; p++)
                    *reinterpret_cast<uint4 *>(out + ((size_t)row * P + p) * a.Wn + w) =
                        make_uint4(o[0][p] & msk[0], o[1][p] & msk[1], o[2][p] & msk[2], o[3][p] & msk[3]);
            }
        }
    }
}

// One tile of the product: column tile bx, row tile by (R * NT / (TWD / 4) rows), slab
// slice bz.
template <int Q, int TWD, int REP, int R, int NT>
__device__ __forceinline__ void m4rm_tile(const MMArgs &a, int bx, int by, int bz) {
    m4rm_tile_rows<Q, TWD, REP, R, NT>(a, bx * TWD, by * (NT / (TWD / 4) * R), bz);
}

// The same tile where the product's edges may cut it (the items of a batch, whose small
// products leave much of a tile empty).
//   Rows: the tile body runs at the fewest rows per lane (R, R / 2, ..., down to 1, F_9: 2)
//   that cover the tile's rows.  Lane row r is tile row rs + r * RS for row slot rs, so R'
//   rows per lane cover the first R' * RS rows.
//   Columns: a tile holding at most half its TWD words runs as a tile of TWD / 2 words with
//   twice the copies per super-row (the same table bytes and LDS) and twice the row slots,
//   so R / 2 rows per lane cover its rows.
// Each choice is the same for the whole workgroup, and every variant is a straight-line copy
// of the tile body of its own.  (The single-product kernels keep one variant: with the others
// compiled in beside it, the F_5 8192^3 product ran 3% slower with the same instructions in
// its slab loop.)
constexpr int fit_rows_min(int q) { return q == 9 ? 2 : 1; }   // F_9 at one row: more VGPRs

template <int Q, int TWD, int REP, int R, int NT>
__device__ __forceinline__ void m4rm_tile_fit_rows(const MMArgs &a, int colw0, int row0, int bz, int rows) {
    constexpr int RS = NT / (TWD / 4);
    if constexpr (R > fit_rows_min(Q)) {
        if (rows <= RS * (R / 2)) {
            m4rm_tile_fit_rows<Q, TWD, REP, R / 2, NT>(a, colw0, row0, bz, rows);
            return;
        }
    }
    m4rm_tile_rows<Q, TWD, REP, R, NT, true>(a, colw0, row0, bz);
}

template <int Q, int TWD, int R> constexpr bool fit_narrow_tile() {
    return TWD >= 8 && R >= 2 * fit_rows_min(Q);
}

template <int Q, int TWD, int REP, int R, int NT>
__device__ __forceinline__ void m4rm_tile_fit(const MMArgs &a, int bx, int by, int bz) {
    constexpr int RS = NT / (TWD / 4);           // row slots: rows per lane row
    const int colw0 = bx * TWD, row0 = by * (RS * R);
    const int rows = __builtin_amdgcn_readfirstlane(min(RS * R, a.m - row0));
    if constexpr (fit_narrow_tile<Q, TWD, R>()) {
        const int words = __builtin_amdgcn_readfirstlane(min(TWD, a.Wn - colw0));
        if (words <= TWD / 2) {
            m4rm_tile_fit_rows<Q, TWD / 2, REP * 2, R / 2, NT>(a, colw0, row0, bz, rows);
            return;
        }
    }
    m4rm_tile_fit_rows<Q, TWD, REP, R, NT>(a, colw0, row0, bz, rows);
}

}  // namespace gfq
