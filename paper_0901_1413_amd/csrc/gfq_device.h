// gfq_device.h -- per-field traits used by the kernels.
//
// Three representations meet in the product kernel:
//   storage     the packed format of the C ABI (Section 4 encodings), P planes;
//   table       how table entries (sums of rows of B) are held in LDS, P planes;
//   accumulator how a lane keeps its running row of C, PA planes (a binary residue
//               modulo 3 for F_3 and two for F_9, a carry-save pair of residues modulo 7
//               for F_7, a three-plane carry-save value modulo 5 for F_5, see gfq_field.h).
// SPLIT_PREFIX: table chunk prefixes are summed one slab ahead by a quarter of the threads
// (fields whose table addition is long) rather than by every build thread for itself.
// EXCHANGE_READS: a lane that reads every table entry with planes 2j and 2j + 1 exchanged (and,
// where EXCHANGE_SLOTS, with its two gathers' table rows exchanged) accumulates a fixed
// invertible linear image of its row of C: -C for F_3 and F_9 (exchanging the planes negates
// an entry), x^2 C^2 for GF(4).  Such fields define exchange_fix, which maps an accumulator
// back where a lane mask is set.
// FRONT_SLOT (three-plane fields F_7, GF(8)): at 128-byte super-rows a table entry gets a
// fourth slot in front, front(t), with plane p of t at slot front_slot(p), such that reading
// slots 0-2 in the order planes are read from slots 1-3 yields lam * t for a fixed nonzero
// lam (F_7: 2t, GF(8): x t).  The second row of every read pass reads that way and
// accumulates lam C; front_fix maps its finished row back where a lane mask is set.
// HALF_BUILD_ROWS: from this many rows per lane on, the gathers of a slab outweigh its
// table build enough that only half of the waves (one per SIMD) build the table, each
// walking twice as far, with half the chunk prefixes (measured faster for every field at
// the rows per lane listed; F_7, whose eleven-instruction table additions face four rows per
// lane of eighteen-instruction accumulates, measured slower: its building waves became the
// tail of every slab).
// Every trait works on one 32-bit word per plane (32 columns); the kernels apply it to
// the four words of a 128-bit LDS read.
#pragma once
#include <hip/hip_runtime.h>

#define GFQ_HD __host__ __device__ __forceinline__
#include "gfq_field.h"
#include "gfq_internal.h"

namespace gfq {

template <int Q> struct FT;

// F_3 (Section 4.1).  Basis {1, -1}: phi_0 = [a = 1] = x0 ^ x1, phi_1 = [a = -1] = x1.
// Table entries and the accumulator are binary residues mod 3 (b0 + 2 b1, 3 meaning 0); per
// slab the accumulator receives T[phi_0] and -T[phi_1], two four-instruction residue
// additions.  Exchanging the two planes of a residue multiplies it by 2 = -1 (mod 3)
// (EXCHANGE_READS): a lane that reads every table entry with its planes exchanged
// accumulates -C, and exchange_fix turns it back.
template <> struct FT<3> {
    static constexpr int P = 2, PT = 2, D = 2, GP = 2, PA = 2;
    static constexpr bool SPLIT_PREFIX = false, HALF_ROWS = false, EXCHANGE_READS = true;
    static constexpr bool EXCHANGE_SLOTS = false;
    static constexpr int HALF_BUILD_ROWS = 8;
    static constexpr int gplane(int, int p) { return p; }
    __device__ static void phis(const u32 *x, u32 *f) { f[0] = x[0] ^ x[1]; f[1] = x[1]; }
    __device__ static void to_table(const u32 *x, u32 *t) { f3_to_bin(x[0], x[1], t); }
    __device__ static void tadd(const u32 *a, const u32 *b, u32 *r) { f3b_add(a, b, r); }
    __device__ static void tsub(const u32 *a, const u32 *b, u32 *r) { f3b_sub(a, b, r); }
    __device__ static void acc_init(u32 *c, int) { for (int i = 0; i < PA; i++) c[i] = 0u; }
    __device__ static void accumulate(u32 *c, const u32 (*t)[P]) {
        u32 x[2];
        f3b_add(c, t[0], x);
        f3b_sub(x, t[1], c);
    }
    // the accumulator negated where gm is all ones (its planes exchanged), kept elsewhere
    __device__ static void exchange_fix(u32 *c, u32 gm) {
        const u32 c0 = c[0];
        c[0] = lut3<0xCA>(gm, c[1], c0);          // gm ? c1 : c0
        c[1] = lut3<0xCA>(gm, c0, c[1]);
    }
    __device__ static void finish(const u32 *c, u32 *out) { f3_from_bin(c, &out[0], &out[1]); }
    __device__ static void sadd(const u32 *a, const u32 *b, u32 *r) {
        F3v z = f3_add(F3v{a[0], a[1]}, F3v{b[0], b[1]});
        r[0] = z.u; r[1] = z.s;
    }
    __device__ static void sneg(const u32 *a, u32 *r) { F3v z = f3_neg(F3v{a[0], a[1]}); r[0] = z.u; r[1] = z.s; }
    __device__ static void scanon(u32 *) {}
};

// F_7 (Section 4.2).  Basis {1, 2, 4}, phi_d = plane d.  Doubling modulo 7 rotates the
// planes, so alpha_d T[phi_d] costs nothing; the accumulator is a carry-save pair mod 7.
template <> struct FT<7> {
    static constexpr int P = 3, PT = 3, D = 3, GP = 3, PA = 6;
    static constexpr bool SPLIT_PREFIX = true, HALF_ROWS = false, EXCHANGE_READS = false;
    // slots (t2, t0, t1, t2): slots 0-2 hold (t2, t0, t1) = 2t; the row of 2C is multiplied
    // by 4, the rotation (c0, c1, c2) -> (c1, c2, c0)
    static constexpr bool FRONT_SLOT = true;
    static constexpr int front_slot(int p) { return p + 1; }
    __device__ static u32 front(const u32 *t) { return t[2]; }
    __device__ static void front_fix(u32 *o, u32 gm) {
        const u32 o0 = o[0];
        o[0] = lut3<0xCA>(gm, o[1], o0);          // gm ? o1 : o0
        o[1] = lut3<0xCA>(gm, o[2], o[1]);
        o[2] = lut3<0xCA>(gm, o0, o[2]);
    }
    static constexpr int HALF_BUILD_ROWS = 1 << 30;
    static constexpr int gplane(int, int p) { return p; }
    __device__ static void phis(const u32 *x, u32 *f) { f[0] = x[0]; f[1] = x[1]; f[2] = x[2]; }
    __device__ static void to_table(const u32 *x, u32 *t) { t[0] = x[0]; t[1] = x[1]; t[2] = x[2]; }
    __device__ static void tadd(const u32 *a, const u32 *b, u32 *r) {
        P3v z = f7_add(P3v{a[0], a[1], a[2]}, P3v{b[0], b[1], b[2]});
        r[0] = z.b0; r[1] = z.b1; r[2] = z.b2;
    }
    __device__ static void tsub(const u32 *a, const u32 *b, u32 *r) {
        P3v z = f7_sub(P3v{a[0], a[1], a[2]}, P3v{b[0], b[1], b[2]});
        r[0] = z.b0; r[1] = z.b1; r[2] = z.b2;
    }
    __device__ static void acc_init(u32 *c, int) { for (int i = 0; i < PA; i++) c[i] = 0u; }
    __device__ static void accumulate(u32 *c, const u32 (*t)[P]) {
        u32 *S = c, *K = c + 3;
        csa_step<3>(S, K, t[0]);
        const u32 x1[3] = {t[1][2], t[1][0], t[1][1]};   // 2 t
        csa_step<3>(S, K, x1);
        const u32 x2[3] = {t[2][1], t[2][2], t[2][0]};   // 4 t
        csa_step<3>(S, K, x2);
    }
    __device__ static void finish(const u32 *c, u32 *out) {
        P3v z = f7_reduce(f7_add(P3v{c[0], c[1], c[2]}, P3v{c[3], c[4], c[5]}));
        out[0] = z.b0; out[1] = z.b1; out[2] = z.b2;
    }
    __device__ static void sadd(const u32 *a, const u32 *b, u32 *r) { tadd(a, b, r); }
    __device__ static void sneg(const u32 *a, u32 *r) { r[0] = ~a[0]; r[1] = ~a[1]; r[2] = ~a[2]; }
    __device__ static void scanon(u32 *v) {
        P3v z = f7_reduce(P3v{v[0], v[1], v[2]});
        v[0] = z.b0; v[1] = z.b1; v[2] = z.b2;
    }
};

// F_5 (Section 4.2).  Basis {1, 2, 4}, phi_d = plane d; table entries are 3-bit
// representatives (f5_add8 / f5_sub8, eight instructions each).  The accumulator is a carry-save value modulo 5
// in three planes (f5_nc_slab): a slab's three scaled rows enter it together, and its value
// is already canonical at the end.
template <> struct FT<5> {
    static constexpr int P = 3, PT = 3, D = 3, GP = 3, PA = 3;
    static constexpr bool SPLIT_PREFIX = true, HALF_ROWS = false, EXCHANGE_READS = false;
    static constexpr int HALF_BUILD_ROWS = 8;
    static constexpr int gplane(int, int p) { return p; }
    __device__ static void phis(const u32 *x, u32 *f) { f[0] = x[0]; f[1] = x[1]; f[2] = x[2]; }
    __device__ static void to_table(const u32 *x, u32 *t) { t[0] = x[0]; t[1] = x[1]; t[2] = x[2]; }
    __device__ static void tadd(const u32 *a, const u32 *b, u32 *r) { f5_add8(a, b, r); }
    __device__ static void tsub(const u32 *a, const u32 *b, u32 *r) { f5_sub8(a, b, r); }
    // the accumulator starts at -2 x slabs (mod 5): each slab step adds 2 beyond its rows
    __device__ static void acc_init(u32 *c, int slabs) { f5_nc_init(c, slabs); }
    __device__ static void accumulate(u32 *c, const u32 (*t)[P]) { f5_nc_slab(c, t[0], t[1], t[2]); }
    __device__ static void finish(const u32 *c, u32 *out) {
        P3v z = f5_nc_value(c);
        out[0] = z.b0; out[1] = z.b1; out[2] = z.b2;
    }
    __device__ static void sadd(const u32 *a, const u32 *b, u32 *r) { tadd(a, b, r); }
    __device__ static void sneg(const u32 *a, u32 *r) {
        P3v z = f5_neg(P3v{a[0], a[1], a[2]});
        r[0] = z.b0; r[1] = z.b1; r[2] = z.b2;
    }
    __device__ static void scanon(u32 *v) {
        P3v z = f5_reduce(P3v{v[0], v[1], v[2]});
        v[0] = z.b0; v[1] = z.b1; v[2] = z.b2;
    }
};

// GF(4) (Section 4.3).  Basis {1, x}, phi_d = c_d.  Per slab the row receives
// T[phi_0] + x T[phi_1]; with x (c0 + c1 x) = c1 + (c0 + c1) x that is two XOR planes.
// Exchanging the planes of an entry t gives c1 + c0 x = x t^2 (squaring is additive here and
// x^3 = 1).  A lane that reads both table rows with planes exchanged and with the two rows
// exchanged (EXCHANGE_SLOTS: T[phi_1] into the slot of T[phi_0] and back) adds
// x T1^2 + x x T0^2 = x^2 (T0 + x T1)^2 per slab, so it accumulates L(C) with L(a) = x^2 a^2;
// L is additive and its own inverse (x^6 = 1, a^4 = a), and L(c0 + c1 x) = c0 + (c0 + c1) x.
template <> struct FT<4> {
    static constexpr int P = 2, PT = 2, D = 2, GP = 2, PA = 2;
    static constexpr bool SPLIT_PREFIX = false, HALF_ROWS = false, EXCHANGE_READS = true;
    static constexpr bool EXCHANGE_SLOTS = true;
    static constexpr int HALF_BUILD_ROWS = 8;
    static constexpr int gplane(int, int p) { return p; }
    __device__ static void phis(const u32 *x, u32 *f) { f[0] = x[0]; f[1] = x[1]; }
    __device__ static void to_table(const u32 *x, u32 *t) { t[0] = x[0]; t[1] = x[1]; }
    __device__ static void tadd(const u32 *a, const u32 *b, u32 *r) { r[0] = a[0] ^ b[0]; r[1] = a[1] ^ b[1]; }
    __device__ static void tsub(const u32 *a, const u32 *b, u32 *r) { tadd(a, b, r); }
    __device__ static void acc_init(u32 *c, int) { c[0] = c[1] = 0u; }
    __device__ static void accumulate(u32 *c, const u32 (*t)[P]) {
        c[0] = xor3(c[0], t[0][0], t[1][1]);
        c[1] = xor3(c[1], t[0][1], t[1][0]) ^ t[1][1];
    }
    // L applied where gm is all ones
    __device__ static void exchange_fix(u32 *c, u32 gm) { c[1] ^= c[0] & gm; }
    __device__ static void finish(const u32 *c, u32 *out) { out[0] = c[0]; out[1] = c[1]; }
    __device__ static void sadd(const u32 *a, const u32 *b, u32 *r) { tadd(a, b, r); }
    __device__ static void sneg(const u32 *a, u32 *r) { r[0] = a[0]; r[1] = a[1]; }
    __device__ static void scanon(u32 *) {}
};

// GF(4) by matrix-level Karatsuba over F_2 (Section 4.3): with A = A0 + x A1 and
// B = B0 + x B1 (coefficient planes), C0 = A0 B0 + A1 B1 and C1 = (A0 + A1)(B0 + B1) + A0 B0,
// three F_2 products.  Each table entry holds the three F_2 tables of the slab (planes
// B0, B1, B0 + B1); a row gathers one plane of three entries: T0[a0], T1[a1], T2[a0 + a1].
// Same packed operands and product as FT<4>; selected by the configuration.
template <> struct FT<GF4_KARATSUBA> {
    static constexpr int P = 2, PT = 3, D = 3, GP = 1, PA = 2;
    static constexpr bool SPLIT_PREFIX = false, HALF_ROWS = false, EXCHANGE_READS = false;
    static constexpr int HALF_BUILD_ROWS = 8;
    static constexpr int gplane(int d, int) { return d; }
    __device__ static void phis(const u32 *x, u32 *f) { f[0] = x[0]; f[1] = x[1]; f[2] = x[0] ^ x[1]; }
    __device__ static void to_table(const u32 *x, u32 *t) { t[0] = x[0]; t[1] = x[1]; t[2] = x[0] ^ x[1]; }
    __device__ static void tadd(const u32 *a, const u32 *b, u32 *r) {
        r[0] = a[0] ^ b[0]; r[1] = a[1] ^ b[1]; r[2] = a[2] ^ b[2];
    }
    __device__ static void tsub(const u32 *a, const u32 *b, u32 *r) { tadd(a, b, r); }
    __device__ static void acc_init(u32 *c, int) { c[0] = c[1] = 0u; }
    __device__ static void accumulate(u32 *c, const u32 (*t)[GP]) {
        c[0] = xor3(c[0], t[0][0], t[1][0]);              // A0 B0 + A1 B1
        c[1] = xor3(c[1], t[2][0], t[0][0]);              // (A0 + A1)(B0 + B1) + A0 B0
    }
    __device__ static void finish(const u32 *c, u32 *out) { out[0] = c[0]; out[1] = c[1]; }
    __device__ static void sadd(const u32 *a, const u32 *b, u32 *r) { r[0] = a[0] ^ b[0]; r[1] = a[1] ^ b[1]; }
    __device__ static void scanon(u32 *) {}
};

// GF(8) (Section 4.3, the power basis of the extension times the basis {1} of F_2).
// Basis {1, x, x^2}, phi_d = c_d.  Per slab the row receives T[phi_0] + x T[phi_1] +
// x^2 T[phi_2] (g8_acc, six operations for three planes).
template <> struct FT<8> {
    static constexpr int P = 3, PT = 3, D = 3, GP = 3, PA = 3;
    static constexpr bool SPLIT_PREFIX = false, HALF_ROWS = false, EXCHANGE_READS = false;
    // slots (t0 + t2, t1, t2, t0): read as planes 0, 1, 2 from slots 2, 0, 1 they give
    // (t2, t0 + t2, t1) = x t (x^3 = x + 1); the row of x C is multiplied by x^6 = x^2 + 1,
    // (c0, c1, c2) -> (c0 + c1, c2, c0)
    static constexpr bool FRONT_SLOT = true;
    static constexpr int front_slot(int p) { return p == 0 ? 3 : p; }
    __device__ static u32 front(const u32 *t) { return t[0] ^ t[2]; }
    __device__ static void front_fix(u32 *o, u32 gm) {
        const u32 o0 = o[0];
        o[0] = o0 ^ (o[1] & gm);
        o[1] = lut3<0xCA>(gm, o[2], o[1]);        // gm ? o2 : o1
        o[2] = lut3<0xCA>(gm, o0, o[2]);
    }
    static constexpr int HALF_BUILD_ROWS = 8;
    static constexpr int gplane(int, int p) { return p; }
    __device__ static void phis(const u32 *x, u32 *f) { f[0] = x[0]; f[1] = x[1]; f[2] = x[2]; }
    __device__ static void to_table(const u32 *x, u32 *t) { t[0] = x[0]; t[1] = x[1]; t[2] = x[2]; }
    __device__ static void tadd(const u32 *a, const u32 *b, u32 *r) {
        r[0] = a[0] ^ b[0]; r[1] = a[1] ^ b[1]; r[2] = a[2] ^ b[2];
    }
    __device__ static void tsub(const u32 *a, const u32 *b, u32 *r) { tadd(a, b, r); }
    __device__ static void acc_init(u32 *c, int) { c[0] = c[1] = c[2] = 0u; }
    __device__ static void accumulate(u32 *c, const u32 (*t)[P]) { g8_acc(c, t[0], t[1], t[2]); }
    __device__ static void finish(const u32 *c, u32 *out) { out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; }
    __device__ static void sadd(const u32 *a, const u32 *b, u32 *r) { tadd(a, b, r); }
    __device__ static void sneg(const u32 *a, u32 *r) { r[0] = a[0]; r[1] = a[1]; r[2] = a[2]; }
    __device__ static void scanon(u32 *) {}
};

// F_9 = F_3[i]/(i^2 + 1) (Section 4.3: the power basis {1, i} of the extension times the
// basis {1, -1} of F_3 gives the additive basis {1, -1, i, -i}).  Storage: the F_3 code of
// a0, then of a1 (four planes); phi = [a0 = 1], [a0 = -1], [a1 = 1], [a1 = -1].  Table
// entries and the accumulator are pairs of binary residues mod 3 (real, imaginary).  With
// i (x + y i) = -y + x i the slab adds T0 - T1 + i T2 - i T3, i.e. real += T0.re - T1.re -
// T2.im + T3.im and imaginary += T0.im - T1.im + T2.re - T3.re: eight four-instruction residue
// additions (as F_3), four accumulator planes, so eight rows per lane fit.
// Exchanging planes 2j and 2j + 1 negates both residues of an entry (EXCHANGE_READS), and the
// residue additions on negated operands give the negated sum, so a lane that reads every entry
// exchanged ends with the negated accumulator.
template <> struct FT<9> {
    static constexpr int P = 4, PT = 4, D = 4, GP = 4, PA = 4;
    // HALF_ROWS: a row's gathers are consumed in two halves (accumulate_half), so only half a
    // row of 128-bit reads is in flight at a time
    static constexpr bool SPLIT_PREFIX = false, HALF_ROWS = true, EXCHANGE_READS = true;
    static constexpr bool EXCHANGE_SLOTS = false;
    static constexpr int HALF_BUILD_ROWS = 4;
    static constexpr int gplane(int, int p) { return p; }
    __device__ static void phis(const u32 *x, u32 *f) { f[0] = x[0] ^ x[1]; f[1] = x[1]; f[2] = x[2] ^ x[3]; f[3] = x[3]; }
    __device__ static void to_table(const u32 *x, u32 *t) { f3_to_bin(x[0], x[1], t); f3_to_bin(x[2], x[3], t + 2); }
    __device__ static void tadd(const u32 *a, const u32 *b, u32 *r) { f3b_add(a, b, r); f3b_add(a + 2, b + 2, r + 2); }
    __device__ static void tsub(const u32 *a, const u32 *b, u32 *r) { f3b_sub(a, b, r); f3b_sub(a + 2, b + 2, r + 2); }
    __device__ static void acc_init(u32 *c, int) { for (int i = 0; i < PA; i++) c[i] = 0u; }
    __device__ static void accumulate(u32 *c, const u32 (*t)[P]) {
        accumulate_half<0>(c, t);
        accumulate_half<1>(c, t + 2);
    }
    // the same additions in two halves: H = 0 takes T[phi_0] - T[phi_1] (t[0], t[1]), H = 1
    // takes i T[phi_2] - i T[phi_3] (t[0], t[1] holding phi_2, phi_3)
    template <int H> __device__ static void accumulate_half(u32 *c, const u32 (*t)[P]) {
        u32 x[2];
        if (H == 0) {
            f3b_add(c, t[0], x);                   // real += T0.re - T1.re
            f3b_sub(x, t[1], c);
            f3b_add(c + 2, t[0] + 2, x);           // imaginary += T0.im - T1.im
            f3b_sub(x, t[1] + 2, c + 2);
        } else {
            f3b_sub(c, t[0] + 2, x);               // real += -T2.im + T3.im
            f3b_add(x, t[1] + 2, c);
            f3b_add(c + 2, t[0], x);               // imaginary += T2.re - T3.re
            f3b_sub(x, t[1], c + 2);
        }
    }
    // the accumulator negated where gm is all ones (the planes of each residue exchanged)
    __device__ static void exchange_fix(u32 *c, u32 gm) {
#pragma unroll
        for (int j = 0; j < PA; j += 2) {
            const u32 c0 = c[j];
            c[j] = lut3<0xCA>(gm, c[j + 1], c0);      // gm ? c1 : c0
            c[j + 1] = lut3<0xCA>(gm, c0, c[j + 1]);
        }
    }
    __device__ static void finish(const u32 *c, u32 *out) {
        f3_from_bin(c, &out[0], &out[1]);
        f3_from_bin(c + 2, &out[2], &out[3]);
    }
    __device__ static void sadd(const u32 *a, const u32 *b, u32 *r) {
        F3v re = f3_add(F3v{a[0], a[1]}, F3v{b[0], b[1]});
        F3v im = f3_add(F3v{a[2], a[3]}, F3v{b[2], b[3]});
        r[0] = re.u; r[1] = re.s; r[2] = im.u; r[3] = im.s;
    }
    __device__ static void sneg(const u32 *a, u32 *r) {
        F3v re = f3_neg(F3v{a[0], a[1]}), im = f3_neg(F3v{a[2], a[3]});
        r[0] = re.u; r[1] = re.s; r[2] = im.u; r[3] = im.s;
    }
    __device__ static void scanon(u32 *) {}
};

// GF(8) by the trinomial formula of Section 4.3, at matrix level over F_2: with A = A0 +
// x A1 + x^2 A2 and B alike, the six F_2 products P_ii = Ai Bi and P_ij = (Ai + Aj)(Bi + Bj)
// give the coefficients of A B before reduction; modulo x^3 + x + 1,
//   C0 = P00 + P11 + P12 + P22,  C1 = P00 + P01 + P12,  C2 = P00 + P02 + P11.
// A table entry holds the six F_2 tables of the slab (planes B0, B1, B2, B0 + B1,
// B0 + B2, B1 + B2); a row gathers one plane of six entries.  Same operands and product as
// FT<8>; selected by the configuration.
template <> struct FT<GF8_TRINOMIAL> {
    static constexpr int P = 3, PT = 6, D = 6, GP = 1, PA = 3;
    static constexpr bool SPLIT_PREFIX = false, HALF_ROWS = false, EXCHANGE_READS = false;
    static constexpr int HALF_BUILD_ROWS = 8;
    static constexpr int gplane(int d, int) { return d; }
    __device__ static void phis(const u32 *x, u32 *f) {
        f[0] = x[0]; f[1] = x[1]; f[2] = x[2]; f[3] = x[0] ^ x[1]; f[4] = x[0] ^ x[2]; f[5] = x[1] ^ x[2];
    }
    __device__ static void to_table(const u32 *x, u32 *t) { phis(x, t); }
    __device__ static void tadd(const u32 *a, const u32 *b, u32 *r) {
        for (int i = 0; i < PT; i++) r[i] = a[i] ^ b[i];
    }
    __device__ static void tsub(const u32 *a, const u32 *b, u32 *r) { tadd(a, b, r); }
    __device__ static void acc_init(u32 *c, int) { c[0] = c[1] = c[2] = 0u; }
    // t[d][0]: P00, P11, P22, P01, P02, P12
    __device__ static void accumulate(u32 *c, const u32 (*t)[GP]) {
        const u32 u = t[0][0] ^ t[5][0], v = t[1][0] ^ t[2][0], w = t[0][0] ^ t[1][0];
        c[0] = xor3(c[0], u, v);          // P00 + P12 + P11 + P22
        c[1] = xor3(c[1], u, t[3][0]);    // P00 + P12 + P01
        c[2] = xor3(c[2], w, t[4][0]);    // P00 + P11 + P02
    }
    __device__ static void finish(const u32 *c, u32 *out) { out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; }
};

// F_9 by Karatsuba at matrix level over F_3 (Section 4.3): with A = A0 + i A1 and B = B0 +
// i B1, A B = (P00 - P11) + i (Pss - P00 - P11) for the three F_3 products P00 = A0 B0,
// P11 = A1 B1, Pss = (A0 + A1)(B0 + B1).  A table entry holds the slab's three F_3 tables
// (rows B0, B1, B0 + B1 as binary residues mod 3, two planes each); a row gathers, per
// product, the entries of its coefficient's [= 1] and [= -1] bits (two planes each) into
// that product's own carry-save pair; the products are combined once, at the end.  Same
// operands and product as FT<9>; selected by the configuration.
template <> struct FT<F9_KARATSUBA> {
    static constexpr int P = 4, PT = 6, D = 6, GP = 2, PA = 12;
    static constexpr bool SPLIT_PREFIX = false, HALF_ROWS = false, EXCHANGE_READS = false;
    static constexpr int HALF_BUILD_ROWS = 1 << 30;
    static constexpr int gplane(int d, int p) { return (d >> 1) * 2 + p; }
    __device__ static void phis(const u32 *x, u32 *f) {
        const F3v s = f3_add(F3v{x[0], x[1]}, F3v{x[2], x[3]});   // a0 + a1
        f[0] = x[0] ^ x[1]; f[1] = x[1];
        f[2] = x[2] ^ x[3]; f[3] = x[3];
        f[4] = s.u ^ s.s; f[5] = s.s;
    }
    __device__ static void to_table(const u32 *x, u32 *t) {
        f3_to_bin(x[0], x[1], t);
        f3_to_bin(x[2], x[3], t + 2);
        f3b_add(t, t + 2, t + 4);
    }
    __device__ static void tadd(const u32 *a, const u32 *b, u32 *r) {
        f3b_add(a, b, r); f3b_add(a + 2, b + 2, r + 2); f3b_add(a + 4, b + 4, r + 4);
    }
    __device__ static void tsub(const u32 *a, const u32 *b, u32 *r) {
        f3b_sub(a, b, r); f3b_sub(a + 2, b + 2, r + 2); f3b_sub(a + 4, b + 4, r + 4);
    }
    __device__ static void acc_init(u32 *c, int) { for (int i = 0; i < PA; i++) c[i] = 0u; }
    __device__ static void accumulate(u32 *c, const u32 (*t)[GP]) {
#pragma unroll
        for (int j = 0; j < 3; j++) {                     // P00, P11, Pss
            csa_step<2>(c + 4 * j, c + 4 * j + 2, t[2 * j]);
            csa_step_neg<2>(c + 4 * j, c + 4 * j + 2, t[2 * j + 1]);
        }
    }
    __device__ static void finish(const u32 *c, u32 *out) {
        u32 p00[2], p11[2], pss[2], re[2], im[2], t[2];
        f3b_add(c, c + 2, p00);
        f3b_add(c + 4, c + 6, p11);
        f3b_add(c + 8, c + 10, pss);
        f3b_sub(p00, p11, re);
        f3b_sub(pss, p00, t);
        f3b_sub(t, p11, im);
        f3_from_bin(re, &out[0], &out[1]);
        f3_from_bin(im, &out[2], &out[3]);
    }
};

}  // namespace gfq
