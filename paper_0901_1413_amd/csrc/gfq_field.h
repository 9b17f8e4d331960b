// gfq_field.h -- bitsliced arithmetic over F_3, F_5, F_7 and GF(4) on 32-bit plane words.
//
// Every function works on one 32-bit word per bit-plane, i.e. on 32 field elements at
// once (paper, Section 3: the bits of one element sit in parallel words), in the element
// encodings of Section 4.  The programs are derived here for gfx950, whose v_bitop3_b32
// computes any Boolean function of three words in one instruction: full adders over
// weight columns, residues of 2^b - 1 and 2^b + 1, and searched three-input programs.
// Where the paper prints a formula for the same operation, the comment says how the two
// relate.
//
// The header is plain C++ so that the host-side truth-table checks can include it; the
// GPU library includes it with GFQ_HD defined as __host__ __device__.
#pragma once
#include <stdint.h>

#ifndef GFQ_HD
#define GFQ_HD inline
#endif

namespace gfq {

typedef uint32_t u32;

// Three-input primitives.  In the device pass each is one v_bitop3_b32 (truth table over
// operands (a, b, c) weighted 0xF0, 0xCC, 0xAA); the host pass spells them out so the
// truth-table checks run the same formulas.  The "n" forms complement their third operand.
#if defined(__HIP_DEVICE_COMPILE__)
GFQ_HD u32 xor3(u32 a, u32 b, u32 c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96); }
GFQ_HD u32 maj3(u32 a, u32 b, u32 c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8); }
GFQ_HD u32 xor3n(u32 a, u32 b, u32 c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0x69); }
GFQ_HD u32 maj3n(u32 a, u32 b, u32 c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0xD4); }
#else
GFQ_HD u32 xor3(u32 a, u32 b, u32 c) { return a ^ b ^ c; }
GFQ_HD u32 maj3(u32 a, u32 b, u32 c) { return (a & b) | (c & (a | b)); }
GFQ_HD u32 xor3n(u32 a, u32 b, u32 c) { return a ^ b ^ ~c; }
GFQ_HD u32 maj3n(u32 a, u32 b, u32 c) { return (a & b) | (~c & (a | b)); }
#endif

// Any three-input function as one instruction: bit (4a + 2b + c) of IMM is the result for
// operand bits (a, b, c), the same truth-table order as above.
template <int IMM> GFQ_HD u32 lut3(u32 a, u32 b, u32 c) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, IMM);
#else
    u32 r = 0;
    for (int v = 0; v < 8; v++)
        if ((IMM >> v) & 1) r |= ((v & 4) ? a : ~a) & ((v & 2) ? b : ~b) & ((v & 1) ? c : ~c);
    return r;
#endif
}
// The table of the same function with the operands selected by mask m (4: a, 2: b, 1: c)
// complemented.
constexpr int lut3_flip(int imm, int m) {
    int r = 0;
    for (int v = 0; v < 8; v++)
        if ((imm >> (v ^ m)) & 1) r |= 1 << v;
    return r;
}

// ---------------------------------------------------------------------------------------
// F_3 (Section 4.1).  Planes (x0, x1): x0 marks a unit, x1 the sign; 0 = 00, 1 = 10,
// -1 = 11.  The code 01 never occurs.
// ---------------------------------------------------------------------------------------
struct F3v { u32 u, s; };

// Negation, 1 operation: (a0, a0 ^ a1).
GFQ_HD F3v f3_neg(F3v a) { F3v r; r.u = a.u; r.s = a.u ^ a.s; return r; }

// ---------------------------------------------------------------------------------------
// F_7 and F_5 (Section 4.2).  Three planes b0, b1, b2 holding the binary digits of a
// representative in [0, 8); representatives are not unique (F_7: 7 = 0; F_5: 5, 6, 7 =
// 0, 1, 2).  Additive basis {1, 2, 4}; phi_d is plane d of any representative.
// ---------------------------------------------------------------------------------------
struct P3v { u32 b0, b1, b2; };
struct P4v { u32 b0, b1, b2, b3; };

// Grade-school addition of two 3-bit numbers into a 4-bit sum (two full adders and a
// half adder).
GFQ_HD P4v add3x3(P3v a, P3v b) {
    P4v s;
    u32 c1 = a.b0 & b.b0;
    s.b0 = a.b0 ^ b.b0;
    s.b1 = xor3(a.b1, b.b1, c1);
    u32 c2 = maj3(a.b1, b.b1, c1);
    s.b2 = xor3(a.b2, b.b2, c2);
    s.b3 = maj3(a.b2, b.b2, c2);
    return s;
}

// F_7 addition (17 two-input operations): add, then add the carry back in (8 = 1 mod 7).
// The second addition never carries out: the sum is at most 14, so s0..s3 are never all 1.
// (A carry-lookahead form that adds the end-around carry in one ripple pass takes 8
// three-input instructions instead of 11, but measured slower in the table build, whose
// Gray-code walk is one long dependency chain.)
GFQ_HD P3v f7_add(P3v a, P3v b) {
    P4v s = add3x3(a, b);
    P3v r;
    u32 d1 = s.b0 & s.b3;
    r.b0 = s.b0 ^ s.b3;
    u32 d2 = s.b1 & d1;
    r.b1 = s.b1 ^ d1;
    r.b2 = s.b2 ^ d2;
    return r;
}
// F_7 subtraction: addition of the complement (7 - b = -b mod 7).
GFQ_HD P3v f7_sub(P3v a, P3v b) { return f7_add(a, P3v{~b.b0, ~b.b1, ~b.b2}); }

// F_7 doubling: a rotation of the planes, no operations.
GFQ_HD P3v f7_dbl(P3v a) { P3v r; r.b0 = a.b2; r.b1 = a.b0; r.b2 = a.b1; return r; }

// F_7 negation: complement (7 - a).
GFQ_HD P3v f7_neg(P3v a) { P3v r; r.b0 = ~a.b0; r.b1 = ~a.b1; r.b2 = ~a.b2; return r; }

// F_7 reduction to [0, 7).  The paper prints r_i = a_i ^ (a0 | a1 | a2); the operator must
// be AND: only the representative 7 (all three bits set) changes, to 0.
GFQ_HD P3v f7_reduce(P3v a) {
    u32 g = a.b0 & a.b1 & a.b2;
    P3v r; r.b0 = a.b0 ^ g; r.b1 = a.b1 ^ g; r.b2 = a.b2 ^ g;
    return r;
}

// F_5 reduction to [0, 5).  The printed six-operation program does not preserve the
// residue; this replacement subtracts 5 exactly when the representative is 5, 6 or 7:
// g = [a >= 5] = a2 & (a0 | a1), result a + 3 g mod 8.
GFQ_HD P3v f5_reduce(P3v a) {
    u32 g = a.b2 & (a.b0 | a.b1);
    P3v r;
    r.b0 = a.b0 ^ g;
    r.b1 = a.b1 ^ (g & ~a.b0);
    r.b2 = a.b2 & ~g;
    return r;
}

// ---------------------------------------------------------------------------------------
// GF(4) = F_2[x]/(x^2 + x + 1) with basis {1, x} (Section 4.3): planes (c0, c1) of
// c0 + c1 x.  Addition is XOR per plane; multiplication by x maps c0 + c1 x to
// c1 + (c0 + c1) x because x^2 = x + 1.
// ---------------------------------------------------------------------------------------
struct G4v { u32 c0, c1; };
GFQ_HD G4v g4_add(G4v a, G4v b) { G4v r; r.c0 = a.c0 ^ b.c0; r.c1 = a.c1 ^ b.c1; return r; }
GFQ_HD G4v g4_mulx(G4v a) { G4v r; r.c0 = a.c1; r.c1 = a.c0 ^ a.c1; return r; }

// ---------------------------------------------------------------------------------------
// GF(8) = F_2[x]/(x^3 + x + 1) with the power basis {1, x, x^2} (Section 4.3): planes
// (c0, c1, c2) of c0 + c1 x + c2 x^2.  Addition is XOR per plane.  With x^3 = x + 1,
// multiplying by x maps (c0, c1, c2) to (c2, c0 + c2, c1) and by x^2 to
// (c1, c1 + c2, c0 + c2).
// ---------------------------------------------------------------------------------------
struct G8v { u32 c0, c1, c2; };
GFQ_HD G8v g8_add(G8v a, G8v b) { G8v r; r.c0 = a.c0 ^ b.c0; r.c1 = a.c1 ^ b.c1; r.c2 = a.c2 ^ b.c2; return r; }
GFQ_HD G8v g8_mulx(G8v a) { G8v r; r.c0 = a.c2; r.c1 = a.c0 ^ a.c2; r.c2 = a.c1; return r; }
GFQ_HD G8v g8_mulx2(G8v a) { G8v r; r.c0 = a.c1; r.c1 = a.c1 ^ a.c2; r.c2 = a.c0 ^ a.c2; return r; }
// c += t + x u + x^2 v in six operations: the x^2 v and x u terms meet in plane 0 as u2 + v1,
// which plane 1 reuses.
GFQ_HD void g8_acc(u32 *c, const u32 *t, const u32 *u, const u32 *v) {
    const u32 s = u[2] ^ v[1];
    c[0] = xor3(c[0], t[0], s);
    c[1] = xor3(xor3(c[1], t[1], u[0]), s, v[2]);
    c[2] = xor3(xor3(c[2], t[2], u[1]), v[0], v[2]);
}


// ---------------------------------------------------------------------------------------
// Working representations used inside the product kernel (not storage formats).
//
// Binary residues modulo 2^NB - 1.  A value is an NB-bit integer taken modulo M = 2^NB - 1,
// so the all-ones word also means 0 and a carry out of the top bit re-enters at bit 0
// (2^NB = 1 mod M).  F_3 is worked modulo 3 = 2^2 - 1 and F_7 modulo 7 = 2^3 - 1; F_5 is
// worked modulo 5 = 2^2 + 1, where a carry out of the top bit re-enters at bit 0
// complemented (f5_nc_slab).
//
// Carry-save accumulation: a running sum is kept as two such integers (S, K) whose sum is
// the value; adding one more integer X costs one full adder per bit, i.e. a three-input
// XOR and a three-input majority per plane (one v_bitop3_b32 each), with no carry chain.
// ---------------------------------------------------------------------------------------

// One carry-save step modulo 2^NB - 1: (S, K) <- S + K + X.
template <int NB> GFQ_HD void csa_step(u32 *S, u32 *K, const u32 *X) {
    u32 c[NB];
#pragma unroll
    for (int i = 0; i < NB; i++) {
        const u32 s = xor3(S[i], K[i], X[i]);
        c[(i + 1) % NB] = maj3(S[i], K[i], X[i]);
        S[i] = s;
    }
#pragma unroll
    for (int i = 0; i < NB; i++) K[i] = c[i];
}

// The same step adding -X, i.e. the complement of X (negation modulo 2^NB - 1).
template <int NB> GFQ_HD void csa_step_neg(u32 *S, u32 *K, const u32 *X) {
    u32 c[NB];
#pragma unroll
    for (int i = 0; i < NB; i++) {
        const u32 s = xor3n(S[i], K[i], X[i]);
        c[(i + 1) % NB] = maj3n(S[i], K[i], X[i]);
        S[i] = s;
    }
#pragma unroll
    for (int i = 0; i < NB; i++) K[i] = c[i];
}

// F_3 in binary modulo 3: planes (b0, b1) of b0 + 2 b1, where 3 also means 0.
// From the storage code (unit x0, sign x1): 1 = 10 -> 01 and -1 = 11 -> 10.
GFQ_HD void f3_to_bin(u32 x0, u32 x1, u32 *b) { b[0] = x0 ^ x1; b[1] = x1; }

// Addition modulo 3 of two 2-bit residues (either of 0 and 3 may stand for 0) in four
// three-input instructions, the fewest possible: an exhaustive search over programs of
// arbitrary three-input gates (the paper's search for minimal programs on 2-bit fields,
// Section 4, re-run with the instruction gfx950 has; search/f3b_add_search.cpp) finds none
// of three and this one of four.  Over operands (a, b, c) weighted 4, 2, 1:
//   h1 = [at most one of b0, a1, a0 set],  h2 = lut 0x49 (b0, a1, a0),
//   r0 = a1 ^ b1 ^ h1,                     r1 = lut 0x49 (r0, h2, b1).
// B_NEG adds the complement of b (3 - b = -b mod 3), i.e. subtracts b: the complemented
// operands are folded into the truth tables.
template <bool B_NEG> GFQ_HD void f3b_add_t(const u32 *a, const u32 *b, u32 *r) {
    const u32 h1 = lut3<lut3_flip(0x17, B_NEG ? 4 : 0)>(b[0], a[1], a[0]);
    const u32 h2 = lut3<lut3_flip(0x49, B_NEG ? 4 : 0)>(b[0], a[1], a[0]);
    r[0] = lut3<lut3_flip(0x96, B_NEG ? 1 : 0)>(a[1], h1, b[1]);
    r[1] = lut3<lut3_flip(0x49, B_NEG ? 1 : 0)>(r[0], h2, b[1]);
}
GFQ_HD void f3b_add(const u32 *a, const u32 *b, u32 *r) { f3b_add_t<false>(a, b, r); }
GFQ_HD void f3b_sub(const u32 *a, const u32 *b, u32 *r) { f3b_add_t<true>(a, b, r); }

// Back to the storage code: residue 0 (00 or 11) -> 00, 1 -> 10, 2 -> 11.
GFQ_HD void f3_from_bin(const u32 *b, u32 *x0, u32 *x1) { *x0 = b[0] ^ b[1]; *x1 = b[1] & ~b[0]; }

// Addition on the storage code of Section 4.1, through the binary residues: both operands
// to b0 + 2 b1 (one XOR each), the four-instruction residue addition, back to the code.
// Used off the product's inner loop (partial sums, Strassen-Winograd operand sums).
GFQ_HD F3v f3_add(F3v x, F3v y) {
    u32 a[2], b[2], r[2];
    f3_to_bin(x.u, x.s, a);
    f3_to_bin(y.u, y.s, b);
    f3b_add(a, b, r);
    F3v z;
    f3_from_bin(r, &z.u, &z.s);
    return z;
}

// Full adder on three bits, the operands selected by NEG (4: x, 2: y, 1: z) complemented:
// sum and carry, one three-input instruction each.
template <int NEG> GFQ_HD u32 fa_sum(u32 x, u32 y, u32 z) { return lut3<lut3_flip(0x96, NEG)>(x, y, z); }
template <int NEG> GFQ_HD u32 fa_carry(u32 x, u32 y, u32 z) { return lut3<lut3_flip(0xE8, NEG)>(x, y, z); }

// F_5 addition and subtraction of 3-bit representatives in eight three-input instructions
// (against eleven to thirteen for a 4-bit sum folded back modulo 5).  Bits of weight 4 = -1 enter
// weight 1 complemented (4x = ~x - 1) and a constant bit fixes the offsets, so that four
// adders reduce the columns to one bit each, the last carry being bit 2 of the result:
//   a + b: weight 2 gets a1, b1 and a constant 1 (sum ~(a1 ^ b1), carry a1 | b1, which goes
//          to weight 1 as ~(a1 | b1)); weight 1 gets a0, b0, ~a2, ~b2 and that bit; the
//          offsets -2 - 1 - 1 - 1 sum to 0 (mod 5).
//   a - b: weight 1 gets a0, ~b0, b2, ~a2, weight 2 a1, ~b1 (offsets -1 - 2 - 1); the carry
//          out of weight 2 enters weight 1 complemented (-1), -5 = 0.
GFQ_HD void f5_add8(const u32 *a, const u32 *b, u32 *r) {
    const u32 n = lut3<0x03>(a[1], b[1], b[1]);                 // ~(a1 | b1)
    const u32 u = lut3<0xC3>(a[1], b[1], b[1]);                 // ~(a1 ^ b1)
    const u32 s1 = fa_sum<1>(a[0], b[0], a[2]), k1 = fa_carry<1>(a[0], b[0], a[2]);
    const u32 k2 = fa_carry<4>(b[2], n, s1);
    r[0] = fa_sum<4>(b[2], n, s1);
    r[1] = fa_sum<0>(u, k1, k2);
    r[2] = fa_carry<0>(u, k1, k2);
}
GFQ_HD void f5_sub8(const u32 *a, const u32 *b, u32 *r) {
    const u32 s1 = fa_sum<2>(a[0], b[0], b[2]), k1 = fa_carry<2>(a[0], b[0], b[2]);
    const u32 u1 = fa_sum<2>(a[1], b[1], k1), c1 = fa_carry<2>(a[1], b[1], k1);
    const u32 k2 = fa_carry<3>(s1, a[2], c1);
    r[0] = fa_sum<3>(s1, a[2], c1);
    r[1] = u1 ^ k2;
    r[2] = u1 & k2;
}
// F_5 negation of a 3-bit representative: 0 - a by the subtraction above (the zero operand
// folds into its truth tables).
GFQ_HD P3v f5_neg(P3v a) {
    const u32 z[3] = {0u, 0u, 0u}, b[3] = {a.b0, a.b1, a.b2};
    u32 r[3];
    f5_sub8(z, b, r);
    P3v n;
    n.b0 = r[0]; n.b1 = r[1]; n.b2 = r[2];
    return n;
}

// One F_5 slab into a carry-save accumulator modulo 5 of three planes (a, b, c): its value
// is a + b + 2c, between 0 and 4.  A bit of weight 4 = -1 (mod 5) re-enters the weight-1
// column complemented (-x = ~x - 1), so the accumulator needs only two columns (weights 1
// and 2).  The slab's table rows are t = T[phi_0], v = T[phi_1] (scale 2), w = T[phi_2]
// (scale 4), each any 3-bit representative; their nine bits sit in the columns as
//   weight 1: t0, ~t2, ~v1, ~w0, w2        weight 2: t1, v0, ~v2, ~w1
// (t2, v1, w0 weigh 4 = -1; v2, w1 weigh 8 = -2; w2 weighs 16 = 1).  Nine full adders and
// one half adder bring the columns back to two bits and one bit; the five carries out of
// the weight-2 column re-enter complemented.  The constants dropped by the complements sum
// to -12, so every slab adds 12 = 2 (mod 5) beyond t + 2v + 4w, which the starting value
// cancels: 20 instructions, three accumulator planes.

GFQ_HD void f5_nc_slab(u32 *s, const u32 *t, const u32 *v, const u32 *w) {
    // weight 1: a, b, t0, ~t2, ~v1, ~w0, w2
    const u32 s1 = fa_sum<0>(s[0], s[1], t[0]), k1 = fa_carry<0>(s[0], s[1], t[0]);
    const u32 s2 = fa_sum<7>(t[2], v[1], w[0]), k2 = fa_carry<7>(t[2], v[1], w[0]);
    const u32 s3 = fa_sum<0>(w[2], s1, s2), k3 = fa_carry<0>(w[2], s1, s2);
    // weight 2: c, t1, v0, ~v2, ~w1 and the carries k1, k2, k3
    const u32 u1 = fa_sum<0>(s[2], t[1], v[0]), m1 = fa_carry<0>(s[2], t[1], v[0]);
    const u32 u2 = fa_sum<6>(v[2], w[1], k1), m2 = fa_carry<6>(v[2], w[1], k1);
    const u32 u3 = fa_sum<0>(k2, k3, u1), m3 = fa_carry<0>(k2, k3, u1);
    // weight 1: s3, ~m1, ~m2, ~m3; weight 2: u2, u3 and the carries
    const u32 s4 = fa_sum<3>(s3, m1, m2), k4 = fa_carry<3>(s3, m1, m2);
    const u32 u4 = fa_sum<0>(u2, u3, k4), m4 = fa_carry<0>(u2, u3, k4);
    const u32 s5 = fa_sum<6>(m3, m4, s4), k5 = fa_carry<6>(m3, m4, s4);
    // half adder on weight 2 (u4, k5): its carry re-enters weight 1 complemented
    s[0] = s5;
    s[1] = lut3<0x3F>(u4, k5, k5);          // ~(u4 & k5)
    s[2] = u4 ^ k5;
}

// Starting value for `slabs` slabs: a + b + 2c = -2 x slabs (mod 5), every plane all-zero
// or all-one.
GFQ_HD void f5_nc_init(u32 *s, int slabs) {
    const int r = (3 * (slabs > 0 ? slabs % 5 : 0)) % 5;
    const u32 one = 0xffffffffu;
    s[0] = (r & 1) || r == 4 ? one : 0u;      // 1 = a, 2 = c, 3 = a + c, 4 = a + b + c
    s[1] = r == 4 ? one : 0u;
    s[2] = r >= 2 ? one : 0u;
}

// The accumulator's value a + b + 2c (at most 4, so already the canonical code).
GFQ_HD P3v f5_nc_value(const u32 *s) {
    P3v z;
    z.b0 = s[0] ^ s[1];
    z.b1 = s[2] ^ (s[0] & s[1]);
    z.b2 = s[0] & s[1] & s[2];
    return z;
}

}  // namespace gfq
