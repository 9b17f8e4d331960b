// gfq_field.h -- bitsliced arithmetic over F_3, F_5, F_7 and GF(4) on 32-bit plane words.
//
// Every function works on one 32-bit word per bit-plane, i.e. on 32 field elements at
// once (paper, Section 3: the bits of one element sit in parallel words).  The formulas
// are the paper's sequential programs of Section 4, with the corrections listed next to
// each one; on gfx950 the compiler fuses them into three-input v_bitop3_b32 operations.
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

GFQ_HD u32 maj3(u32 a, u32 b, u32 c) { return (a & b) | (c & (a | b)); }

// ---------------------------------------------------------------------------------------
// F_3 (Section 4.1).  Planes (x0, x1): x0 marks a unit, x1 the sign; 0 = 00, 1 = 10,
// -1 = 11.  The code 01 never occurs.
// ---------------------------------------------------------------------------------------
struct F3v { u32 u, s; };

// Addition, 6 operations.  The printed formula swaps its two outputs: (x0 ^ y1) & (x1 ^ y0)
// is the sign plane and s | t the unit plane (checked on all nine pairs).
GFQ_HD F3v f3_add(F3v x, F3v y) {
    u32 s = x.u ^ y.s ^ x.s;
    u32 t = x.s ^ y.u ^ y.s;
    F3v r;
    r.u = s | t;
    r.s = (x.u ^ y.s) & (x.s ^ y.u);
    return r;
}

// Subtraction x - y, 6 operations, as printed.
GFQ_HD F3v f3_sub(F3v x, F3v y) {
    u32 t = x.u ^ y.u;
    F3v r;
    r.u = t | (x.s ^ y.s);
    r.s = (t ^ y.s) & (y.u ^ x.s);
    return r;
}

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
    s.b1 = a.b1 ^ b.b1 ^ c1;
    u32 c2 = maj3(a.b1, b.b1, c1);
    s.b2 = a.b2 ^ b.b2 ^ c2;
    s.b3 = maj3(a.b2, b.b2, c2);
    return s;
}

// F_7 addition (17 two-input operations): add, then add the carry back in (8 = 1 mod 7).
// The second addition never carries out: the sum is at most 14, so s0..s3 are never all 1.
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

// fold5: a 4-bit value s3 s2 s1 s0 to a 3-bit representative of the same residue mod 5.
// This is the paper's 8-operation search-found program, correct as printed.
GFQ_HD P3v fold5(u32 s0, u32 s1, u32 s2, u32 s3) {
    u32 t = s2 | s1;
    P3v r;
    r.b2 = s0 ^ t;
    r.b1 = (r.b2 & s0) ^ (s3 ^ s1);
    r.b0 = (t ^ s2) | (r.b1 & s3);
    return r;
}

// F_5 addition: 4-bit sum, then fold5.
GFQ_HD P3v f5_add(P3v a, P3v b) {
    P4v s = add3x3(a, b);
    return fold5(s.b0, s.b1, s.b2, s.b3);
}

// F_5 doubling: fold5 of the shifted value a2 a1 a0 0.
GFQ_HD P3v f5_dbl(P3v a) { return fold5(0u, a.b0, a.b1, a.b2); }

// F_5 negation: fold5 of a1 a0 0 a2 (value 8 a1 + 4 a0 + a2 = -(a0 + 2 a1 + 4 a2) mod 5).
GFQ_HD P3v f5_neg(P3v a) { return fold5(a.b2, 0u, a.b0, a.b1); }

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

}  // namespace gfq
