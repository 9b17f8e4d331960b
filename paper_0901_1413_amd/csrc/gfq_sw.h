// gfq_sw.h -- the Strassen–Winograd schedule used above the Four-Russians product: seven
// products of half-size operands, each operand a signed sum of quadrants, and the four
// quadrants of the product as signed sums of the seven products.  Plain C++ (no HIP), so
// the tables can be checked on the host.
//
// Quadrants are numbered 0..3 for X11, X12, X21, X22.  With
//   S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21, S4 = A12 - S2,
//   T1 = B12 - B11, T2 = B22 - T1, T3 = B22 - B12, T4 = T2 - B21,
// the products are P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4, P5 = S1 T1,
// P6 = S2 T2, P7 = S3 T3, and C11 = P1 + P2, C12 = P1 + P6 + P5 + P3,
// C21 = P1 + P6 + P7 - P4, C22 = P1 + P6 + P7 + P5 (Winograd's form of Strassen's method:
// seven multiplications instead of eight per level).
#pragma once

namespace gfq {

// left operand of product c: sum over quadrants j of SW_A[c][j] * A_j
constexpr int SW_A[7][4] = {
    {1, 0, 0, 0},     // A11
    {0, 1, 0, 0},     // A12
    {1, 1, -1, -1},   // S4 = A11 + A12 - A21 - A22
    {0, 0, 0, 1},     // A22
    {0, 0, 1, 1},     // S1 = A21 + A22
    {-1, 0, 1, 1},    // S2 = A21 + A22 - A11
    {1, 0, -1, 0},    // S3 = A11 - A21
};
// right operand of product c: sum over quadrants j of SW_B[c][j] * B_j
constexpr int SW_B[7][4] = {
    {1, 0, 0, 0},     // B11
    {0, 0, 1, 0},     // B21
    {0, 0, 0, 1},     // B22
    {1, -1, -1, 1},   // T4 = B11 - B12 - B21 + B22
    {-1, 1, 0, 0},    // T1 = B12 - B11
    {1, -1, 0, 1},    // T2 = B11 - B12 + B22
    {0, -1, 0, 1},    // T3 = B22 - B12
};
// quadrant j of the product: sum over c of SW_C[j][c] * P_c
constexpr int SW_C[4][7] = {
    {1, 1, 0, 0, 0, 0, 0},    // C11 = P1 + P2
    {1, 0, 1, 0, 1, 1, 0},    // C12 = P1 + P3 + P5 + P6
    {1, 0, 0, -1, 0, 1, 1},   // C21 = P1 - P4 + P6 + P7
    {1, 0, 0, 0, 1, 1, 1},    // C22 = P1 + P5 + P6 + P7
};

// Half of a dimension at one level: rows split at ceil(d / 2); columns (and the inner
// dimension, a column dimension of the left operand) at ceil(d / 2) rounded up to whole
// 32-bit words, so every quadrant starts at a word boundary.  Missing rows and columns of
// the second half are zero.
inline long long sw_half_rows(long long d) { return (d + 1) / 2; }
inline long long sw_half_cols(long long d) { return ((d + 1) / 2 + 31) / 32 * 32; }

}  // namespace gfq
