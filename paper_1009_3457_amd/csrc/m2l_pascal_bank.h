// Pascal-form FP32 M2L: shapes and operator-bank layout (private to the
// library).
//
// The scaled operator of Eq. (eq:M2Lmat) factorises exactly as
//     A~(d) = D1(d) B D2(d),   B[n][k] = C(n+k, k),
//     D1(d) = diag((-1)^n d^-(n+1)),   D2(d) = diag(d^-k),
// with d = x_t - x_s in box widths.  B is real, symmetric and the same for
// every translation, so the contraction of one offset is two real products
// with a constant operand (one for Re, one for Im of the scaled source
// D2 x) instead of three, and the offset enters only through the two complex
// diagonal scalings, done on the VALU.  The adjoint is A~(d)^T = D2(d) B D1(d).
//
// MFMA layout as for the Gauss-form kernel (m2l_bank.h): rows are output
// orders, columns the 16 target boxes of a class, the contraction index k is
// split into S = p/4 k-steps with lane l holding k = S (l/16) + s.  An input
// scaling ("in" record) therefore covers the k values of one lane group,
// and an output scaling ("out" record) the rows 16 mt + 4 (l/16) + r,
// r < 4, that an MFMA output fragment gives lane l.
//
// Symmetric offsets.  With S1 = diag(-(-1)^n) and S2 = diag((-1)^k),
// D1(-d) = D1(d) S1 and D2(-d) = D2(d) S2, so
//     A~(-d) = D1(d) B' D2(d),   B' = S1 B S2,  B'[n][k] = -(-1)^(n+k) C(n+k, k).
// Offsets o and -o that are both in a class's list (8 pairs of its 27) are
// therefore taken together: both sources are scaled by D2(d), the products
// B D2 x(t+o) + B' D2 x(t-o) are summed in the MFMA accumulator, and D1(d)
// is applied once.  The adjoint pairs the same way with B'^T = B'.
//
// When p is not a multiple of 16, rows p .. p+3 carry the log-potential
// constant.  B rows: p = (0, -1/1, -1/2, ...), p+1 = p+2 = e_0, p+3 = 0;
// B' rows: p = (0, +1/1, -1/2, +1/3, ...) (row p of B times (-1)^k),
// p+1 = p+2 = p+3 = e_0.  Output scalings 1, log d, 1 and, for a pair,
// log(-d) - log d (= +-i pi; 0 for a single offset), so that
//     b = L[p] + L[p+1] + L[p+3] + log(h) L[p+2].
// For p = 16 (no spare rows) the kernel forms b from the D2-scaled sources.
#pragma once

#include <cstddef>

#include "m2l_bank.h"

namespace fmm2d {

template <int P>
struct PascalCfg {
  static constexpr int S = P / 4;                      // k-steps of 4
  static constexpr bool kLogInRows = (P % 16) != 0;    // rows p .. p+3 fit in the last M tile
  static constexpr int ROWS = P + (kLogInRows ? 4 : 0);
  static constexpr int MT = (ROWS + 15) / 16;          // M tiles of 16 rows
  static constexpr int LI = ((2 * S + 3) / 4) * 4;     // floats of an "in" record (S complex, padded)
  static constexpr int LO = 8;                         // floats of an "out" record (4 complex)
};

// Sections (floats):
//   bf   [mt][s][lane]                     A fragments of B (rows extended as above)
//   bfp  [mt][s][lane]                     A fragments of B' (rows extended as above)
//   tin  [dir][cls][q][kk][LI]             forward: d^-k;        adjoint: (-1)^k d^-(k+1)
//   tout [dir][cls][q][mt][kk][LO]         forward: D1 and the log rows; adjoint: d^-n (rows < p)
//   lg   [dir][cls][q][2]                  log d
//   zero [64][P][2]                        zeros: the source record of a box outside
//                                          the level, for any box position in an 8x8 block
// dir 0 is the forward translation (d = -o for source t + o of class cls,
// offset q of the list), dir 1 the adjoint (d = +o, gathered over the
// class's own list); cls = cx + 2 cy.
template <int P>
struct PascalBank {
  using C = PascalCfg<P>;
  static constexpr size_t bf_floats = size_t(C::MT) * C::S * 64;
  static constexpr size_t bfp_floats = bf_floats;
  static constexpr size_t tin_floats = size_t(2) * 4 * 27 * 4 * C::LI;
  static constexpr size_t tout_floats = size_t(2) * 4 * 27 * C::MT * 4 * C::LO;
  static constexpr size_t lg_floats = size_t(2) * 4 * 27 * 2;
  static constexpr size_t zero_floats = size_t(64) * P * 2;
  static constexpr size_t bf_off = 0;
  static constexpr size_t bfp_off = (bf_off + bf_floats + 63) / 64 * 64;
  static constexpr size_t tin_off = (bfp_off + bfp_floats + 63) / 64 * 64;
  static constexpr size_t tout_off = (tin_off + tin_floats + 63) / 64 * 64;
  static constexpr size_t lg_off = (tout_off + tout_floats + 63) / 64 * 64;
  static constexpr size_t zero_off = (lg_off + lg_floats + 63) / 64 * 64;
  static constexpr size_t total_floats = (zero_off + zero_floats + 63) / 64 * 64;
  __host__ __device__ static constexpr size_t tin_rec(int dir, int cls, int q) {
    return tin_off + ((size_t(dir) * 4 + cls) * 27 + q) * 4 * C::LI;
  }
  __host__ __device__ static constexpr size_t tout_rec(int dir, int cls, int q, int mt) {
    return tout_off + (((size_t(dir) * 4 + cls) * 27 + q) * C::MT + mt) * 4 * C::LO;
  }
  __host__ __device__ static constexpr size_t lg_rec(int dir, int cls, int q) {
    return lg_off + ((size_t(dir) * 4 + cls) * 27 + q) * 2;
  }
};

// Offsets of class (0, 0) taken together with their negatives: entry j of
// the step list is list index q1 alone (q2 < 0) or q1 with q2, o(q2) = -o(q1).
struct PascalSteps {
  int n;
  int q1[27], q2[27];
};

constexpr PascalSteps make_pascal_steps(bool pairs) {
  PascalSteps st{};
  bool used[27] = {};
  for (int a = 0; a < 27; ++a) {
    if (used[a]) continue;
    int partner = -1;
    for (int b = a + 1; b < 27 && pairs; ++b)
      if (!used[b] && kOff00.ox[b] == -kOff00.ox[a] && kOff00.oy[b] == -kOff00.oy[a]) partner = b;
    used[a] = true;
    if (partner >= 0) used[partner] = true;
    st.q1[st.n] = a;
    st.q2[st.n] = partner;
    ++st.n;
  }
  return st;
}

constexpr PascalSteps kPascalSteps = make_pascal_steps(true);
constexpr PascalSteps kPascalSingles = make_pascal_steps(false);
static_assert(kPascalSteps.n == 19, "8 symmetric pairs and 11 single offsets");
static_assert(kPascalSingles.n == 27, "every offset alone");

// list index of the negative of offset q of class (0, 0), or -1
__host__ __device__ constexpr int pascal_partner(int q) {
  for (int j = 0; j < kPascalSteps.n; ++j) {
    if (kPascalSteps.q1[j] == q) return kPascalSteps.q2[j];
    if (kPascalSteps.q2[j] == q) return kPascalSteps.q1[j];
  }
  return -1;
}

inline size_t pascal_bank_bytes(int p) {
  switch (p) {
    case 8: return PascalBank<8>::total_floats * 4;
    case 12: return PascalBank<12>::total_floats * 4;
    case 16: return PascalBank<16>::total_floats * 4;
    case 20: return PascalBank<20>::total_floats * 4;
  }
  return 0;
}

}  // namespace fmm2d
