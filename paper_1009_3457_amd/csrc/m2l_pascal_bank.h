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
// When p is not a multiple of 16, rows p .. p+2 carry the log-potential
// constant: B row p = (0, -1/1, -1/2, ...), rows p+1 and p+2 = e_0, with
// output scalings 1, log d and 1, so that
//     b = L[p] + L[p+1] + log(h) L[p+2].
// For p = 16 the separate b pass reads section r (the forward log rows).
#pragma once

#include <cstddef>

#include "m2l_bank.h"

namespace fmm2d {

template <int P>
struct PascalCfg {
  static constexpr int S = P / 4;                      // k-steps of 4
  static constexpr bool kLogInRows = (P % 16) != 0;    // rows p .. p+2 fit in the last M tile
  static constexpr int ROWS = P + (kLogInRows ? 3 : 0);
  static constexpr int MT = (ROWS + 15) / 16;          // M tiles of 16 rows
  static constexpr int LI = ((2 * S + 3) / 4) * 4;     // floats of an "in" record (S complex, padded)
  static constexpr int LO = 8;                         // floats of an "out" record (4 complex)
};

// Sections (floats):
//   bf   [mt][s][lane]                     A fragments of B (rows extended as above)
//   tin  [dir][cls][q][kk][LI]             forward: d^-k;        adjoint: (-1)^k d^-(k+1)
//   tout [dir][cls][q][mt][kk][LO]         forward: D1 and the log rows; adjoint: d^-n (rows < p)
//   lg   [dir][cls][q][2]                  log d
//   r    [slot][P][2]                      forward log row r_o (separate b pass, p = 16)
//   zero [64][P][2]                        zeros: the source record of a box outside
//                                          the level, for any box position in an 8x8 block
// dir 0 is the forward translation (d = -o for source t + o of class cls,
// offset q of the list), dir 1 the adjoint (d = +o, gathered over the
// class's own list); cls = cx + 2 cy.
template <int P>
struct PascalBank {
  using C = PascalCfg<P>;
  static constexpr size_t bf_floats = size_t(C::MT) * C::S * 64;
  static constexpr size_t tin_floats = size_t(2) * 4 * 27 * 4 * C::LI;
  static constexpr size_t tout_floats = size_t(2) * 4 * 27 * C::MT * 4 * C::LO;
  static constexpr size_t lg_floats = size_t(2) * 4 * 27 * 2;
  static constexpr size_t r_floats = size_t(kSlots) * P * 2;
  static constexpr size_t zero_floats = size_t(64) * P * 2;
  static constexpr size_t bf_off = 0;
  static constexpr size_t tin_off = (bf_off + bf_floats + 63) / 64 * 64;
  static constexpr size_t tout_off = (tin_off + tin_floats + 63) / 64 * 64;
  static constexpr size_t lg_off = (tout_off + tout_floats + 63) / 64 * 64;
  static constexpr size_t r_off = (lg_off + lg_floats + 63) / 64 * 64;
  static constexpr size_t zero_off = (r_off + r_floats + 63) / 64 * 64;
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
