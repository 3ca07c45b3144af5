// Layout of the M2L operator bank (private to the library).
//
// The interaction list of a box t at level l >= 2 with child class
// c = (ix & 1, iy & 1) is the set of boxes t + o for the 27 offsets
//   o in O_c = { (ox, oy) : ox in [-2-cx, 3-cx], oy in [-2-cy, 3-cy], max(|ox|,|oy|) >= 2 }
// (children of the parent's neighbours that do not touch t), clipped to the
// grid.  The four classes together use 40 distinct offsets in [-3,3]^2; the
// bank keeps one slot per point of the 7x7 offset grid (9 central slots stay
// zero) so a slot index is plain arithmetic: slot(o) = (ox+3) + 7 (oy+3).
// O_c for c = (1, .) is the mirror image of O_(0, .): every list is
// (sx ox0, sy oy0) over the fixed list (ox0, oy0) of class (0, 0) below,
// with sx = 1 - 2 cx, sy = 1 - 2 cy.
//
// The translation from source s = t + o to target t uses Eq. (eq:M2Lmat) at
// d = x_t - x_s, which in box widths is d = -(ox + i oy).  In the scaled
// basis the matrix is level independent:
//   A~_o[n][k] = (-1)^n C(n+k, k) d^-(n+k+1),  n, k < p,
// and the log-potential row is r_o[0] = log d, r_o[k] = -d^-k / k.
#pragma once

#include <cstddef>
#include <cstdint>

namespace fmm2d {

constexpr int kSlots = 49;
__host__ __device__ constexpr int slot_of(int ox, int oy) { return (ox + 3) + 7 * (oy + 3); }

// The 27 offsets of class (0, 0) in the fixed order every kernel uses.
struct OffList {
  int ox[27];
  int oy[27];
};

constexpr OffList make_offsets00() {
  OffList L{};
  int n = 0;
  for (int oy = -2; oy <= 3; ++oy)
    for (int ox = -2; ox <= 3; ++ox) {
      if (ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1) continue;
      L.ox[n] = ox;
      L.oy[n] = oy;
      ++n;
    }
  return L;
}

constexpr OffList kOff00 = make_offsets00();

// ------------------------------------------------------------ FP32 bank --
// The FP32 contraction runs on v_mfma_f32_16x16x4_f32 in Gauss's
// three-multiplication form of the complex product:
//   T1 = Ar Xr,  T2 = Ai Xi,  T3 = (Ar + Ai)(Xr + Xi),
//   Re Y = T1 - T2,  Im Y = T3 - T1 - T2.
// MFMA rows are output orders n (16 per M-tile, MT tiles), columns are 16
// target boxes, and the contraction index k is split into S = p/4 steps of 4.
// Lane l of a wave owns row n = 16 mt + l % 16 of the A operand and the k
// values k = S (l / 16) + s, s < S, so its A fragment for one offset is
// 2 S floats: part q (0: Ar, 1: Ai) at position q S + s.  The kernels form
// the third Gauss operand Ar + Ai (and Xr + Xi) in FP32 as they go.
//
// When p is not a multiple of 16 the last M tile has spare rows.  Row p then
// carries the log-potential row r_o and row p + 1 the unit row e_0, so the
// same products also deliver b = Y[p] + log(h) Y[p+1] (Y[p+1] = sum of M~_0
// over the list) at no extra cost.  For p = 16 a separate pass computes b.
//
// Adjoint log-row part.  The transpose of the log row adds
//   gM~_n(s) += sum_o r_n(+o) gb(s + o)   (+ log(h) sum_o gb(s + o) for n = 0),
// a contraction over the 27 offsets of s's class.  It runs on the same MFMA
// with the offset list as the contraction index: k-step g covers list
// entries 4 g .. 4 g + 3 (entry 27 is padding), lane l contributing entry
// 4 g + l / 16.  Section 3 holds the A fragments of that product, negated
// (the adjoint negates the whole accumulator once at the end), and when there
// is a spare row p + 2 it holds -1 so the same product yields -sum_o gb.
template <int P>
struct F32Bank {
  static constexpr int S = P / 4;                   // k steps of 4
  static constexpr int MT = (P + 15) / 16;          // M tiles of 16 output rows
  static constexpr int LS = ((2 * S + 3) / 4) * 4;  // floats per lane fragment (padded to float4)
  static constexpr bool kLogInRows = (P % 16) != 0; // rows p, p+1 hold r_o and e_0
  static constexpr bool kGbSumRow = (P + 2) < 16 * MT;  // row p+2 free for sum_o gb
  static constexpr int kGbSteps = 7;                // ceil(27 / 4) k-steps over the offset list
  // section 1: A fragments  [slot][mt][lane][LS] floats
  static constexpr size_t a_floats = size_t(kSlots) * MT * 64 * LS;
  // section 2: forward log row  [slot][k] complex: r_o[k]  (used by the separate b pass)
  static constexpr size_t r_floats = size_t(kSlots) * P * 2;
  // section 3: adjoint log-row A fragments  [class][g][mt][lane] complex
  static constexpr size_t ga_floats = size_t(4) * kGbSteps * MT * 64 * 2;
  static constexpr size_t a_off = 0;
  static constexpr size_t r_off = (a_off + a_floats + 63) / 64 * 64;
  static constexpr size_t ga_off = (r_off + r_floats + 63) / 64 * 64;
  static constexpr size_t total_floats = (ga_off + ga_floats + 63) / 64 * 64;
};

inline size_t f32_bank_bytes(int p) {
  switch (p) {
    case 8: return F32Bank<8>::total_floats * 4;
    case 12: return F32Bank<12>::total_floats * 4;
    case 16: return F32Bank<16>::total_floats * 4;
    case 20: return F32Bank<20>::total_floats * 4;
  }
  return 0;
}

}  // namespace fmm2d
