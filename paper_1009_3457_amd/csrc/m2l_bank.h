// Layout of the M2L operator bank (private to the library).
//
// The interaction list of a box t at level l >= 2 with child class
// c = (ix & 1, iy & 1) is the set of boxes t + o for the 27 offsets
//   o in O_c = { (ox, oy) : ox in [-2-cx, 3-cx], oy in [-2-cy, 3-cy], max(|ox|,|oy|) >= 2 }
// (children of the parent's neighbours that do not touch t), clipped to the
// grid.  The four classes together use 40 distinct offsets in [-3,3]^2; the
// bank keeps one slot per point of the 7x7 offset grid (9 central slots stay
// zero) so a slot index is plain arithmetic: slot(o) = (ox+3) + 7 (oy+3).
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

// ------------------------------------------------------------ FP32 bank --
// The FP32 contraction runs on v_mfma_f32_16x16x4_f32 in Gauss's
// three-multiplication form of the complex product:
//   T1 = Ar Xr,  T2 = Ai Xi,  T3 = (Ar + Ai)(Xr + Xi),
//   Re Y = T1 - T2,  Im Y = T3 - T1 - T2.
// MFMA rows are output orders n (16 per M-tile, MT tiles), columns are 16
// target boxes, and the contraction index k is split into S = p/4 steps of 4.
// Lane l of a wave owns row n = 16 mt + l % 16 of the A operand and the k
// values k = S (l / 16) + s, s < S, so its A fragment for one offset is
// 3 S floats: part q (0: Ar, 1: Ai, 2: Ar + Ai) at position q S + s.
template <int P>
struct F32Bank {
  static constexpr int S = P / 4;                   // k steps of 4
  static constexpr int MT = (P + 15) / 16;          // M tiles of 16 output rows
  static constexpr int LS = ((3 * S + 3) / 4) * 4;  // floats per lane fragment (padded to float4)
  // section 1: A fragments  [slot][mt][lane][LS] floats
  static constexpr size_t a_floats = size_t(kSlots) * MT * 64 * LS;
  // section 2: forward log row  [slot][kk (4)][S] complex: r_o[S kk + s]
  static constexpr size_t r_floats = size_t(kSlots) * 4 * S * 2;
  // section 3: adjoint log row  [slot][mt][kk (4)][4] complex: r_(-o)[16 mt + 4 kk + i]
  //   (the adjoint gathers gb(s + o') with the row of d = +o', see m2l_f32.hip)
  static constexpr size_t ra_floats = size_t(kSlots) * MT * 16 * 2;
  static constexpr size_t a_off = 0;
  static constexpr size_t r_off = (a_off + a_floats + 63) / 64 * 64;
  static constexpr size_t ra_off = (r_off + r_floats + 63) / 64 * 64;
  static constexpr size_t total_floats = (ra_off + ra_floats + 63) / 64 * 64;
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
