// Split-precision (BF16x3 / FP16x3) M2L: shapes and operator-bank layout
// (private to the library).
//
// The complex product y = A x of one translation is run as the real product
//   [y] = E(A) [x],   E(A)[2n + pr][2k + pc] = { Re a  (pr = pc = 0), -Im a (0, 1),
//                                                Im a  (1, 0),          Re a  (1, 1) },
// with rows and columns interleaved (Re, Im) exactly as complex numbers are
// stored, so a box's expansion is its own column of X and an MFMA output lane
// holds (Re y_n, Im y_n, Re y_n+1, Im y_n+1).  R = 2p real rows and columns.
//
// Each real operand is split v = hi + lo with hi = round(v), lo = round(v - hi)
// in the 16-bit format, and the three products that matter are concatenated
// along the contraction index:
//   E X ~ [E_hi | E_hi | E_lo] [X_hi; X_lo; X_hi]      (K = 3R, FP32 accumulate),
// dropping only E_lo X_lo.  The k-steps of v_mfma_f32_16x16x32_{bf16,f16}
// cover K in chunks of 8 values: lane group g = lane / 16 of k-step s holds
// chunk q = 4 s + g, i.e. segment q / (R/8) and chunk q % (R/8) of a box
// (4 complex coefficients).  Chunks past 3R are zero in the operator.
//
// When R is not a multiple of 16 (p = 12, 20) the last M tile has spare rows;
// rows R .. R+3 then carry the log row r_o (Re, Im) and the unit row e_0
// (Re, Im), so b = (Y[R] + log(h) Y[R+2]) + i (Y[R+1] + log(h) Y[R+3]) comes
// from the same products.  Otherwise (p = 8, 16) a separate pass computes b
// from section r.
//
// Adjoint log-row part gM~_n(s) += sum_o r_n(+o) gb(s + o): a contraction
// over the class's offset list, K = 2 x 28 (entry q, Re/Im of gb), two
// k-steps per split product; section ga holds its operator, negated like the
// forward products of the adjoint.
#pragma once

#include <cstddef>

#include "m2l_bank.h"

namespace fmm2d {

template <int P>
struct MixCfg {
  static constexpr int R = 2 * P;              // real rows / columns of E(A)
  static constexpr int NPL = R / 8;            // 8-value chunks per box and split part
  static constexpr bool kLogRows = (R % 16) != 0;
  static constexpr int ROWS = R + (kLogRows ? 4 : 0);
  static constexpr int MT = (ROWS + 15) / 16;  // M tiles of 16 rows
  static constexpr int KS = (3 * R + 31) / 32; // k-steps over the concatenated K
  // chunk of the A operand for (k-step, lane group): -1 zero, else part << 8 | chunk
  // (part 0: hi, 1: lo); segments 0, 1 use hi, segment 2 lo
  static constexpr int a_chunk(int ks, int g) {
    const int q = 4 * ks + g, seg = q / NPL;
    return seg >= 3 ? -1 : (((seg == 2) ? 1 : 0) << 8) | (q % NPL);
  }
  // chunk of the B operand: segments 0, 2 use hi, segment 1 lo
  static constexpr int b_chunk(int ks, int g) {
    const int q = 4 * ks + g, seg = q / NPL;
    return seg >= 3 ? -1 : (((seg == 1) ? 1 : 0) << 8) | (q % NPL);
  }
  // earliest k-step whose fragment equals that of k-step ks in every lane
  static constexpr int a_src(int ks) {
    for (int k2 = 0; k2 < ks; ++k2) {
      bool same = true;
      for (int g = 0; g < 4; ++g) same = same && a_chunk(k2, g) == a_chunk(ks, g);
      if (same) return k2;
    }
    return ks;
  }
  static constexpr int b_src(int ks) {
    for (int k2 = 0; k2 < ks; ++k2) {
      bool same = true;
      for (int g = 0; g < 4; ++g) same = same && b_chunk(k2, g) == b_chunk(ks, g);
      if (same) return k2;
    }
    return ks;
  }
  // k-steps whose fragments are loaded (the others repeat an earlier one)
  static constexpr int count_unique(bool a) {
    int n = 0;
    for (int ks = 0; ks < KS; ++ks) n += (a ? a_src(ks) : b_src(ks)) == ks;
    return n;
  }
  static constexpr int kUniqueA = count_unique(true);
  static constexpr int kUniqueB = count_unique(false);
};

// Bank: section a [slot][mt][ks][lane] 8 x 16-bit;  section ga
// [class][part][mt][t][lane] 8 x 16-bit;  section r [slot][k] complex FP32
// (the forward log row, for the separate b pass).
template <int P>
struct MixedBank {
  using C = MixCfg<P>;
  static constexpr size_t kFrag = 64 * 16;  // bytes of one fragment (64 lanes x 16 B)
  static constexpr size_t a_bytes = size_t(kSlots) * C::MT * C::KS * kFrag;
  static constexpr size_t ga_bytes = size_t(4) * 2 * C::MT * 2 * kFrag;
  static constexpr size_t r_bytes = size_t(kSlots) * P * 8;
  static constexpr size_t a_off = 0;
  static constexpr size_t ga_off = (a_off + a_bytes + 255) / 256 * 256;
  static constexpr size_t r_off = (ga_off + ga_bytes + 255) / 256 * 256;
  static constexpr size_t total_bytes = (r_off + r_bytes + 255) / 256 * 256;
  static constexpr size_t a_frag(int slot, int mt, int ks) {
    return a_off + ((size_t(slot) * C::MT + mt) * C::KS + ks) * kFrag;
  }
  static constexpr size_t ga_frag(int cls, int part, int mt, int t) {
    return ga_off + (((size_t(cls) * 2 + part) * C::MT + mt) * 2 + t) * kFrag;
  }
};

size_t mixed_bank_bytes(int p, int precision);

}  // namespace fmm2d
