// Hankel form of the M2L (private to the library): shapes and bank layout.
//
// The scaled operator of Eq. (eq:M2Lmat) is, up to two diagonal scalings, a
// Hankel matrix (its entries depend on n + k only):
//     A~(d)[n][k] = (-1)^n C(n+k, k) d^-(n+k+1)
//                 = [(-1)^n rho^n / n!]  g_(n+k)(d)  [rho^k / k!],
//     g_m(d) = m! rho^-m d^-(m+1),   m = 0 .. 2p - 2,
// for any rho > 0.  A Hankel product y_n = sum_k g_(n+k) z_k is a linear
// convolution of g with the reversed z, read at n + p - 1, so with length-N
// discrete Fourier transforms (N >= 2p - 1 avoids wrap-around at those
// outputs) every translation of a target's interaction list becomes N complex
// multiply-adds of spectra, and the sum over the list can be taken in the
// frequency domain:
//     Y^(t) = sum_o G^(d_o) . Z^(t + o),   Z^(s) = DFT(reverse(D_R M~(s))),
//     L~_n(t) = D_L[n] IDFT(Y^(t))[n + p - 1].
// Spectra of the operators G^ are built once per p (FP64, as every bank).
// The arithmetic runs in FP64: m! against rho^m spans many decades, and FP32
// spectra lose the small coefficients (relative error ~1e-3 at p = 20).  With
// rho near 0.4 p the FP64 result agrees with the dense operator to ~1e-11.
//
// The adjoint is the same product transposed: A~(d)^T = D_R G(d) D_L (a
// Hankel matrix is symmetric), gathered over each source's own list with
// d = +o, i.e. the operator spectrum of the mirrored offset.
#pragma once

#include <cstddef>

#include "m2l_bank.h"

namespace fmm2d {

template <int P>
struct HankelCfg {
  static constexpr int N = 2 * P;  // transform length (>= 2p - 1)
  static constexpr double rho() { return P == 8 ? 3.0 : P == 12 ? 4.0 : P == 16 ? 6.0 : 8.0; }
};

// Sections (bytes; complex = two doubles unless stated):
//   ghat [slot][N]   complex   G^ of d = -o for slot(o) (the forward
//                              translation from source t + o); the adjoint
//                              reads slot(-o)
//   dr   [P]         double    rho^k / k!
//   dl   [P]         double    (-1)^n rho^n / n!
//   tw   [N]         complex   exp(-2 pi i j / N)
//   r    [slot][P]   complex float  forward log row r_o (log d, -d^-k / k), d = -o
template <int P>
struct HankelBank {
  using C = HankelCfg<P>;
  static constexpr int N = C::N;
  static constexpr size_t ghat_off = 0;
  static constexpr size_t dr_off = ghat_off + size_t(kSlots) * N * 16;
  static constexpr size_t dl_off = dr_off + size_t(P) * 8;
  static constexpr size_t tw_off = (dl_off + size_t(P) * 8 + 255) / 256 * 256;
  static constexpr size_t r_off = (tw_off + size_t(N) * 16 + 255) / 256 * 256;
  static constexpr size_t total_bytes = (r_off + size_t(kSlots) * P * 8 + 255) / 256 * 256;
};

inline size_t hankel_bank_bytes(int p) {
  switch (p) {
    case 8: return HankelBank<8>::total_bytes;
    case 12: return HankelBank<12>::total_bytes;
    case 16: return HankelBank<16>::total_bytes;
    case 20: return HankelBank<20>::total_bytes;
  }
  return 0;
}

}  // namespace fmm2d
