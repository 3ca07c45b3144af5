/*
 * fgt2d.h -- C ABI of the fast Gauss transform's Hermite stage in libfmm2d.so
 * (Cruz, Layton & Barba, arXiv:1009.3457, Sec. 2.2 and Sec. 4.2), on AMD
 * MI355X (gfx950).  Status codes, fmm2d_last_error() and the memory and
 * stream rules are those of fmm2d.h.
 *
 * In two dimensions, for a Gaussian of width sigma, the discrete Gauss
 * transform (Eq. (eqn:dgt)) is
 *     G(y) = sum_i q_i exp(-|x_i - y|^2 / (2 sigma^2)).
 * Its sources are grouped into the 4^depth boxes of the uniform grid over
 * [0,1]^2 that fmm2d_build_tree uses (box of width w = 2^-depth, centre s_B,
 * Morton numbering).  Each box's Gaussians are summed into a Hermite series
 * about s_B (Eq. (eqn:A_alpha)), truncated to the multi-indices
 * alpha = (a, b) with 0 <= a, b < p:
 *     A_ab(B) = 1/(a! b!) sum_{j in B} q_j s1^a s2^b,   s = (x_j - s_B) / (sqrt(2) sigma),
 * and a target y in box (tx, ty) sums the series of the boxes (bx, by) with
 * |bx - tx| <= K and |by - ty| <= K (Eq. (eqn:hermite)):
 *     G_K(y) = sum_B sum_{a,b<p} A_ab(B) h_a(t1) h_b(t2),   t = (y - s_B) / (sqrt(2) sigma),
 * with h_n(t) = exp(-t^2) H_n(t), H_n the physicists' Hermite polynomials.
 *
 * Accuracy (a guide for choosing p, K and sigma): with w = r sqrt(2) sigma,
 * sources lie within r/2 of their box centre in s, the sources cut off by K
 * contribute at most sum|q| exp(-K^2 r^2), and the truncation to p terms per
 * dimension errs by at most sum|q| (2 rho + rho^2) with
 * rho = 1.0865 sum_{n>=p} (r/sqrt(2))^n / sqrt(n!).
 * Supported: p = 1..FGT2D_MAX_P, depth 0..12, 0 <= K < 2^depth.
 */
#ifndef FGT2D_H
#define FGT2D_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "fmm2d.h"

#ifdef __cplusplus
extern "C" {
#endif

#define FGT2D_MAX_P 16

/*
 * Hermite coefficients of every box (Eq. (eqn:A_alpha)).
 *   xy_sorted [n][2] float, q_sorted [n] float: the sources in box order, with
 *   leaf_start [4^depth + 1] from fmm2d_build_tree at the same depth (sources
 *   of box m are leaf_start[m] .. leaf_start[m+1]-1).
 *   A [4^depth][p][p] float, indexed [box][a][b]: written for every box (zero
 *   for empty boxes).  Sums are formed in FP64 and rounded once.
 * Errors: FMM2D_EDEPTH, FMM2D_EUNSUPPORTED_P (p outside 1..16), FMM2D_EINVAL
 * (NULL pointer, sigma not finite and positive), FMM2D_EHIP.
 */
int fgt2d_hermite_coeffs(const float *xy_sorted, const float *q_sorted, const int32_t *leaf_start,
                         int depth, int p, float sigma, float *A, hipStream_t stream);

/*
 * Hermite evaluation (Eq. (eqn:hermite)): G[t] = G_K(txy[t]) for t < nt,
 * OVERWRITTEN.  FP32 arithmetic.
 *   txy [nt][2] float in [0,1]^2, any order (coordinates outside are clamped
 *   to the edge boxes, NaN to box 0; they are not rejected).  Targets sorted
 *   by box (e.g. gathered with a perm from fmm2d_build_tree) run fastest.
 *   A [4^depth][p][p] float from fgt2d_hermite_coeffs with the same depth, p
 *   and sigma.
 * Errors: as fgt2d_hermite_coeffs, plus FMM2D_EINVAL for nt outside
 * [0, 2^31) or K outside 0..2^depth - 1.  nt = 0 enqueues nothing.
 */
int fgt2d_hermite_eval(const float *txy, int64_t nt, int depth, int p, float sigma, int K,
                       const float *A, float *G, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* FGT2D_H */
