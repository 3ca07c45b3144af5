// Fast Gauss transform, Hermite stage (Sec. 2.2; Sec. 4.2): the coefficients
// of Eq. (eqn:A_alpha) per box and their evaluation, Eq. (eqn:hermite), at
// the targets, in two dimensions on the 4^depth boxes of the uniform grid.
//
// Evaluation is the hot part (the paper finds it about 90% of the transform).
// For a target and one box it is the bilinear form
//     sum_{a,b<p} h_a(t1) A_ab h_b(t2),   t = (y - s_B) / (sqrt(2) sigma),
// p^2 multiply-adds on one box's coefficient matrix after two Hermite-function
// recurrences.  One target per lane; every lane of a wave visits the same box
// at the same time, so the box's coefficients are wave-uniform and come in
// through scalar loads, feeding the multiply-adds as scalar operands: no LDS
// and no vector memory traffic in the inner loop.  A wave covers either the
// bounding rectangle of its targets' (2K+1)^2 neighbourhoods, each lane
// masked to its own neighbourhood, or each distinct target box in turn,
// whichever visits fewer boxes.  Targets sorted by box (Morton order) keep a
// wave within one or two adjacent boxes, where the rectangle costs about 6%
// over the lanes' own neighbourhoods.
#include <cmath>

#include "fgt2d.h"
#include "fmm2d_internal.h"

namespace fmm2d {

namespace {

// ------------------------------------------------------- coefficients --

// A[box][a][b] = 1/(a! b!) sum_j q_j s1^a s2^b, s = (x_j - s_B) / (sqrt(2) sigma):
// one thread per (box, a), FP64 sums rounded once.
template <int P>
__global__ __launch_bounds__(256) void fgt_coeffs_kernel(const float2 *__restrict__ xy, const float *__restrict__ q,
                                                         const int32_t *__restrict__ ls, int depth, double scale,
                                                         float *__restrict__ A) {
  const int64_t nbox = int64_t(1) << (2 * depth);
  const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (e >= nbox * P) return;
  const int64_t m = e / P;
  const int a = int(e - m * P);
  uint32_t bx, by;
  unmorton2(uint32_t(m), bx, by);
  const double w = ldexp(1.0, -depth);
  const double c1 = (double(bx) + 0.5) * w, c2 = (double(by) + 0.5) * w;
  double acc[P];
#pragma unroll
  for (int b = 0; b < P; ++b) acc[b] = 0.0;
  for (int32_t j = ls[m]; j < ls[m + 1]; ++j) {
    const float2 x = xy[j];
    const double s1 = (double(x.x) - c1) * scale, s2 = (double(x.y) - c2) * scale;
    double pa = double(q[j]);  // q s1^a
    for (int i = 0; i < a; ++i) pa *= s1;
    double pb = pa;  // q s1^a s2^b
#pragma unroll
    for (int b = 0; b < P; ++b) {
      acc[b] += pb;
      pb *= s2;
    }
  }
  double fa = 1.0;  // a!
  for (int i = 2; i <= a; ++i) fa *= double(i);
  float *out = A + (m * P + a) * P;
  double fb = 1.0;  // b!
#pragma unroll
  for (int b = 0; b < P; ++b) {
    if (b >= 2) fb *= double(b);
    out[b] = float(acc[b] / (fa * fb));
  }
}

// --------------------------------------------------------- evaluation --

// h_n(t) = exp(-t^2) H_n(t) for n < P by H_{n+1} = 2t H_n - 2n H_{n-1}, with
// e = exp(-t^2) already applied (zero masks the lane).
template <int P>
__device__ __forceinline__ void hermite_fns(float t, float e, float (&h)[P]) {
  const float tt = 2.f * t;
  h[0] = e;
  if (P > 1) h[1] = tt * e;
#pragma unroll
  for (int n = 1; n + 1 < P; ++n) h[n + 1] = fmaf(tt, h[n], -2.f * float(n) * h[n - 1]);
}

__device__ __forceinline__ float gauss(float t) { return __expf(-t * t); }

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m));
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m));
  return __builtin_amdgcn_readfirstlane(v);
}

// acc += sum_a h1[a] sum_b Ab[a][b] h2[b]; Ab is wave-uniform.
template <int P>
__device__ __forceinline__ float bilinear(const float *__restrict__ Ab, const float (&h1)[P], const float (&h2)[P],
                                          float acc) {
#pragma unroll
  for (int a = 0; a < P; ++a) {
    float v = 0.f;
#pragma unroll
    for (int b = 0; b < P; ++b) v = fmaf(Ab[a * P + b], h2[b], v);
    acc = fmaf(h1[a], v, acc);
  }
  return acc;
}

// Box columns per strip of the sweep: h1 of a strip's columns stays in
// registers while the rows go by, so h1 is formed once per column and h2
// once per strip and row, against h1 once per box.  For p >= 10 the
// strips were slower (8.9-9.3 ms against 8.3 ms at p = 12, 6.5M targets):
// a box's p^2 coefficients then fill the scalar registers and the unrolled
// strip holds back their loads, so those orders sweep box by box (1).
template <int P>
constexpr int kStrip = P <= 9 ? 4 : 1;

// Sum over boxes (i, j), x0 <= i <= x1, y0 <= j <= y1 (all wave-uniform);
// a lane takes box (i, j) only if |i - bx| <= K and |j - by| <= K and sel.
template <int P>
__device__ __forceinline__ float sweep(const float *__restrict__ A, float2 y, int bx, int by, bool sel, int K,
                                       int x0, int x1, int y0, int y1, float wb, float inv_s, float acc) {
  constexpr int W = kStrip<P>;
  if constexpr (W == 1) {
    for (int j = y0; j <= y1; ++j) {
      const float t2 = (y.y - (float(j) + 0.5f) * wb) * inv_s;
      const bool row = sel && abs(j - by) <= K;
      float h2[P];
      hermite_fns<P>(t2, row ? gauss(t2) : 0.f, h2);
      for (int i = x0; i <= x1; ++i) {
        const float t1 = (y.x - (float(i) + 0.5f) * wb) * inv_s;
        const bool in = abs(i - bx) <= K;
        float h1[P];
        hermite_fns<P>(t1, in ? gauss(t1) : 0.f, h1);
        const float *Ab = A + int64_t(morton2(uint32_t(i), uint32_t(j))) * (P * P);
        acc = bilinear<P>(Ab, h1, h2, acc);
      }
    }
    return acc;
  }
  for (int i0 = x0; i0 <= x1; i0 += W) {
    float h1[W][P];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int i = i0 + w;  // past x1: never used
      const float t1 = (y.x - (float(i) + 0.5f) * wb) * inv_s;
      const bool in = abs(i - bx) <= K;
      hermite_fns<P>(t1, in ? gauss(t1) : 0.f, h1[w]);
    }
    for (int j = y0; j <= y1; ++j) {
      const float t2 = (y.y - (float(j) + 0.5f) * wb) * inv_s;
      const bool row = sel && abs(j - by) <= K;
      float h2[P];
      hermite_fns<P>(t2, row ? gauss(t2) : 0.f, h2);
#pragma unroll
      for (int w = 0; w < W; ++w) {
        if (i0 + w > x1) break;  // wave-uniform: no coefficients past the rectangle
        const float *Ab = A + int64_t(morton2(uint32_t(i0 + w), uint32_t(j))) * (P * P);
        acc = bilinear<P>(Ab, h1[w], h2, acc);
      }
    }
  }
  return acc;
}

template <int P>
__global__ __launch_bounds__(256) void fgt_eval_kernel(const float2 *__restrict__ txy, int64_t nt, int depth,
                                                       float inv_s, int K, const float *__restrict__ A,
                                                       float *__restrict__ G) {
  // Blocks are dispatched to the 8 XCDs in turn (b mod 8).  Each XCD takes a
  // contiguous eighth of the (box-ordered) targets, so the coefficient boxes
  // that neighbouring waves visit are fetched once into that XCD's L2.
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t lb = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int64_t t0 = (lb * 4 + (threadIdx.x >> 6)) * 64;
  if (t0 >= nt) return;  // whole wave
  const int lane = threadIdx.x & 63;
  const int64_t t = t0 + lane;
  const bool act = t < nt;
  const float2 y = txy[act ? t : t0];  // idle lanes follow lane 0's target
  const int side = 1 << depth;
  const float fs = float(side), wb = 1.f / fs;  // exact powers of two
  // box of the target, clamped (fminf/fmaxf also map NaN into the grid)
  const int bx = int(fminf(fmaxf(floorf(y.x * fs), 0.f), fs - 1.f));
  const int by = int(fminf(fmaxf(floorf(y.y * fs), 0.f), fs - 1.f));

  // option 1: the bounding rectangle of the wave's neighbourhoods
  const int x0 = max(wave_min(bx) - K, 0), x1 = min(wave_max(bx) + K, side - 1);
  const int y0 = max(wave_min(by) - K, 0), y1 = min(wave_max(by) + K, side - 1);
  const int64_t rect = int64_t(x1 - x0 + 1) * (y1 - y0 + 1);
  // option 2: each distinct target box with its own clipped neighbourhood
  const int key = bx | (by << 16);
  int64_t per_box = 0;
  uint64_t left = __ballot(1);
  while (left) {
    const int k = __builtin_amdgcn_readfirstlane(__shfl(key, __ffsll(static_cast<long long>(left)) - 1));
    const int kx = k & 0xffff, ky = k >> 16;
    per_box += int64_t(min(kx + K, side - 1) - max(kx - K, 0) + 1) * (min(ky + K, side - 1) - max(ky - K, 0) + 1);
    left &= ~__ballot(key == k);
  }

  float acc = 0.f;
  if (rect <= per_box) {
    acc = sweep<P>(A, y, bx, by, true, K, x0, x1, y0, y1, wb, inv_s, acc);
  } else {
    left = __ballot(1);
    while (left) {
      const int k = __builtin_amdgcn_readfirstlane(__shfl(key, __ffsll(static_cast<long long>(left)) - 1));
      const int kx = k & 0xffff, ky = k >> 16;
      acc = sweep<P>(A, y, bx, by, key == k, K, max(kx - K, 0), min(kx + K, side - 1), max(ky - K, 0),
                     min(ky + K, side - 1), wb, inv_s, acc);
      left &= ~__ballot(key == k);
    }
  }
  if (act) G[t] = acc;
}

inline unsigned blocks_of(int64_t work) { return unsigned((work + 255) / 256); }

template <int P>
void launch_coeffs_p(const float *xy, const float *q, const int32_t *ls, int depth, double scale, float *A,
                     hipStream_t s) {
  const int64_t work = (int64_t(1) << (2 * depth)) * P;
  hipLaunchKernelGGL(fgt_coeffs_kernel<P>, dim3(blocks_of(work)), dim3(256), 0, s,
                     reinterpret_cast<const float2 *>(xy), q, ls, depth, scale, A);
}

template <int P>
void launch_eval_p(const float *txy, int64_t nt, int depth, float inv_s, int K, const float *A, float *G,
                   hipStream_t s) {
  hipLaunchKernelGGL(fgt_eval_kernel<P>, dim3(blocks_of(nt)), dim3(256), 0, s,
                     reinterpret_cast<const float2 *>(txy), nt, depth, inv_s, K, A, G);
}

#define FGT_FOR_EACH_P(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

int check_fgt_common(const char *fn, int depth, int p, float sigma) {
  if (depth < 0 || depth > kMaxDepth) return set_error(FMM2D_EDEPTH, "%s: depth %d outside 0..%d", fn, depth, kMaxDepth);
  if (p < 1 || p > FGT2D_MAX_P) return set_error(FMM2D_EUNSUPPORTED_P, "%s: p = %d outside 1..%d", fn, p, FGT2D_MAX_P);
  if (!(sigma > 0.f) || !std::isfinite(sigma)) return set_error(FMM2D_EINVAL, "%s: sigma must be finite and > 0", fn);
  return FMM2D_OK;
}

}  // namespace

}  // namespace fmm2d

using namespace fmm2d;

extern "C" {

int fgt2d_hermite_coeffs(const float *xy_sorted, const float *q_sorted, const int32_t *leaf_start, int depth, int p,
                         float sigma, float *A, hipStream_t stream) {
  const char *fn = "fgt2d_hermite_coeffs";
  clear_error();
  const int rc = check_fgt_common(fn, depth, p, sigma);
  if (rc != FMM2D_OK) return rc;
  if (!xy_sorted || !q_sorted || !leaf_start || !A) return set_error(FMM2D_EINVAL, "%s: NULL pointer", fn);
  const double scale = 1.0 / (std::sqrt(2.0) * double(sigma));
  switch (p) {
#define X(P_) \
  case P_: launch_coeffs_p<P_>(xy_sorted, q_sorted, leaf_start, depth, scale, A, stream); break;
    FGT_FOR_EACH_P(X)
#undef X
  }
  return check_launch(fn);
}

int fgt2d_hermite_eval(const float *txy, int64_t nt, int depth, int p, float sigma, int K, const float *A, float *G,
                       hipStream_t stream) {
  const char *fn = "fgt2d_hermite_eval";
  clear_error();
  const int rc = check_fgt_common(fn, depth, p, sigma);
  if (rc != FMM2D_OK) return rc;
  if (nt < 0 || nt >= (int64_t(1) << 31)) return set_error(FMM2D_EINVAL, "%s: nt out of range", fn);
  if (K < 0 || K >= (1 << depth))
    return set_error(FMM2D_EINVAL, "%s: K = %d outside 0..%d", fn, K, (1 << depth) - 1);
  if (!A) return set_error(FMM2D_EINVAL, "%s: A is NULL", fn);
  if (nt == 0) return FMM2D_OK;
  if (!txy || !G) return set_error(FMM2D_EINVAL, "%s: NULL pointer", fn);
  const float inv_s = float(1.0 / (std::sqrt(2.0) * double(sigma)));
  switch (p) {
#define X(P_) \
  case P_: launch_eval_p<P_>(txy, nt, depth, inv_s, K, A, G, stream); break;
    FGT_FOR_EACH_P(X)
#undef X
  }
  return check_launch(fn);
}

}  // extern "C"
