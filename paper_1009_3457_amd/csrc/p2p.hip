// Near field (Sec. 2.1, stage 5): direct interactions with the 3x3 block of
// leaves around each target's leaf, and the transpose for gradients.  One
// thread per target (per source for the transpose), FP32 arithmetic.
#include "fmm2d_internal.h"

namespace fmm2d {

__device__ inline int64_t leaf_of_p2p(const int32_t *__restrict__ ls, int64_t nleaf, int64_t i) {
  int64_t lo = 0, hi = nleaf;  // invariant: ls[lo] <= i < ls[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (int64_t(ls[mid]) <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void p2p_kernel(const float2 *__restrict__ xy, const float *__restrict__ q, const int32_t *__restrict__ ls,
                           const float2 *__restrict__ txy, const int32_t *__restrict__ tls, int64_t nt, int depth,
                           float2 *__restrict__ phi, float2 *__restrict__ field) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int64_t nleaf = int64_t(1) << (2 * depth);
  if (t >= nt || t >= int64_t(tls[nleaf])) return;
  const int64_t m = leaf_of_p2p(tls, nleaf, t);
  uint32_t ix, iy;
  unmorton2(uint32_t(m), ix, iy);
  const int side = 1 << depth;
  const float2 z = txy[t];
  float pr = 0.f, pi = 0.f, fr = 0.f, fi = 0.f;
  for (int dy = -1; dy <= 1; ++dy) {
    const int sy = int(iy) + dy;
    if (sy < 0 || sy >= side) continue;
    for (int dx = -1; dx <= 1; ++dx) {
      const int sx = int(ix) + dx;
      if (sx < 0 || sx >= side) continue;
      const uint32_t sm = morton2(uint32_t(sx), uint32_t(sy));
      for (int32_t s = ls[sm]; s < ls[sm + 1]; ++s) {
        const float2 zs = xy[s];
        const float rx = z.x - zs.x, ry = z.y - zs.y;
        const float r2 = rx * rx + ry * ry;
        if (r2 == 0.f) continue;  // coincident pair
        const float qs = q[s];
        pr += qs * 0.5f * logf(r2);
        pi += qs * atan2f(ry, rx);
        const float inv = qs / r2;
        fr += inv * rx;
        fi -= inv * ry;
      }
    }
  }
  if (phi) {
    const float2 o = phi[t];
    phi[t] = make_float2(o.x + pr, o.y + pi);
  }
  if (field) {
    const float2 o = field[t];
    field[t] = make_float2(o.x + fr, o.y + fi);
  }
}

__global__ void p2p_backward_kernel(const float2 *__restrict__ xy, const float *__restrict__ q,
                                    const int32_t *__restrict__ ls, int64_t n, const float2 *__restrict__ txy,
                                    const int32_t *__restrict__ tls, int depth, const float2 *__restrict__ cphi,
                                    const float2 *__restrict__ cfield, float *__restrict__ gq,
                                    float2 *__restrict__ G) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int64_t nleaf = int64_t(1) << (2 * depth);
  if (i >= n || i >= int64_t(ls[nleaf])) return;
  const int64_t m = leaf_of_p2p(ls, nleaf, i);
  uint32_t ix, iy;
  unmorton2(uint32_t(m), ix, iy);
  const int side = 1 << depth;
  const float2 zs = xy[i];
  float aqr = 0.f, agr = 0.f, agi = 0.f;
  for (int dy = -1; dy <= 1; ++dy) {
    const int ty = int(iy) + dy;
    if (ty < 0 || ty >= side) continue;
    for (int dx = -1; dx <= 1; ++dx) {
      const int tx = int(ix) + dx;
      if (tx < 0 || tx >= side) continue;
      const uint32_t tm = morton2(uint32_t(tx), uint32_t(ty));
      for (int32_t t = tls[tm]; t < tls[tm + 1]; ++t) {
        const float2 z = txy[t];
        const float rx = z.x - zs.x, ry = z.y - zs.y;  // r = z_t - z_s
        const float r2 = rx * rx + ry * ry;
        if (r2 == 0.f) continue;
        const float ir = rx / r2, ii = -ry / r2;  // 1/r
        if (cphi) {
          const float2 c = cphi[t];
          const float lr = 0.5f * logf(r2), li = atan2f(ry, rx);
          aqr += c.x * lr - c.y * li;
          agr -= c.x * ir - c.y * ii;
          agi -= c.x * ii + c.y * ir;
        }
        if (cfield) {
          const float2 c = cfield[t];
          aqr += c.x * ir - c.y * ii;
          const float i2r = ir * ir - ii * ii, i2i = 2.f * ir * ii;  // 1/r^2
          agr += c.x * i2r - c.y * i2i;
          agi += c.x * i2i + c.y * i2r;
        }
      }
    }
  }
  const float qs = q[i];
  gq[i] += aqr;
  const float2 o = G[i];
  G[i] = make_float2(o.x + qs * agr, o.y + qs * agi);
}

int launch_p2p(const float *xy, const float *q, const int32_t *ls, const float *txy, const int32_t *tls,
                 int64_t nt, int depth, float *phi, float *field, hipStream_t s) {
  if (nt == 0) return FMM2D_OK;
  hipLaunchKernelGGL(p2p_kernel, dim3(unsigned((nt + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const float2 *>(xy), q, ls, reinterpret_cast<const float2 *>(txy), tls, nt,
                     depth, reinterpret_cast<float2 *>(phi), reinterpret_cast<float2 *>(field));
  return check_launch("p2p");
}

int launch_p2p_backward(const float *xy, const float *q, const int32_t *ls, int64_t n, const float *txy,
                          const int32_t *tls, int depth, const float *cphi, const float *cfield, float *gq, float *G,
                          hipStream_t s) {
  if (n == 0) return FMM2D_OK;
  hipLaunchKernelGGL(p2p_backward_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const float2 *>(xy), q, ls, n, reinterpret_cast<const float2 *>(txy), tls,
                     depth, reinterpret_cast<const float2 *>(cphi), reinterpret_cast<const float2 *>(cfield), gq,
                     reinterpret_cast<float2 *>(G));
  return check_launch("p2p_backward");
}

}  // namespace fmm2d
