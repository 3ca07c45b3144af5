// Near field (Sec. 2.1, stage 5): direct interactions with the 3x3 block of
// leaves around each target's leaf, and the transpose for gradients, in FP32
// arithmetic.  The forward pass runs one wave per target leaf, the transpose
// one wave per source leaf.
#include "fmm2d_internal.h"

namespace fmm2d {

// atan2(y, x) for (x, y) != (0, 0): octant reduction to a = min/max in
// [0, 1] and atan(a) = a P(a^2), P the degree-7 minimax polynomial (Remez
// exchange on the odd basis a^(2j+1); fit_atan.py beside this file computes
// the coefficients): largest error 3.7e-8 in exact arithmetic, 1.5e-7
// evaluated in FP32.  Principal branch, (-pi, pi].
__device__ inline float atan2_p2p(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float a = mn * __builtin_amdgcn_rcpf(mx);
  const float t = a * a;
  float r = -0.004054567310959101f;
  r = fmaf(r, t, 0.021862957626581192f);
  r = fmaf(r, t, -0.0559123270213604f);
  r = fmaf(r, t, 0.0964219719171524f);
  r = fmaf(r, t, -0.1390862911939621f);
  r = fmaf(r, t, 0.19946566224098206f);
  r = fmaf(r, t, -0.33329859375953674f);
  r = fmaf(r, t, 0.9999993443489075f);
  r *= a;
  if (ay > ax) r = 1.57079632679f - r;
  if (x < 0.f) r = 3.14159265359f - r;
  return copysignf(r, y);
}

// Lanes of one wave over a chunk of `cnt` (1..64) items (targets of the
// forward pass, sources of the transpose), each summed over the other side in
// nph = 64 / cnt phases: lane = ph * cnt + i, and lanes past nph * cnt idle.
struct ChunkLanes {
  int cnt, nph, i, ph;
  __device__ ChunkLanes(int c, int lane) : cnt(c), nph(64 / c), i(lane % c), ph(lane / c) {}
  __device__ bool active() const { return ph < nph; }
};

// Sum over the phases of a chunk, in a fixed tree order: lane (i, 0) ends
// with the total of lanes (i, 0 .. nph-1).
__device__ inline float phase_sum(float v, const ChunkLanes &c, int lane) {
  int m = 1;
  while (2 * m < c.nph) m <<= 1;
  for (; m >= 1; m >>= 1) {
    const float o = __shfl(v, lane + m * c.cnt);
    if (c.ph < m && c.ph + m < c.nph) v += o;
  }
  return v;
}

// One wave per target leaf.  Targets go in chunks of up to 64; the lanes of a
// chunk of n targets are split into n targets x 64 / n source phases: lane
// (i, ph) sums sources ph, ph + nph, ... of each of the 3x3 neighbour leaves
// for target i, and the phases are then combined in a fixed order.  The
// sources of a neighbour leaf pass through the wave's own slice of LDS, 64 at
// a time (one coalesced load per array), and the lanes read them from there:
// a global load per pair would cost each pair a trip through the vector
// memory path.  Only the target's own leaf can hold a source at the target's
// position; that pair is skipped.
template <bool PHI, bool FIELD>
__global__ __launch_bounds__(256) void p2p_kernel(const float2 *__restrict__ xy, const float *__restrict__ q,
                                                  const int32_t *__restrict__ ls, const float2 *__restrict__ txy,
                                                  const int32_t *__restrict__ tls, int depth,
                                                  float2 *__restrict__ phi, float2 *__restrict__ field) {
  __shared__ float4 stage[4][64];  // per wave: (x, y, q, -) of up to 64 sources
  const int64_t nleaf = int64_t(1) << (2 * depth);
  const int wave = threadIdx.x >> 6;
  const int64_t leaf = blockIdx.x * int64_t(4) + wave;
  if (leaf >= nleaf) return;
  const int lane = threadIdx.x & 63;
  const int32_t t0 = tls[leaf], nt = tls[leaf + 1] - t0;
  if (nt <= 0) return;
  uint32_t ix, iy;
  unmorton2(uint32_t(leaf), ix, iy);
  const int side = 1 << depth;
  int32_t sb[9], se[9];  // source ranges of the 3x3 neighbourhood (empty outside the grid)
#pragma unroll
  for (int d = 0; d < 9; ++d) {
    const int sx = int(ix) + d % 3 - 1, sy = int(iy) + d / 3 - 1;
    const bool in = sx >= 0 && sy >= 0 && sx < side && sy < side;
    const uint32_t sm = in ? morton2(uint32_t(sx), uint32_t(sy)) : 0u;
    sb[d] = in ? ls[sm] : 0;
    se[d] = in ? ls[sm + 1] : 0;
  }
  float4 *st = stage[wave];
  constexpr float kHalfLn2 = 0.346573590279972654709f;  // log(r2) / 2 = kHalfLn2 log2(r2)
  for (int32_t c0 = 0; c0 < nt; c0 += 64) {
    const ChunkLanes cl(nt - c0 < 64 ? nt - c0 : 64, lane);
    const int32_t t = t0 + c0 + cl.i;
    const bool act = cl.active();
    const int ph = act ? cl.ph : 0, nph = cl.nph;
    const float2 z = txy[t];
    float pr = 0.f, pi = 0.f, fr = 0.f, fi = 0.f;
#pragma unroll
    for (int d = 0; d < 9; ++d) {
      for (int32_t b0 = sb[d]; b0 < se[d]; b0 += 64) {  // the same trip count in every lane
        const int m = se[d] - b0 < 64 ? se[d] - b0 : 64;
        if (lane < m) {
          const float2 zs = xy[b0 + lane];
          st[lane] = make_float4(zs.x, zs.y, q[b0 + lane], 0.f);
        }
        __builtin_amdgcn_wave_barrier();
        for (int k = act ? ph : m; k < m; k += nph) {
          const float4 sv = st[k];
          const float rx = z.x - sv.x, ry = z.y - sv.y;
          const float r2 = fmaf(rx, rx, ry * ry);
          float qs = sv.z, r2s = r2, ax = rx;
          if (d == 4) {  // own leaf: a coincident pair is skipped
            const bool self = r2 == 0.f;
            qs = self ? 0.f : qs;
            r2s = self ? 1.f : r2;
            ax = self ? 1.f : rx;
          }
          if (PHI) {
            pr = fmaf(qs, __builtin_amdgcn_logf(r2s), pr);  // hardware log2
            pi = fmaf(qs, atan2_p2p(ry, ax), pi);
          }
          if (FIELD) {
            const float inv = qs * __builtin_amdgcn_rcpf(r2s);  // hardware reciprocal (1 ulp)
            fr = fmaf(inv, rx, fr);
            fi = fmaf(-inv, ry, fi);
          }
        }
        // every lane's reads of this batch are issued before the next
        // batch's writes (the wave's LDS accesses complete in order)
        __builtin_amdgcn_wave_barrier();
      }
    }
    if (nph > 1) {  // combine the phases: lane ph = 0 ends with the total
      if (PHI) {
        pr = phase_sum(pr, cl, lane);
        pi = phase_sum(pi, cl, lane);
      }
      if (FIELD) {
        fr = phase_sum(fr, cl, lane);
        fi = phase_sum(fi, cl, lane);
      }
    }
    if (act && cl.ph == 0) {
      if (PHI) {
        const float2 o = phi[t];
        phi[t] = make_float2(o.x + kHalfLn2 * pr, o.y + pi);
      }
      if (FIELD) {
        const float2 o = field[t];
        field[t] = make_float2(o.x + fr, o.y + fi);
      }
    }
  }
}

// P2P^T with the same layout: one wave per source leaf, sources in chunks of
// up to 64, each chunk's lanes split into sources x target phases over the
// 3x3 neighbour leaves, the targets (positions and cotangents) passing
// through the wave's LDS slice 64 at a time.  For the pair r = z_t - z_s and
// cotangents (c, e) of (phi, field) at target t:
//   dq_s += Re(c log r) + Re(e / r),   G_s += q_s (-c / r + e / r^2),
// G_s being conj of the position gradient packed as dRe + i dIm.
template <bool CPHI, bool CF>
__global__ __launch_bounds__(256) void p2p_backward_kernel(const float2 *__restrict__ xy, const float *__restrict__ q,
                                                           const int32_t *__restrict__ ls,
                                                           const float2 *__restrict__ txy,
                                                           const int32_t *__restrict__ tls, int depth,
                                                           const float2 *__restrict__ cphi,
                                                           const float2 *__restrict__ cfield, float *__restrict__ gq,
                                                           float2 *__restrict__ G) {
  // per wave, up to 64 targets: (x, y, and the cotangent of phi, or of the
  // field when phi has none), and the field's when both are present
  __shared__ float4 stage[4][64];
  __shared__ float2 stage2[4][CPHI && CF ? 64 : 1];
  const int64_t nleaf = int64_t(1) << (2 * depth);
  const int wave = threadIdx.x >> 6;
  const int64_t leaf = blockIdx.x * int64_t(4) + wave;
  if (leaf >= nleaf) return;
  const int lane = threadIdx.x & 63;
  const int32_t s0 = ls[leaf], ns = ls[leaf + 1] - s0;
  if (ns <= 0) return;
  uint32_t ix, iy;
  unmorton2(uint32_t(leaf), ix, iy);
  const int side = 1 << depth;
  int32_t tb[9], te[9];  // target ranges of the 3x3 neighbourhood (empty outside the grid)
#pragma unroll
  for (int d = 0; d < 9; ++d) {
    const int tx = int(ix) + d % 3 - 1, ty = int(iy) + d / 3 - 1;
    const bool in = tx >= 0 && ty >= 0 && tx < side && ty < side;
    const uint32_t tm = in ? morton2(uint32_t(tx), uint32_t(ty)) : 0u;
    tb[d] = in ? tls[tm] : 0;
    te[d] = in ? tls[tm + 1] : 0;
  }
  float4 *st = stage[wave];
  float2 *st2 = stage2[wave];
  constexpr float kHalfLn2 = 0.346573590279972654709f;  // log(r2) / 2 = kHalfLn2 log2(r2)
  for (int32_t c0 = 0; c0 < ns; c0 += 64) {
    const ChunkLanes cl(ns - c0 < 64 ? ns - c0 : 64, lane);
    const int32_t sidx = s0 + c0 + cl.i;
    const bool act = cl.active();
    const int ph = act ? cl.ph : 0, nph = cl.nph;
    const float2 zs = xy[sidx];
    float alog = 0.f, aang = 0.f, aq = 0.f, gr = 0.f, gi = 0.f;
#pragma unroll
    for (int d = 0; d < 9; ++d) {
      for (int32_t b0 = tb[d]; b0 < te[d]; b0 += 64) {  // the same trip count in every lane
        const int m = te[d] - b0 < 64 ? te[d] - b0 : 64;
        if (lane < m) {
          const float2 z = txy[b0 + lane];
          const float2 c = CPHI ? cphi[b0 + lane] : cfield[b0 + lane];
          st[lane] = make_float4(z.x, z.y, c.x, c.y);
          if (CPHI && CF) st2[lane] = cfield[b0 + lane];
        }
        __builtin_amdgcn_wave_barrier();
        for (int k = act ? ph : m; k < m; k += nph) {
          const float4 tv = st[k];
          const float2 e0 = CPHI && CF ? st2[k] : make_float2(tv.z, tv.w);
          const float rx = tv.x - zs.x, ry = tv.y - zs.y;
          const float r2 = fmaf(rx, rx, ry * ry);
          // own leaf: a coincident pair is skipped
          const bool self = d == 4 && r2 == 0.f;
          const float r2s = self ? 1.f : r2;
          const float inv = __builtin_amdgcn_rcpf(r2s);
          const float ir = rx * inv, ii = -ry * inv;  // 1/r
          // G_s gathers (-c + e / r) / r: w = -c + e / r, then w times 1/r
          float wr = 0.f, wi = 0.f, cy = 0.f;
          if (CPHI) {
            const float cx = self ? 0.f : tv.z;
            cy = self ? 0.f : tv.w;
            alog = fmaf(cx, __builtin_amdgcn_logf(r2s), alog);  // hardware log2
            wr = -cx;
            wi = -cy;
          }
          if (CF) {
            const float ex = self ? 0.f : e0.x, ey = self ? 0.f : e0.y;
            const float ur = fmaf(ex, ir, -ey * ii), ui = fmaf(ex, ii, ey * ir);  // e / r
            aq += ur;
            wr += ur;
            wi += ui;
          }
          gr = fmaf(wr, ir, fmaf(-wi, ii, gr));
          gi = fmaf(wr, ii, fmaf(wi, ir, gi));
          // Re(c log r) needs the angle of r only for a cotangent with an
          // imaginary part (a loss on Im phi); for the common real one (a
          // loss on Re phi) it is skipped whenever no active lane has one
          if (CPHI && __ballot(cy != 0.f) != 0ull) aang = fmaf(cy, atan2_p2p(ry, self ? 1.f : rx), aang);
        }
        // every lane's reads of this batch are issued before the next
        // batch's writes (the wave's LDS accesses complete in order)
        __builtin_amdgcn_wave_barrier();
      }
    }
    if (nph > 1) {  // combine the phases: lane ph = 0 ends with the total
      if (CPHI) {
        alog = phase_sum(alog, cl, lane);
        aang = phase_sum(aang, cl, lane);
      }
      if (CF) aq = phase_sum(aq, cl, lane);
      gr = phase_sum(gr, cl, lane);
      gi = phase_sum(gi, cl, lane);
    }
    if (act && cl.ph == 0) {
      const float qs = q[sidx];
      gq[sidx] += fmaf(kHalfLn2, alog, aq) - aang;
      const float2 o = G[sidx];
      G[sidx] = make_float2(fmaf(qs, gr, o.x), fmaf(qs, gi, o.y));
    }
  }
}

int launch_p2p(const float *xy, const float *q, const int32_t *ls, const float *txy, const int32_t *tls,
                 int64_t nt, int depth, float *phi, float *field, hipStream_t s) {
  if (nt == 0 || (!phi && !field)) return FMM2D_OK;
  const int64_t nleaf = int64_t(1) << (2 * depth);
  const dim3 grid(unsigned((nleaf + 3) / 4)), block(256);
  auto X = reinterpret_cast<const float2 *>(xy);
  auto T = reinterpret_cast<const float2 *>(txy);
  auto Ph = reinterpret_cast<float2 *>(phi);
  auto F = reinterpret_cast<float2 *>(field);
  if (phi && field) hipLaunchKernelGGL((p2p_kernel<true, true>), grid, block, 0, s, X, q, ls, T, tls, depth, Ph, F);
  else if (phi) hipLaunchKernelGGL((p2p_kernel<true, false>), grid, block, 0, s, X, q, ls, T, tls, depth, Ph, F);
  else hipLaunchKernelGGL((p2p_kernel<false, true>), grid, block, 0, s, X, q, ls, T, tls, depth, Ph, F);
  return check_launch("p2p");
}

int launch_p2p_backward(const float *xy, const float *q, const int32_t *ls, int64_t n, const float *txy,
                          const int32_t *tls, int depth, const float *cphi, const float *cfield, float *gq, float *G,
                          hipStream_t s) {
  if (n == 0 || (!cphi && !cfield)) return FMM2D_OK;
  const int64_t nleaf = int64_t(1) << (2 * depth);
  const dim3 grid(unsigned((nleaf + 3) / 4)), block(256);
  auto X = reinterpret_cast<const float2 *>(xy);
  auto T = reinterpret_cast<const float2 *>(txy);
  auto C = reinterpret_cast<const float2 *>(cphi);
  auto E = reinterpret_cast<const float2 *>(cfield);
  auto Go = reinterpret_cast<float2 *>(G);
  if (cphi && cfield)
    hipLaunchKernelGGL((p2p_backward_kernel<true, true>), grid, block, 0, s, X, q, ls, T, tls, depth, C, E, gq, Go);
  else if (cphi)
    hipLaunchKernelGGL((p2p_backward_kernel<true, false>), grid, block, 0, s, X, q, ls, T, tls, depth, C, E, gq, Go);
  else
    hipLaunchKernelGGL((p2p_backward_kernel<false, true>), grid, block, 0, s, X, q, ls, T, tls, depth, C, E, gq, Go);
  return check_launch("p2p_backward");
}

}  // namespace fmm2d
