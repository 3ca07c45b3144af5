// The log-potential row of the M2L for the forms that do not produce it in
// their own products (p = 16 in FP32; p = 8, 16 in split precision; every p
// in the Hankel form):
//   b(t) = sum_{o in O_c(t)} [ r_o . M~(t + o) + log(h) M~_0(t + o) ],
// the constant term the complex logarithm adds to Eq. (eq:M2Lmat)'s local
// expansion.  One workgroup per 8x8 target tile stages the 12x12 source block
// and the 49 log-row slots in LDS as float4 chunks (two coefficients each);
// four lanes share a target box, each summing a quarter of the k range over
// the box's 27 offsets with float4 reads, then reduce with lane shuffles.
// Vector-ALU work of 1/p of the M2L itself.  Its transpose (below) adds the
// row's contribution to the adjoint's gM~.
#include "fmm2d_internal.h"
#include "m2l_bank.h"
#include "m2l_common.h"

namespace fmm2d {

template <int P>
__global__ __launch_bounds__(256) void m2l_logrow_fwd_kernel(const float2 *__restrict__ X, float2 *__restrict__ bout,
                                                             const float2 *__restrict__ rsrc, TileMap map) {
  constexpr int C4 = P / 2;   // float4 chunks of a box record; lane g takes chunks g, g + 4, ...
  constexpr int kStride = C4 + 1;  // padded box stride: boxes read together spread over the banks
  __shared__ float4 lx[kRegBoxes * kStride];
  __shared__ float4 lr[kSlots * C4];
  const int tid = threadIdx.x;

  int level, tile;
  tile_of(map, blockIdx.x, level, tile);
  const int nside = 1 << level;
  uint32_t tX, tY;
  unmorton2(uint32_t(tile), tX, tY);
  const int X0 = int(tX) * kTile, Y0 = int(tY) * kTile;
  const int64_t off = level_off(level);

  const float4 *r4 = reinterpret_cast<const float4 *>(rsrc);
  for (int e = tid; e < kSlots * C4; e += 256) lr[e] = r4[e];
  for (int e = tid; e < kRegBoxes * C4; e += 256) {
    const int rb = e / C4, c = e % C4;
    const int gx = X0 - kHalo + rb % kReg, gy = Y0 - kHalo + rb / kReg;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (gx >= 0 && gy >= 0 && gx < nside && gy < nside)
      v = reinterpret_cast<const float4 *>(X + (off + morton2(uint32_t(gx), uint32_t(gy))) * P)[c];
    lx[rb * kStride + c] = v;
  }
  __syncthreads();

  const int box = tid >> 2, g = tid & 3;  // 64 target boxes x 4 k groups
  const int tx = box & 7, ty = box >> 3;
  const int sx = 1 - 2 * (tx & 1), sy = 1 - 2 * (ty & 1);
  float br = 0.f, bi = 0.f, s0r = 0.f, s0i = 0.f;
#pragma unroll 3
  for (int q = 0; q < 27; ++q) {
    const int ox = sx * kOff00.ox[q], oy = sy * kOff00.oy[q];
    const int rb = (ty + kHalo + oy) * kReg + (tx + kHalo + ox);
    const float4 *m4 = lx + rb * kStride;
    const float4 *v4 = lr + slot_of(ox, oy) * C4;
#pragma unroll
    for (int h0 = 0; h0 < C4; h0 += 4) {
      const int h = h0 + g;
      if (h < C4) {
        const float4 m = m4[h], rv = v4[h];
        br += rv.x * m.x - rv.y * m.y + rv.z * m.z - rv.w * m.w;
        bi += rv.x * m.y + rv.y * m.x + rv.z * m.w + rv.w * m.z;
        if (h == 0) {  // k = 0 for lane g = 0, the only lane whose sum is used
          s0r += m.x;
          s0i += m.y;
        }
      }
    }
  }
  br += __shfl_xor(br, 1);
  bi += __shfl_xor(bi, 1);
  br += __shfl_xor(br, 2);
  bi += __shfl_xor(bi, 2);
  const int gx = X0 + tx, gy = Y0 + ty;
  if (g == 0 && gx < nside && gy < nside) {
    const float logh = -float(level) * 0.69314718055994530942f;
    bout[off + morton2(uint32_t(gx), uint32_t(gy))] = make_float2(br + logh * s0r, bi + logh * s0i);
  }
}

int launch_m2l_logrow_fwd(const float *M, float *b, int p, int lmin, int lmax, const float *r, hipStream_t s) {
  const TileMap map = make_tile_map(lmin, lmax);
  const int ntiles = map.first[map.nlev];
  const float2 *X = reinterpret_cast<const float2 *>(M);
  float2 *bo = reinterpret_cast<float2 *>(b);
  const float2 *rs = reinterpret_cast<const float2 *>(r);
  switch (p) {
    case 8: hipLaunchKernelGGL(m2l_logrow_fwd_kernel<8>, dim3(ntiles), dim3(256), 0, s, X, bo, rs, map); break;
    case 12: hipLaunchKernelGGL(m2l_logrow_fwd_kernel<12>, dim3(ntiles), dim3(256), 0, s, X, bo, rs, map); break;
    case 16: hipLaunchKernelGGL(m2l_logrow_fwd_kernel<16>, dim3(ntiles), dim3(256), 0, s, X, bo, rs, map); break;
    case 20: hipLaunchKernelGGL(m2l_logrow_fwd_kernel<20>, dim3(ntiles), dim3(256), 0, s, X, bo, rs, map); break;
    default: return set_error(FMM2D_EINVAL, "internal: log-row pass for p = %d", p);
  }
  return check_launch("m2l log row");
}

// Transpose of the log row, added to the adjoint's output: for every source
// box s of levels lmin..lmax,
//   gM~_k(s) += sum_{o in O_c(s)} r_k(+o) gb(s + o)   (+ log(h) sum_o gb(s + o) at k = 0),
// gathered over s's own list (s is in IL(t) exactly when t is in IL(s)), with
// the row at d = +o read from the forward table at the mirrored slot.  One
// workgroup per 8x8 source tile; one lane per (box, k).
template <int P>
__global__ __launch_bounds__(256) void m2l_logrow_bwd_kernel(const float2 *__restrict__ gb, float2 *__restrict__ gM,
                                                             const float2 *__restrict__ rsrc, TileMap map) {
  __shared__ float2 lg[kRegBoxes];
  __shared__ float2 lr[kSlots * P];
  const int tid = threadIdx.x;
  int level, tile;
  tile_of(map, blockIdx.x, level, tile);
  const int nside = 1 << level;
  uint32_t tX, tY;
  unmorton2(uint32_t(tile), tX, tY);
  const int X0 = int(tX) * kTile, Y0 = int(tY) * kTile;
  const int64_t off = level_off(level);
  for (int e = tid; e < kSlots * P; e += 256) lr[e] = rsrc[e];
  for (int e = tid; e < kRegBoxes; e += 256) {
    const int gx = X0 - kHalo + e % kReg, gy = Y0 - kHalo + e / kReg;
    float2 v = make_float2(0.f, 0.f);
    if (gx >= 0 && gy >= 0 && gx < nside && gy < nside) v = gb[off + morton2(uint32_t(gx), uint32_t(gy))];
    lg[e] = v;
  }
  __syncthreads();
  const float logh = -float(level) * 0.69314718055994530942f;
  for (int e = tid; e < 64 * P; e += 256) {
    const int box = e / P, k = e % P;
    const int sxb = box & 7, syb = box >> 3;
    const int gx = X0 + sxb, gy = Y0 + syb;
    if (gx >= nside || gy >= nside) continue;
    const int sx = 1 - 2 * (sxb & 1), sy = 1 - 2 * (syb & 1);
    float ar = 0.f, ai = 0.f, sr = 0.f, si = 0.f;
#pragma unroll 3
    for (int q = 0; q < 27; ++q) {
      const int ox = sx * kOff00.ox[q], oy = sy * kOff00.oy[q];
      const float2 g = lg[(syb + kHalo + oy) * kReg + (sxb + kHalo + ox)];
      const float2 r = lr[slot_of(-ox, -oy) * P + k];
      ar += r.x * g.x - r.y * g.y;
      ai += r.x * g.y + r.y * g.x;
      sr += g.x;
      si += g.y;
    }
    if (k == 0) {
      ar += logh * sr;
      ai += logh * si;
    }
    float2 *dst = gM + (off + morton2(uint32_t(gx), uint32_t(gy))) * P + k;
    const float2 o = *dst;
    *dst = make_float2(o.x + ar, o.y + ai);
  }
}

int launch_m2l_logrow_bwd(const float *gb, float *gM, int p, int lmin, int lmax, const float *r, hipStream_t s) {
  const TileMap map = make_tile_map(lmin, lmax);
  const int ntiles = map.first[map.nlev];
  const float2 *G = reinterpret_cast<const float2 *>(gb);
  float2 *Y = reinterpret_cast<float2 *>(gM);
  const float2 *rs = reinterpret_cast<const float2 *>(r);
  switch (p) {
    case 8: hipLaunchKernelGGL(m2l_logrow_bwd_kernel<8>, dim3(ntiles), dim3(256), 0, s, G, Y, rs, map); break;
    case 12: hipLaunchKernelGGL(m2l_logrow_bwd_kernel<12>, dim3(ntiles), dim3(256), 0, s, G, Y, rs, map); break;
    case 16: hipLaunchKernelGGL(m2l_logrow_bwd_kernel<16>, dim3(ntiles), dim3(256), 0, s, G, Y, rs, map); break;
    case 20: hipLaunchKernelGGL(m2l_logrow_bwd_kernel<20>, dim3(ntiles), dim3(256), 0, s, G, Y, rs, map); break;
    default: return set_error(FMM2D_EINVAL, "internal: log-row transpose for p = %d", p);
  }
  return check_launch("m2l log row (transpose)");
}

}  // namespace fmm2d
