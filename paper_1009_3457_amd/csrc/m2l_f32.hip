// FP32 M2L contraction with the fused reduction (Sec. 4.1, steps 2-3 of the
// downward sweep), and its adjoint, on gfx950 matrix cores.
//
// For every target box t of levels lmin..lmax (scaled basis, see fmm2d.h):
//   L~(t) = sum_{o in O_c(t)} A~_o M~(t + o),
//   b(t)  = sum_o [ r_o . M~(t + o) + log(h) M~_0(t + o) ].
// A workgroup of four waves owns an 8x8 target tile (m2l_common.h); wave w
// handles the 16 boxes of child class w.  For each of the class's 27 offsets
// the wave multiplies the offset's operator (rows = output orders n, 16 per
// M tile) by the 16 source expansions M~(t + o) (columns = boxes) with
// v_mfma_f32_16x16x4_f32, using Gauss's three real products per complex
// product (m2l_bank.h).  The source expansions of the whole tile are staged in
// LDS once and read by all 27 offsets of all four classes.  The reduction over
// the interaction list happens in the MFMA accumulators in a fixed offset
// order, so each L~(t) is written exactly once and results are reproducible.
// The log row b is a one-row product done on the vector ALU from the same
// staged operands, reduced across the four k-groups of a wave with lane
// shuffles.
//
// The adjoint uses the same stencil: since s in IL(t) <=> t in IL(s) and
// A~(d)^T = -A~(-d), the transpose gathers over s's own list with the
// negated forward operator of each offset; the log-row part becomes a rank-one
// update per offset with the row at d = +o.
#include "fmm2d_internal.h"
#include "m2l_bank.h"
#include "m2l_common.h"

namespace fmm2d {

typedef float f4_t __attribute__((ext_vector_type(4)));

template <int P, bool ADJ>
struct F32Acc {
  static constexpr int MT = F32Bank<P>::MT;
  f4_t t[MT][3];       // Gauss products T1, T2, T3 per M tile
  float br, bi;        // forward: partial log-row sum over this lane's k values
  float s0r, s0i;      // forward: sum of M~_0 over the list (k-group 0 only)
  float gr[MT][4];     // adjoint: rank-one log-row part, per output row
  float gi[MT][4];
  float gsr, gsi;      // adjoint: sum of gb over the list
};

// One class (CX, CY): all 27 offsets unrolled at compile time.
template <int P, bool ADJ, int CX, int CY>
__device__ __forceinline__ void m2l_f32_class(const float *__restrict__ lx, const float2 *__restrict__ lgb,
                                              const float *__restrict__ bank, int lane, F32Acc<P, ADJ> &a) {
  using B = F32Bank<P>;
  constexpr int S = B::S, MT = B::MT, LS = B::LS;
  const int j = lane & 15, kk = lane >> 4;
  const int tx = 2 * (j & 3) + CX, ty = 2 * (j >> 2) + CY;
  const float *lbase = lx + (kk * kRegBoxes + (ty + kHalo) * kReg + (tx + kHalo)) * LS;
  const float *abase = bank + B::a_off + size_t(lane) * LS;
#pragma unroll
  for (int oyi = 0; oyi < 6; ++oyi) {
#pragma unroll
    for (int oxi = 0; oxi < 6; ++oxi) {
      const int ox = oxi - 2 - CX, oy = oyi - 2 - CY;
      if (ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1) continue;  // resolved at compile time
      const int slot = slot_of(ox, oy);
      // B operand: this lane's k values of the source box t + o
      float bx[LS];
      const float4 *bs = reinterpret_cast<const float4 *>(lbase + (oy * kReg + ox) * LS);
#pragma unroll
      for (int e = 0; e < LS / 4; ++e) {
        float4 v = bs[e];
        bx[4 * e] = v.x;
        bx[4 * e + 1] = v.y;
        bx[4 * e + 2] = v.z;
        bx[4 * e + 3] = v.w;
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        float ax[LS];
        const float4 *as = reinterpret_cast<const float4 *>(abase + size_t(slot * MT + mt) * 64 * LS);
#pragma unroll
        for (int e = 0; e < LS / 4; ++e) {
          float4 v = as[e];
          ax[4 * e] = v.x;
          ax[4 * e + 1] = v.y;
          ax[4 * e + 2] = v.z;
          ax[4 * e + 3] = v.w;
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
          a.t[mt][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax[s], bx[s], a.t[mt][0], 0, 0, 0);
          a.t[mt][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax[S + s], bx[S + s], a.t[mt][1], 0, 0, 0);
          a.t[mt][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax[2 * S + s], bx[2 * S + s], a.t[mt][2], 0, 0, 0);
        }
      }
      if (!ADJ) {
        const float2 *r = reinterpret_cast<const float2 *>(bank + B::r_off) + (slot * 4 + kk) * S;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          float2 rv = r[s];
          a.br += rv.x * bx[s] - rv.y * bx[S + s];
          a.bi += rv.x * bx[S + s] + rv.y * bx[s];
        }
        a.s0r += bx[0];
        a.s0i += bx[S];
      } else {
        const int rb = (ty + oy + kHalo) * kReg + (tx + ox + kHalo);
        const float2 g = lgb[rb];
        a.gsr += g.x;
        a.gsi += g.y;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const float4 *r = reinterpret_cast<const float4 *>(bank + B::ra_off) + ((slot * MT + mt) * 16 + kk * 4) / 2;
          float4 r01 = r[0], r23 = r[1];
          float rr[4] = {r01.x, r01.z, r23.x, r23.z}, ri[4] = {r01.y, r01.w, r23.y, r23.w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            a.gr[mt][i] += rr[i] * g.x - ri[i] * g.y;
            a.gi[mt][i] += rr[i] * g.y + ri[i] * g.x;
          }
        }
      }
    }
  }
}

template <int P, bool ADJ>
__global__ __launch_bounds__(256) void m2l_f32_kernel(const float2 *__restrict__ X, const float2 *__restrict__ gbin,
                                                      float2 *__restrict__ Y, float2 *__restrict__ bout,
                                                      const float *__restrict__ bank, TileMap map) {
  using B = F32Bank<P>;
  constexpr int S = B::S, MT = B::MT, LS = B::LS;
  __shared__ __attribute__((aligned(16))) float lx[4 * kRegBoxes * LS];
  __shared__ float2 lgb[ADJ ? kRegBoxes : 1];

  int level, tile;
  tile_of(map, blockIdx.x, level, tile);
  const int nside = 1 << level;
  uint32_t tX, tY;
  unmorton2(uint32_t(tile), tX, tY);
  const int X0 = int(tX) * kTile, Y0 = int(tY) * kTile;
  const int64_t off = level_off(level);
  const int tid = threadIdx.x;

  // Stage the 12x12 source block: lx[kk][box][q S + s] holds part q of
  // coefficient k = S kk + s (q = 0: Re, 1: Im, 2: Re + Im); zero outside the grid.
  for (int idx = tid; idx < kRegBoxes * P; idx += 256) {
    const int rb = idx / P, k = idx - rb * P;
    const int gx = X0 - kHalo + rb % kReg, gy = Y0 - kHalo + rb / kReg;
    float2 v = make_float2(0.f, 0.f);
    if (gx >= 0 && gy >= 0 && gx < nside && gy < nside) v = X[(off + morton2(gx, gy)) * P + k];
    const int kk = k / S, s = k - kk * S;
    float *d = lx + (kk * kRegBoxes + rb) * LS;
    d[s] = v.x;
    d[S + s] = v.y;
    d[2 * S + s] = v.x + v.y;
  }
  if (ADJ) {
    for (int rb = tid; rb < kRegBoxes; rb += 256) {
      const int gx = X0 - kHalo + rb % kReg, gy = Y0 - kHalo + rb / kReg;
      float2 v = make_float2(0.f, 0.f);
      if (gbin && gx >= 0 && gy >= 0 && gx < nside && gy < nside) v = gbin[off + morton2(gx, gy)];
      lgb[rb] = v;
    }
  }
  __syncthreads();

  const int wave = tid >> 6, lane = tid & 63;
  F32Acc<P, ADJ> a;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int q = 0; q < 3; ++q) a.t[mt][q] = f4_t{0.f, 0.f, 0.f, 0.f};
  a.br = a.bi = a.s0r = a.s0i = a.gsr = a.gsi = 0.f;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) a.gr[mt][i] = a.gi[mt][i] = 0.f;

  switch (wave) {
    case 0: m2l_f32_class<P, ADJ, 0, 0>(lx, lgb, bank, lane, a); break;
    case 1: m2l_f32_class<P, ADJ, 1, 0>(lx, lgb, bank, lane, a); break;
    case 2: m2l_f32_class<P, ADJ, 0, 1>(lx, lgb, bank, lane, a); break;
    default: m2l_f32_class<P, ADJ, 1, 1>(lx, lgb, bank, lane, a); break;
  }

  const int cx = wave & 1, cy = wave >> 1;
  const int j = lane & 15, kk = lane >> 4;
  const int gx = X0 + 2 * (j & 3) + cx, gy = Y0 + 2 * (j >> 2) + cy;
  const bool valid = gx < nside && gy < nside;
  const int64_t gbox = off + morton2(uint32_t(gx), uint32_t(gy));
  const float logh = -float(level) * 0.69314718055994530942f;

  if (!ADJ) {
    // log row: sum the four k-groups of each box (lanes j, j+16, j+32, j+48)
    float br = a.br, bi = a.bi;
    br += __shfl_xor(br, 16);
    bi += __shfl_xor(bi, 16);
    br += __shfl_xor(br, 32);
    bi += __shfl_xor(bi, 32);
    if (bout && valid && kk == 0) bout[gbox] = make_float2(br + logh * a.s0r, bi + logh * a.s0i);
  }
  if (valid) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int n0 = 16 * mt + 4 * kk;
      if (n0 < P) {
        float yr[4], yi[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float t1 = a.t[mt][0][i], t2 = a.t[mt][1][i], t3 = a.t[mt][2][i];
          yr[i] = t1 - t2;
          yi[i] = t3 - t1 - t2;
          if (ADJ) {
            yr[i] = a.gr[mt][i] - yr[i];
            yi[i] = a.gi[mt][i] - yi[i];
          }
        }
        if (ADJ && n0 == 0) {
          yr[0] += logh * a.gsr;
          yi[0] += logh * a.gsi;
        }
        float4 *dst = reinterpret_cast<float4 *>(Y + gbox * P + n0);
        dst[0] = make_float4(yr[0], yi[0], yr[1], yi[1]);
        dst[1] = make_float4(yr[2], yi[2], yr[3], yi[3]);
      }
    }
  }
}

template <int P>
static void launch_p(const float *M, const float *gb_in, float *L, float *b, const TileMap &map, int ntiles,
                     bool adjoint, const void *ops, hipStream_t s) {
  const float2 *X = reinterpret_cast<const float2 *>(M);
  float2 *Y = reinterpret_cast<float2 *>(L);
  const float *bank = static_cast<const float *>(ops);
  if (adjoint)
    hipLaunchKernelGGL((m2l_f32_kernel<P, true>), dim3(ntiles), dim3(256), 0, s, X,
                       reinterpret_cast<const float2 *>(gb_in), Y, nullptr, bank, map);
  else
    hipLaunchKernelGGL((m2l_f32_kernel<P, false>), dim3(ntiles), dim3(256), 0, s, X, nullptr, Y,
                       reinterpret_cast<float2 *>(b), bank, map);
}

int launch_m2l_f32(const float *M, const float *gb_in, float *L, float *b, int depth, int p, int lmin, int lmax,
                   bool adjoint, const void *ops, hipStream_t s) {
  (void)depth;
  TileMap map = make_tile_map(lmin, lmax);
  const int ntiles = map.first[map.nlev];
  switch (p) {
    case 8: launch_p<8>(M, gb_in, L, b, map, ntiles, adjoint, ops, s); break;
    case 12: launch_p<12>(M, gb_in, L, b, map, ntiles, adjoint, ops, s); break;
    case 16: launch_p<16>(M, gb_in, L, b, map, ntiles, adjoint, ops, s); break;
    case 20: launch_p<20>(M, gb_in, L, b, map, ntiles, adjoint, ops, s); break;
  }
  return check_launch(adjoint ? "m2l_backward (f32)" : "m2l (f32)");
}

}  // namespace fmm2d
