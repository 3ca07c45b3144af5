// Staging of source expansions for the FP32 M2L kernels (private to the
// library): the LDS layout of a tile's 12x12 source block and its fetch from
// HBM in register batches.  Shared by the Gauss-form and Pascal-form FP32
// kernels, which read the block with the same lane mapping: MFMA column j of
// a k-group is one of the 16 target boxes of a class, and lane (kk, j) takes
// the coefficients k = S kk + s, s < S, S = p / 4.
#pragma once

#include "m2l_common.h"

namespace fmm2d {

// Work split of the fetch: T threads move the block's 144 p / 2 float4 chunks.
template <int P, int T>
struct StageCfg {
  static constexpr int S = P / 4;
  static constexpr int kThreads = T;
  static constexpr int kChunks = kRegBoxes * P / 2;        // float4 chunks of a source block
  static constexpr int kPf = (kChunks + T - 1) / T;        // chunks per thread
};

// Layout of a staged 12x12 source block in LDS, in 16-byte units.  The B
// fragment of lane (kk, j) for one offset is NE units (2S floats: Re, Im of
// k = S kk + s) of one box; the 16 lanes of a k-group read a 4x4 window of
// same-class boxes (stride 2 in the region).  Boxes are therefore stored by
// class: unit = kRow v' + 6 class + u' with (u', v') = (u, v) / 2.
// A 16-byte LDS read serves 32 lanes (two k-groups) per pass over 128
// four-byte banks, i.e. 32 units.  kRow makes the 16 units of a window
// distinct modulo 32, and the plane stride puts the next k-group's window
// (NE kPlane units on) on the other 16 residues, so the reads are free of
// bank conflicts: kRow 28, kPlane 168 for NE = 2; kRow 24, kPlane 148 for
// NE = 1 and 3 (found by search over the strides that fit the block).
template <int P>
struct XLayout {
  static constexpr int S = P / 4;
  static constexpr int NE = (2 * S + 3) / 4;  // units per (k-group, box) record
  static constexpr int kRow = NE == 2 ? 28 : 24;        // 4 classes x 6 (+ 4 spare units)
  static constexpr int kPlane = NE == 2 ? 6 * kRow : 148;  // units per (k-group, unit index)
  static constexpr int kFloats = 4 * NE * kPlane * 4;
  __device__ static int unit(int kk, int e, int u, int v) {  // u, v in [0, 12)
    return (kk * NE + e) * kPlane + kRow * (v >> 1) + 6 * ((u & 1) + 2 * (v & 1)) + (u >> 1);
  }
};

// Source block of one tile held in registers between the global load and the
// LDS store.  Every load is issued unconditionally (from box 0 when the box
// lies outside the grid) and masked when stored, so no branch forces an
// early wait.
template <int P, int T>
struct Prefetch {
  float4 v[StageCfg<P, T>::kPf];
  float2 g;
  uint32_t ok;  // bit r: chunk r is inside the grid; bit 31: the gb entry is
};

struct TileGeo {
  int level, nside, X0, Y0;
  int64_t off;
  uint32_t tm;  // the tile's Morton index in its level: morton2(X0 / 8, Y0 / 8)
};

__device__ inline TileGeo tile_geo(const TileMap &map, int t) {
  TileGeo g;
  int tile;
  tile_of(map, t, g.level, tile);
  g.nside = 1 << g.level;
  uint32_t tX, tY;
  unmorton2(uint32_t(tile), tX, tY);
  g.X0 = int(tX) * kTile;
  g.Y0 = int(tY) * kTile;
  g.off = level_off(g.level);
  g.tm = uint32_t(tile);
  return g;
}

// Loads chunks r0 .. r1-1 (and, with the first batch, the adjoint's gb).
template <int P, int T, bool ADJ>
__device__ inline void prefetch_issue(Prefetch<P, T> &pf, const TileGeo &g, const float2 *__restrict__ X,
                                      const float2 *__restrict__ gbin, int tid, int r0, int r1) {
  using C = StageCfg<P, T>;
  if (r0 == 0) pf.ok = 0;
#pragma unroll
  for (int r = 0; r < C::kPf; ++r) {
    if (r < r0 || r >= r1) continue;
    const int e = tid + C::kThreads * r;
    const int rb = e / (P / 2), q = e - rb * (P / 2);
    const int gx = g.X0 - kHalo + rb % kReg, gy = g.Y0 - kHalo + rb / kReg;
    const bool in = e < C::kChunks && gx >= 0 && gy >= 0 && gx < g.nside && gy < g.nside;
    const int64_t idx = in ? (g.off + morton2(uint32_t(gx), uint32_t(gy))) * P + 2 * q : 0;
    pf.v[r] = *reinterpret_cast<const float4 *>(X + idx);
    pf.ok |= uint32_t(in) << r;
  }
  if (ADJ && r0 == 0 && gbin) {  // gbin is uniform
    const int gx = g.X0 - kHalo + tid % kReg, gy = g.Y0 - kHalo + tid / kReg;
    const bool in = tid < kRegBoxes && gx >= 0 && gy >= 0 && gx < g.nside && gy < g.nside;
    pf.g = gbin[in ? g.off + morton2(uint32_t(gx), uint32_t(gy)) : 0];
    pf.ok |= uint32_t(in) << 31;
  }
}

// Stores chunks r0 .. r1-1 into the XLayout buffer (and, with the first
// batch, gb[box]; entry kRegBoxes of gb stays zero).
template <int P, int T, bool ADJ>
__device__ inline void prefetch_store(const Prefetch<P, T> &pf, float *__restrict__ lx, float2 *__restrict__ lgb,
                                      int tid, int r0, int r1) {
  using C = StageCfg<P, T>;
  constexpr int S = C::S;
#pragma unroll
  for (int r = 0; r < C::kPf; ++r) {
    if (r < r0 || r >= r1) continue;
    const int e = tid + C::kThreads * r;
    if (e < C::kChunks) {
      const int rb = e / (P / 2), q = e - rb * (P / 2);
      const bool in = (pf.ok >> r) & 1u;
      const float re[2] = {in ? pf.v[r].x : 0.f, in ? pf.v[r].z : 0.f};
      const float im[2] = {in ? pf.v[r].y : 0.f, in ? pf.v[r].w : 0.f};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 2 * q + h;
        const int kk = k / S, s = k - kk * S;
        const int u = rb % kReg, v = rb / kReg;
        lx[XLayout<P>::unit(kk, s >> 2, u, v) * 4 + (s & 3)] = re[h];
        lx[XLayout<P>::unit(kk, (S + s) >> 2, u, v) * 4 + ((S + s) & 3)] = im[h];
      }
    }
  }
  if (ADJ && r0 == 0 && tid <= kRegBoxes)
    lgb[tid] = (tid < kRegBoxes && (pf.ok >> 31)) ? pf.g : make_float2(0.f, 0.f);
}


}  // namespace fmm2d
