// Work decomposition shared by the M2L contraction kernels.
//
// One workgroup owns an 8x8 tile of target boxes of one level (a contiguous
// Morton range of 64 boxes, aligned to parent boundaries).  The sources of all
// 64 targets lie in the 12x12 block of boxes around the tile (a halo of two
// boxes on every side), which is staged once in LDS and shared by the whole
// interaction list of every target in the tile.  Inside the tile, the 16
// boxes of one child class (ix & 1, iy & 1) share one list of 27 offsets, so
// for each offset they form the columns of one dense product with a single
// operator: one wave per class, 16 target boxes per MFMA column block.
#pragma once

#include "fmm2d_internal.h"

namespace fmm2d {

constexpr int kTile = 8;                  // target tile side (boxes)
constexpr int kHalo = 2;                  // source halo on each side
constexpr int kReg = kTile + 2 * kHalo;   // staged source block side (12)
constexpr int kRegBoxes = kReg * kReg;    // 144

// Maps a flat tile index to (level, tile-in-level).  Levels are laid out
// deepest first.  With tiles of 2^shift x 2^shift boxes, level l has
// max(1, 4^(l - shift)) tiles; a level smaller than one tile uses one
// partially filled tile.
struct TileMap {
  int nlev;
  int level[kMaxDepth + 1];
  int first[kMaxDepth + 2];  // first[i] = flat index of level[i]'s first tile; first[nlev] = total
};

inline TileMap make_tile_map(int lmin, int lmax, int shift = 3) {
  TileMap m{};
  int acc = 0;
  m.nlev = 0;
  for (int l = lmax; l >= lmin; --l) {
    m.level[m.nlev] = l;
    m.first[m.nlev] = acc;
    acc += (l >= shift) ? (1 << (2 * (l - shift))) : 1;
    ++m.nlev;
  }
  m.first[m.nlev] = acc;
  return m;
}

__device__ inline void tile_of(const TileMap &m, int g, int &level, int &tile) {
  int i = 0;
  while (i + 1 < m.nlev && g >= m.first[i + 1]) ++i;
  level = m.level[i];
  tile = g - m.first[i];
}

}  // namespace fmm2d
