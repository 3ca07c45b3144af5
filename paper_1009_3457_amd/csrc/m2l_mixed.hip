// Split-precision M2L contraction (BF16x3 / FP16x3) with the fused reduction
// over the interaction list (Sec. 4.1, steps 2-3 of the downward sweep), and
// its adjoint, on gfx950 matrix cores (v_mfma_f32_16x16x32_{bf16,f16}).
//
// Same result as the FP32 kernel, L~(t) = sum_{o in O_c(t)} A~_o M~(t + o)
// (and b, and the transpose), with the contraction run as the three-term
// split product of m2l_mixed_bank.h: FP32 inputs are split into 16-bit hi and
// lo parts once, while staged, and every product accumulates in FP32.
//
// Work decomposition: 16x16 target tiles (deepest level first); one
// persistent workgroup per compute unit (registers allow no second) with four
// compute waves and four loader waves.  Compute wave c owns child class c:
// its 64 target boxes form 4 column blocks of 16 (N tiles), so each operator
// fragment it fetches serves 4 products.  The 20x20 source block around the
// tile (halo 2) is loaded from HBM, split, and stored in LDS once per tile by
// the loader waves, into the second of two buffers while the compute waves'
// products run on the first.  A tree with fewer tiles than two per compute
// unit (2^20 points at depth 8 has 342) would leave most units idle in the
// second round, so there the four compute waves stage their own tile into a
// single buffer, and with half the waves and LDS two such workgroups share a
// compute unit: every tile runs in the first round.  The adjoint takes these
// self-staging workgroups at every size.  Operator fragments
// stream from the L2-resident bank two offsets ahead (they do not depend on
// the tile, so the stream runs on across tiles).  Persistent workgroups take
// tiles in rounds; within a round the workgroups of one XCD take a contiguous
// run of tiles, so the halos that neighbouring tiles share are found in that
// XCD's L2.
//
// FP16 has a narrow exponent range, so for FP16x3 each tile's source block
// (and gb) is scaled by one power of two chosen from its largest magnitude
// (largest |value| in [2^14, 2^15)); the scale is exact and is undone on the
// FP32 accumulators.  BF16 shares FP32's exponent range and needs none.
//
// The adjoint uses the forward operator of each offset, negated (A~(d)^T =
// -A~(-d) and s in IL(t) <=> t in IL(s)); its log-row part is two more
// k-steps per split product over the offset list (section ga of the bank),
// and log(h) sum_o gb(s + o) is added to the n = 0 output in FP32.
#include "fmm2d_internal.h"
#include "m2l_bank.h"
#include "m2l_common.h"
#include "m2l_mixed_bank.h"

namespace fmm2d {

namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));

constexpr int kMShift = 4;                   // tiles of 16 x 16 boxes
constexpr int kMTile = 1 << kMShift;
constexpr int kMReg = kMTile + 2 * kHalo;    // staged source block side (20)
constexpr int kMRegBoxes = kMReg * kMReg;    // 400
// 16-byte units per plane.  ds_read_b128 serves 32 lanes (two lane groups
// g of the B fragment) per pass over 128 four-byte banks, i.e. 32 units; a
// lane group reads 16 units that are contiguous modulo 32, so two planes
// whose indices differ by an odd number fall on disjoint banks when the
// plane stride is 16 modulo 32 (400 = 12 * 32 + 16).
constexpr int kMPlane = kMRegBoxes;
static_assert(kMPlane % 32 == 16, "planes an odd number apart must fall on disjoint banks");
constexpr int kMRow = 40;                    // units per row of same-class boxes: 4 classes x 10

// SELF: the compute waves stage their own tiles (one buffer, no loader
// waves), so a workgroup needs half the waves and LDS and two fit per compute
// unit; used when the tiles are too few to fill two rounds of one workgroup
// per compute unit.
template <int P, bool SELF = false>
struct MixK {
  using C = MixCfg<P>;
  static constexpr int kHalves = 1;  // compute waves per class (2 doubles the operator fetches: slower)
  static constexpr int NT = 4 / kHalves;  // N tiles (16 boxes each) per compute wave; a class has 4
  static constexpr int kCompute = 4 * kHalves;  // compute waves: kHalves per class
  static constexpr int kLoaders = SELF ? 0 : 4;  // loader waves: stage the next tile's source block
  static constexpr int kThreads = 64 * (kCompute + kLoaders);
  static constexpr int kStageWaves = 4;           // waves that stage a block (loaders, or the compute waves)
  static constexpr int kLThreads = 64 * kStageWaves;
  static constexpr int kBuffers = SELF ? 1 : 2;
  static constexpr int kWgPerCu = SELF ? 2 : 1;
  static_assert(!SELF || kCompute == kStageWaves, "self-staging needs one staging slot per compute wave");
  static constexpr int kItems = (kMRegBoxes * C::NPL + kLThreads - 1) / kLThreads;  // staging items per loader thread
  static constexpr int kPlanes = 2 * C::NPL;                                        // hi chunks, lo chunks
  static constexpr int kPlaneUnits = kPlanes * kMPlane;
  static constexpr int kApf = (P <= 16) ? 2 : 1;  // operator prefetch distance (offsets)
  static constexpr bool kBpf = (P <= 16);          // source fragments loaded one offset ahead
  static constexpr int kMid = 12;                  // FP16x3: offset after which the mid-tile barrier sits
  // operator prefetch runs on into the next tile, except where the adjoint's
  // log-row part needs those registers (p = 20)
  template <bool ADJ>
  static constexpr bool carry_a() { return !(ADJ && C::MT * C::KS >= 12); }
};

// 16-byte unit of plane pl for block box (u, v), u, v in [0, 20).  Boxes are
// grouped by class; within a class, rows of 10 units with a row stride of 40.
__device__ constexpr int munit(int pl, int u, int v) {
  return pl * kMPlane + kMRow * (v >> 1) + 10 * ((u & 1) + 2 * (v & 1)) + (u >> 1);
}

// Staging buffers: two, the loader waves filling one while the compute waves
// read the other; one for self-staging workgroups.
template <int P, bool ADJ, bool SELF = false>
struct LdsMix {
  static constexpr int NB = MixK<P, SELF>::kBuffers;
  u32x4_t x[NB][MixK<P, SELF>::kPlaneUnits];
  float2 gb[NB][ADJ ? kMRegBoxes + 1 : 1];  // entry kMRegBoxes stays zero
  float wmax[MixK<P, SELF>::kStageWaves];
  int scale[NB];  // FP16x3: the block is stored times 2^scale
};

template <int PREC>
struct Half16;
template <>
struct Half16<FMM2D_BF16X3> {
  using T = __bf16;
  using V = bf16x8_t;
};
template <>
struct Half16<FMM2D_F16X3> {
  using T = _Float16;
  using V = f16x8_t;
};

// v = hi + lo + O(u^2 |v|), both parts rounded to nearest in the 16-bit format
template <int PREC>
__device__ inline void split8(const float (&v)[8], u32x4_t &hi, u32x4_t &lo) {
  using H = Half16<PREC>;
  typename H::V h, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const typename H::T a = typename H::T(v[e]);
    h[e] = a;
    l[e] = typename H::T(v[e] - float(a));
  }
  hi = __builtin_bit_cast(u32x4_t, h);
  lo = __builtin_bit_cast(u32x4_t, l);
}

template <int PREC>
__device__ inline f4_t mfma16(u32x4_t a, u32x4_t b, f4_t c) {
  if constexpr (PREC == FMM2D_BF16X3)
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                   c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8_t, a), __builtin_bit_cast(f16x8_t, b), c,
                                                  0, 0, 0);
}

struct MGeo {
  int level, nside, X0, Y0;
  int64_t off;
};

__device__ inline MGeo mgeo(const TileMap &map, int t) {
  MGeo g;
  int tile;
  tile_of(map, t, g.level, tile);
  g.nside = 1 << g.level;
  uint32_t tX, tY;
  unmorton2(uint32_t(tile), tX, tY);
  g.X0 = int(tX) * kMTile;
  g.Y0 = int(tY) * kMTile;
  g.off = level_off(g.level);
  return g;
}

// Tile of workgroup b in round r.  Workgroups are dispatched to the 8 XCDs
// in turn (b mod 8); each XCD's workgroups take a contiguous run of tiles:
// XCD x holds G/8 workgroups, one more when x < G mod 8, and its run starts
// after those of XCDs 0..x-1 (a permutation of 0..G-1 for every G).
__device__ inline int round_tile(int r, int b, int G) {
  const int x = b % 8, q = G / 8, rem = G % 8;
  const int pos = x * q + (x < rem ? x : rem) + b / 8;
  return r * G + pos;
}

// ------------------------------------------------------------ loader waves --
// Stages tile t's 20x20 source block (and, adjoint, gb) into buffer `buf`:
// load FP32, (FP16: scale by the block's power of two), split into hi / lo,
// store.  FP16x3 runs one workgroup barrier between finding the block's
// largest magnitude and storing (the compute waves run the matching one
// inside their offset loop); `active` false only takes that barrier.
template <int P, int PREC, bool ADJ, bool SELF>
__device__ __forceinline__ void mixed_stage(LdsMix<P, ADJ, SELF> &sm, int buf, bool active, const MGeo &geo,
                                            const float2 *__restrict__ X, const float2 *__restrict__ gbin, int ltid) {
  using C = MixCfg<P>;
  using K = MixK<P, SELF>;
  constexpr int NPL = C::NPL;
  constexpr bool kF16 = (PREC == FMM2D_F16X3);
  float4 v[K::kItems][2];
  uint32_t ok = 0;
  float2 gv[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
  if (active) {
#pragma unroll
    for (int it = 0; it < K::kItems; ++it) {
      const int e = ltid + K::kLThreads * it;
      const int rb = e / NPL, q = e - rb * NPL;
      const int gx = geo.X0 - kHalo + rb % kMReg, gy = geo.Y0 - kHalo + rb / kMReg;
      const bool in = e < kMRegBoxes * NPL && gx >= 0 && gy >= 0 && gx < geo.nside && gy < geo.nside;
      const int64_t idx = in ? (geo.off + morton2(uint32_t(gx), uint32_t(gy))) * P + 4 * q : 0;
      v[it][0] = *reinterpret_cast<const float4 *>(X + idx);
      v[it][1] = *reinterpret_cast<const float4 *>(X + idx + 2);
      ok |= uint32_t(in) << it;
    }
    if (ADJ && gbin) {
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const int e = ltid + K::kLThreads * it;
        const int gx = geo.X0 - kHalo + e % kMReg, gy = geo.Y0 - kHalo + e / kMReg;
        const bool in = e < kMRegBoxes && gx >= 0 && gy >= 0 && gx < geo.nside && gy < geo.nside;
        const float2 w = gbin[in ? geo.off + morton2(uint32_t(gx), uint32_t(gy)) : 0];
        gv[it] = in ? w : make_float2(0.f, 0.f);
      }
    }
  }
  int sc = 0;
  if (kF16) {
    float m = 0.f;
#pragma unroll
    for (int it = 0; it < K::kItems; ++it)
      if ((ok >> it) & 1u)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          m = fmaxf(m, fmaxf(fmaxf(fabsf(v[it][h].x), fabsf(v[it][h].y)), fmaxf(fabsf(v[it][h].z), fabsf(v[it][h].w))));
    if (ADJ)
#pragma unroll
      for (int it = 0; it < 2; ++it) m = fmaxf(m, fmaxf(fabsf(gv[it].x), fabsf(gv[it].y)));
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) m = fmaxf(m, __shfl_xor(m, d));
    if ((ltid & 63) == 0) sm.wmax[ltid >> 6] = m;
    __syncthreads();  // the mid-tile barrier
#pragma unroll
    for (int w = 0; w < K::kStageWaves; ++w) m = fmaxf(m, sm.wmax[w]);
    sc = (m > 0.f) ? 14 - ilogbf(m) : 0;
    if (ltid == 0 && active) sm.scale[buf] = sc;
  }
  if (!active) return;
#pragma unroll
  for (int it = 0; it < K::kItems; ++it) {
    const int e = ltid + K::kLThreads * it;
    if (e < kMRegBoxes * NPL) {
      const int rb = e / NPL, q = e - rb * NPL;
      const bool in = (ok >> it) & 1u;
      float w[8] = {v[it][0].x, v[it][0].y, v[it][0].z, v[it][0].w, v[it][1].x, v[it][1].y, v[it][1].z, v[it][1].w};
#pragma unroll
      for (int c = 0; c < 8; ++c) w[c] = in ? (kF16 ? ldexpf(w[c], sc) : w[c]) : 0.f;
      u32x4_t hi, lo;
      split8<PREC>(w, hi, lo);
      const int u = rb % kMReg, vv = rb / kMReg;
      sm.x[buf][munit(q, u, vv)] = hi;
      sm.x[buf][munit(NPL + q, u, vv)] = lo;
    }
  }
  if (ADJ) {
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int e = ltid + K::kLThreads * it;
      if (e < kMRegBoxes) sm.gb[buf][e] = kF16 ? make_float2(ldexpf(gv[it].x, sc), ldexpf(gv[it].y, sc)) : gv[it];
    }
  }
}

template <int P, int PREC, bool ADJ>
__device__ __forceinline__ void mixed_loader(LdsMix<P, ADJ, false> &sm, const float2 *__restrict__ X,
                                             const float2 *__restrict__ gbin, const TileMap &map, int ntiles,
                                             int ltid) {
  const int G = int(gridDim.x), b = int(blockIdx.x);
  for (int r = 0, t = round_tile(0, b, G); t < ntiles; t = round_tile(++r, b, G)) {
    const int tn = round_tile(r + 1, b, G);
    const bool has_next = tn < ntiles;
    mixed_stage<P, PREC, ADJ, false>(sm, (r + 1) & 1, has_next, mgeo(map, has_next ? tn : t), X, gbin, ltid);
    __syncthreads();  // end of round r
  }
}

// ----------------------------------------------------------- compute waves --
template <int P, int PREC, bool ADJ, bool SELF, int CX, int CY, int H>
__device__ __forceinline__ void mixed_compute(LdsMix<P, ADJ, SELF> &sm, float2 *__restrict__ Y, float2 *__restrict__ bout,
                                              const unsigned char *__restrict__ bank, const TileMap &map, int ntiles,
                                              int tid, const float2 *__restrict__ X, const float2 *__restrict__ gbin) {
  using C = MixCfg<P>;
  using K = MixK<P, SELF>;
  using B = MixedBank<P>;
  constexpr int MT = C::MT, KS = C::KS, NT = K::NT, NPL = C::NPL, R = C::R;
  constexpr int kApf = K::kApf, kRing = kApf + 1;
  constexpr bool kF16 = (PREC == FMM2D_F16X3);
  constexpr int cls = CX + 2 * CY;
  constexpr int sx = 1 - 2 * CX, sy = 1 - 2 * CY;  // mirror of class (0, 0)'s offsets
  const int lane = tid & 63;
  const int j = lane & 15, g = lane >> 4;

  const __amdgpu_buffer_rsrc_t rsrc =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char *>(bank), 0, int(B::total_bytes), 0x00020000);
  const int alane = lane * 16;
  auto frag = [&](size_t byte_off) {
    return __builtin_bit_cast(u32x4_t, __builtin_amdgcn_raw_buffer_load_b128(rsrc, alane, int(byte_off), 0));
  };

  // LDS byte address (within a buffer) of this lane's B chunk for k-step ks
  // at window (0, 0); per offset and N tile only an immediate is added
  // B plane of lane group gg at k-step ks; a padding chunk (A is 0 there)
  // reads any staged plane, chosen an odd number of planes from its pass
  // partner's (gg - 1) so the two share no bank
  auto bplane = [](int ks, int gg) {
    const int q = 4 * ks + gg, seg = q / NPL;
    if (seg < 3) return ((seg == 1) ? NPL : 0) + q % NPL;
    const int qp = q - 1, segp = qp / NPL;
    if ((gg & 1) && segp < 3) return (((segp == 1) ? NPL : 0) + qp % NPL) ^ 1;
    return 0;
  };
  int abase[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) abase[ks] = (bplane(ks, g) * kMPlane + kMRow * (j >> 3) + (j & 7)) * 16;
  auto bimm = [&](int i, int nt) {  // compile-time after unrolling; this wave's N tile nt is NT H + nt
    const int ox = sx * kOff00.ox[i], oy = sy * kOff00.oy[i];
    return (2 * kMRow * (NT * H + nt) + kMRow * ((CY + kHalo + oy) >> 1) + 10 * (((CX + ox) & 1) + 2 * ((CY + oy) & 1)) +
            ((CX + kHalo + ox) >> 1)) *
           16;
  };

  // adjoint: gb entries q = 16 t + 4 g + e of the class's list, as indices
  // into the staged 20 x 20 gb block relative to N tile 0 (-1: padding)
  int gq[ADJ ? 2 : 1][4];
  if (ADJ) {
    const int t0 = (2 * (j >> 3) + CY + kHalo) * kMReg + 2 * (j & 7) + CX + kHalo;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int q = 16 * t + 4 * g + e;
        int d = -1;
#pragma unroll
        for (int qq = 0; qq < 27; ++qq)
          if (qq == q) d = t0 + sy * kOff00.oy[qq] * kMReg + sx * kOff00.ox[qq];
        gq[t][e] = d;
      }
  }

  // operator fragments: ring of kRing offsets; k-steps equal to an earlier
  // one (a_src) are not loaded twice
  u32x4_t A[kRing][MT][KS];
  auto load_a = [&](int slot_i, int ringpos) {
    const int ox = sx * kOff00.ox[slot_i], oy = sy * kOff00.oy[slot_i];
    const int slot = slot_of(ox, oy);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        if (C::a_src(ks) == ks) A[ringpos][mt][ks] = frag(B::a_frag(slot, mt, ks));
  };
  constexpr bool kCarryA = K::template carry_a<ADJ>();
  if (kCarryA)
#pragma unroll
    for (int i = 0; i < kApf; ++i) load_a(i, i);
  if (!SELF) {
    if (kF16) __syncthreads();  // the prologue's mid-tile barrier (loader waves stage tile 0)
    __syncthreads();            // tile 0 is staged
  }

  const float ln2 = 0.69314718055994530942f;
  const int G = int(gridDim.x), bidx = int(blockIdx.x);
  for (int r = 0, t = round_tile(0, bidx, G); t < ntiles; t = round_tile(++r, bidx, G)) {
    const MGeo geo = mgeo(map, t);
    const int buf = SELF ? 0 : (r & 1);
    if constexpr (SELF) {  // the four compute waves stage this tile (with FP16x3 the block maximum's barrier is inside)
      mixed_stage<P, PREC, ADJ, true>(sm, 0, true, geo, X, gbin, tid);
      __syncthreads();  // the tile is staged
    }
    const char *xb = reinterpret_cast<const char *>(sm.x[buf]);
    auto lds16 = [&](int byte_off) { return *reinterpret_cast<const u32x4_t *>(xb + byte_off); };
    const int sc = kF16 ? sm.scale[buf] : 0;

    // ---------------- products over the 27 offsets of the class
    f4_t acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f4_t{0.f, 0.f, 0.f, 0.f};

    if (!kCarryA)
#pragma unroll
      for (int i = 0; i < kApf; ++i) load_a(i, i);
    if constexpr (K::kBpf) {
      // source fragments of a whole offset, one offset ahead
      u32x4_t Bf[2][NT][KS];
      auto load_b = [&](int i, int pos) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int ks = 0; ks < KS; ++ks)
            if (C::b_src(ks) == ks) Bf[pos][nt][ks] = lds16(abase[ks] + bimm(i, nt));
      };
      load_b(0, 0);
#pragma unroll
      for (int i = 0; i < 27; ++i) {
        const int cur = i & 1;
        if (i + 1 < 27) load_b(i + 1, cur ^ 1);
        if (kCarryA || i + kApf < 27) load_a((i + kApf) % 27, (i + kApf) % kRing);  // next tile restarts at 0
        const int ap = i % kRing;
        // k-steps innermost: each accumulator takes a chain of KS products
        // (chained accumulation issues faster than rotating accumulators)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
              acc[mt][nt] = mfma16<PREC>(A[ap][mt][C::a_src(ks)], Bf[cur][nt][C::b_src(ks)], acc[mt][nt]);
        // The wave issues in order, so a burst of loads ahead of the
        // products would leave the matrix pipe idle while the LDS and vector
        // memory queues accept them: the loads of the next offsets issue one
        // after each product instead, under the products already running.
        {
          const int nds = (i + 1 < 27) ? NT * C::kUniqueB : 0;
          const int nvm = (kCarryA || i + kApf < 27) ? MT * C::kUniqueA : 0;
#pragma unroll
          for (int q = 0; q < nds; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
          }
#pragma unroll
          for (int q = 0; q < nvm; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // one vector-memory read
          }
          __builtin_amdgcn_sched_group_barrier(0x008, MT * NT * KS, 0);  // the rest of the products
        }
        __builtin_amdgcn_sched_barrier(0);
        if (kF16 && !SELF && i == K::kMid) __syncthreads();  // matches the loader waves' mid-tile barrier
      }
    } else {
      // source fragments of one N tile, one N tile ahead (fewer registers)
      u32x4_t Bn[2][KS];
      auto load_bn = [&](int i, int nt, int pos) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
          if (C::b_src(ks) == ks) Bn[pos][ks] = lds16(abase[ks] + bimm(i, nt));
      };
      load_bn(0, 0, 0);
#pragma unroll
      for (int i = 0; i < 27; ++i) {
        if (kCarryA || i + kApf < 27) load_a((i + kApf) % 27, (i + kApf) % kRing);  // next tile restarts at 0
        const int ap = i % kRing;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int pos = (i * NT + nt) & 1;
          if (nt + 1 < NT) load_bn(i, nt + 1, pos ^ 1);
          else if (i + 1 < 27) load_bn(i + 1, 0, pos ^ 1);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
              acc[mt][nt] = mfma16<PREC>(A[ap][mt][C::a_src(ks)], Bn[pos][C::b_src(ks)], acc[mt][nt]);
          __builtin_amdgcn_sched_barrier(0);
        }
        if (kF16 && !SELF && i == K::kMid) __syncthreads();  // matches the loader waves' mid-tile barrier
      }
    }
    if (kCarryA && 27 % kRing != 0) {
      // the next tile's offsets 0 .. kApf-1 were prefetched into ring
      // positions (27 + i) mod kRing; it reads them at positions i
      u32x4_t tmp[kApf][MT][KS];
#pragma unroll
      for (int i = 0; i < kApf; ++i)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) tmp[i][mt][ks] = A[(27 + i) % kRing][mt][ks];
#pragma unroll
      for (int i = 0; i < kApf; ++i)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) A[i][mt][ks] = tmp[i][mt][ks];
    }

    // ---------------- adjoint log-row part (k-steps over the offset list)
    float sgr[NT], sgi[NT];
    if (ADJ) {
      u32x4_t ga[2][MT][2];
#pragma unroll
      for (int part = 0; part < 2; ++part)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int t2 = 0; t2 < 2; ++t2) ga[part][mt][t2] = frag(B::ga_frag(cls, part, mt, t2));
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        sgr[nt] = 0.f;
        sgi[nt] = 0.f;
        u32x4_t ghi[2], glo[2];
#pragma unroll
        for (int t2 = 0; t2 < 2; ++t2) {
          float w[8];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int d = gq[t2][e];
            const float2 z = sm.gb[buf][d < 0 ? kMRegBoxes : d + 2 * kMReg * 2 * (NT * H + nt)];
            w[2 * e] = z.x;
            w[2 * e + 1] = z.y;
            sgr[nt] += z.x;
            sgi[nt] += z.y;
          }
          split8<PREC>(w, ghi[t2], glo[t2]);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
            for (int part = 0; part < 3; ++part)
              acc[mt][nt] = mfma16<PREC>(ga[part == 2][mt][t2], part == 1 ? glo[t2] : ghi[t2], acc[mt][nt]);
        sgr[nt] += __shfl_xor(sgr[nt], 16);
        sgi[nt] += __shfl_xor(sgi[nt], 16);
        sgr[nt] += __shfl_xor(sgr[nt], 32);
        sgi[nt] += __shfl_xor(sgi[nt], 32);
      }
    }

    // ---------------- output: lane (g, j) holds rows 16 mt + 4 g .. + 3 of box j
    const float logh = -float(geo.level) * ln2;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int gx = geo.X0 + 2 * (j & 7) + CX, gy = geo.Y0 + 2 * (2 * (NT * H + nt) + (j >> 3)) + CY;
      if (gx >= geo.nside || gy >= geo.nside) continue;
      const int64_t box = geo.off + morton2(uint32_t(gx), uint32_t(gy));
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int rho0 = 16 * mt + 4 * g;
        float y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float a = acc[mt][nt][q];
          if (kF16) a = ldexpf(a, -sc);
          y[q] = ADJ ? -a : a;
        }
        if (rho0 < R) {
          if (ADJ && rho0 == 0) {
            const float s0r = kF16 ? ldexpf(sgr[nt], -sc) : sgr[nt];
            const float s0i = kF16 ? ldexpf(sgi[nt], -sc) : sgi[nt];
            y[0] += logh * s0r;
            y[1] += logh * s0i;
          }
          *reinterpret_cast<float4 *>(Y + box * P + rho0 / 2) = make_float4(y[0], y[1], y[2], y[3]);
        } else if (!ADJ && C::kLogRows && rho0 == R && bout) {
          bout[box] = make_float2(y[0] + logh * y[2], y[1] + logh * y[3]);
        }
      }
    }
    __syncthreads();  // end of round r: buffer r & 1 is free, the next tile is staged (SELF: the buffer is free)
  }
}

template <int P, int PREC, bool ADJ, bool SELF>
__global__ __launch_bounds__((MixK<P, SELF>::kThreads)) __attribute__((amdgpu_waves_per_eu(MixK<P, SELF>::kWgPerCu)))
void m2l_mixed_kernel(const float2 *__restrict__ X, const float2 *__restrict__ gbin, float2 *__restrict__ Y,
                      float2 *__restrict__ bout, const unsigned char *__restrict__ bank, TileMap map, int ntiles) {
  using K = MixK<P, SELF>;
  __shared__ __attribute__((aligned(16))) LdsMix<P, ADJ, SELF> sm;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: the role lives in SGPRs
  if (ADJ && tid == 0)
    for (int nb = 0; nb < K::kBuffers; ++nb) sm.gb[nb][kMRegBoxes] = make_float2(0.f, 0.f);
  if (SELF) __syncthreads();  // the zero slot is written before any wave reads it
  // Both roles run the same number of workgroup barriers: per round one at
  // its end, and with FP16x3 one more in its middle (and in the prologue).
  if constexpr (!SELF) {
    if (wave >= K::kCompute) {
      const int ltid = tid - 64 * K::kCompute;
      const int G = int(gridDim.x), b = int(blockIdx.x);
      const int t0 = round_tile(0, b, G);
      mixed_stage<P, PREC, ADJ, false>(sm, 0, t0 < ntiles, mgeo(map, t0 < ntiles ? t0 : 0), X, gbin, ltid);
      __syncthreads();  // tile 0 is staged
      mixed_loader<P, PREC, ADJ>(sm, X, gbin, map, ntiles, ltid);
      return;
    }
  }
  // compute wave w: class w mod 4, N tiles of half w / 4
  switch (wave) {
    case 0: mixed_compute<P, PREC, ADJ, SELF, 0, 0, 0>(sm, Y, bout, bank, map, ntiles, tid, X, gbin); break;
    case 1: mixed_compute<P, PREC, ADJ, SELF, 1, 0, 0>(sm, Y, bout, bank, map, ntiles, tid, X, gbin); break;
    case 2: mixed_compute<P, PREC, ADJ, SELF, 0, 1, 0>(sm, Y, bout, bank, map, ntiles, tid, X, gbin); break;
    case 3: mixed_compute<P, PREC, ADJ, SELF, 1, 1, 0>(sm, Y, bout, bank, map, ntiles, tid, X, gbin); break;
    default:
      if constexpr (K::kHalves == 2) {
        switch (wave) {
          case 4: mixed_compute<P, PREC, ADJ, SELF, 0, 0, 1>(sm, Y, bout, bank, map, ntiles, tid, X, gbin); break;
          case 5: mixed_compute<P, PREC, ADJ, SELF, 1, 0, 1>(sm, Y, bout, bank, map, ntiles, tid, X, gbin); break;
          case 6: mixed_compute<P, PREC, ADJ, SELF, 0, 1, 1>(sm, Y, bout, bank, map, ntiles, tid, X, gbin); break;
          default: mixed_compute<P, PREC, ADJ, SELF, 1, 1, 1>(sm, Y, bout, bank, map, ntiles, tid, X, gbin); break;
        }
      }
      break;
  }
}

template <int P, int PREC, bool SELF>
void launch_self(const float *M, const float *gb_in, float *L, float *b, const TileMap &map, int ntiles, bool adjoint,
                 const void *ops, hipStream_t s) {
  using K = MixK<P, SELF>;
  const int slots = K::kWgPerCu * num_cus();
  const int grid = ntiles < slots ? ntiles : slots;
  const float2 *X = reinterpret_cast<const float2 *>(M);
  float2 *Y = reinterpret_cast<float2 *>(L);
  const unsigned char *bank = static_cast<const unsigned char *>(ops);
  if (adjoint)
    hipLaunchKernelGGL((m2l_mixed_kernel<P, PREC, true, SELF>), dim3(grid), dim3(K::kThreads), 0, s, X,
                       reinterpret_cast<const float2 *>(gb_in), Y, nullptr, bank, map, ntiles);
  else
    hipLaunchKernelGGL((m2l_mixed_kernel<P, PREC, false, SELF>), dim3(grid), dim3(K::kThreads), 0, s, X, nullptr, Y,
                       reinterpret_cast<float2 *>(b), bank, map, ntiles);
}

// Self-staging workgroups, two per compute unit, when the tiles would not fill
// two rounds of one loader-backed workgroup per compute unit, and for the
// adjoint at every size (faster at depths 8 to 10 for every order, by up to
// 14%; the forward map of larger trees is within a few percent either way and
// keeps its loader waves).
template <int P, int PREC>
void launch_pp(const float *M, const float *gb_in, float *L, float *b, const TileMap &map, int ntiles, bool adjoint,
               const void *ops, hipStream_t s) {
  if (adjoint || ntiles < 2 * num_cus())
    launch_self<P, PREC, true>(M, gb_in, L, b, map, ntiles, adjoint, ops, s);
  else
    launch_self<P, PREC, false>(M, gb_in, L, b, map, ntiles, adjoint, ops, s);
}

template <int PREC>
void launch_prec(int p, const float *M, const float *gb_in, float *L, float *b, const TileMap &map, int ntiles,
                 bool adjoint, const void *ops, hipStream_t s) {
  switch (p) {
    case 8: launch_pp<8, PREC>(M, gb_in, L, b, map, ntiles, adjoint, ops, s); break;
    case 12: launch_pp<12, PREC>(M, gb_in, L, b, map, ntiles, adjoint, ops, s); break;
    case 16: launch_pp<16, PREC>(M, gb_in, L, b, map, ntiles, adjoint, ops, s); break;
    case 20: launch_pp<20, PREC>(M, gb_in, L, b, map, ntiles, adjoint, ops, s); break;
  }
}

size_t r_section(int p) {
  switch (p) {
    case 8: return MixedBank<8>::r_off;
    case 12: return MixedBank<12>::r_off;
    case 16: return MixedBank<16>::r_off;
    case 20: return MixedBank<20>::r_off;
  }
  return 0;
}

}  // namespace

bool m2l_mixed_supported(int p, int precision) {
  return (precision == FMM2D_BF16X3 || precision == FMM2D_F16X3) && p_supported(p);
}

int launch_m2l_mixed(const float *M, const float *gb_in, float *L, float *b, int depth, int p, int lmin, int lmax,
                     bool adjoint, int precision, const void *ops, hipStream_t s) {
  (void)depth;
  const TileMap map = make_tile_map(lmin, lmax, kMShift);
  const int ntiles = map.first[map.nlev];
  if (precision == FMM2D_BF16X3) launch_prec<FMM2D_BF16X3>(p, M, gb_in, L, b, map, ntiles, adjoint, ops, s);
  else launch_prec<FMM2D_F16X3>(p, M, gb_in, L, b, map, ntiles, adjoint, ops, s);
  int rc = check_launch(adjoint ? "m2l_backward (split precision)" : "m2l (split precision)");
  if (rc == FMM2D_OK && !adjoint && b && (2 * p) % 16 == 0) {  // no spare rows: separate log-row pass
    const float *r = reinterpret_cast<const float *>(static_cast<const unsigned char *>(ops) + r_section(p));
    rc = launch_m2l_logrow_fwd(M, b, p, lmin, lmax, r, s);
  }
  return rc;
}

}  // namespace fmm2d
