// Split-precision M2L contraction (BF16x3 / FP16x3) with the fused reduction
// over the interaction list (Sec. 4.1, steps 2-3 of the downward sweep), and
// its adjoint, on gfx950 matrix cores (v_mfma_f32_16x16x32_{bf16,f16}).
//
// Same result as the FP32 kernel, L~(t) = sum_{o in O_c(t)} A~_o M~(t + o)
// (and b, and the transpose), with the contraction run as the three-term
// split product of m2l_mixed_bank.h: FP32 inputs are split into 16-bit hi and
// lo parts once, while staged, and every product accumulates in FP32.
//
// Work decomposition: 16x16 target tiles (deepest level first), one
// four-wave workgroup per tile, two workgroups per compute unit.  Wave c owns
// child class c: its 64 target boxes form 4 column blocks of 16 (N tiles),
// so each operator fragment it fetches serves 4 products.  The 20x20 source
// block around the tile (halo 2) is loaded from HBM, split, and stored in LDS
// once per tile; while one workgroup stages, the other's products keep the
// matrix cores busy.  Operator fragments stream from the L2-resident bank
// two offsets ahead (they do not depend on the tile, so the stream runs on
// across tiles).  Persistent workgroups take tiles in rounds; within a round
// the workgroups of one XCD take a contiguous run of tiles, so the halos that
// neighbouring tiles share are found in that XCD's L2.
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
constexpr int kMPlane = kMRegBoxes + 1;      // 16-byte units per plane (+1: planes start on different banks)
constexpr int kMRow = 40;                    // units per row of same-class boxes: 4 classes x 10

template <int P>
struct MixK {
  using C = MixCfg<P>;
  static constexpr int NT = 4;  // N tiles (16 boxes each) per wave: the 64 boxes of one class
  static constexpr int kThreads = 256;
  static constexpr int kItems = (kMRegBoxes * C::NPL + kThreads - 1) / kThreads;  // staging items per thread
  static constexpr int kPlanes = 2 * C::NPL;                                       // hi chunks, lo chunks
  static constexpr int kApf = (P <= 16) ? 2 : 1;  // operator prefetch distance (offsets)
  static constexpr bool kBpf = (P <= 16);          // source fragments loaded one offset ahead
  // operator prefetch runs on into the next tile, except where the adjoint's
  // log-row part needs those registers (p = 20)
  template <bool ADJ>
  static constexpr bool carry_a() { return !(ADJ && C::MT * C::KS >= 12); }
};

// 16-byte unit of plane pl for block box (u, v), u, v in [0, 20).  Boxes are
// grouped by class; within a class, rows of 10 units with a row stride of 40
// (= 8 mod 16), so the 16 lanes of a lane group, which read an 8 x 2 window
// of same-class boxes, hit 16 distinct 16-byte bank groups.
__device__ constexpr int munit(int pl, int u, int v) {
  return pl * kMPlane + kMRow * (v >> 1) + 10 * ((u & 1) + 2 * (v & 1)) + (u >> 1);
}

template <int P, bool ADJ>
struct LdsMix {
  u32x4_t x[MixK<P>::kPlanes * kMPlane];
  float2 gb[ADJ ? kMRegBoxes + 1 : 1];  // entry kMRegBoxes stays zero
  float wmax[4];
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
// in turn (b mod 8); each XCD's workgroups take a contiguous run of G/8 tiles.
__device__ inline int round_tile(int r, int b, int G) {
  const int pos = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  return r * G + pos;
}

template <int P, int PREC, bool ADJ, int CX, int CY>
__device__ __forceinline__ void m2l_mixed_run(LdsMix<P, ADJ> &sm, const float2 *__restrict__ X,
                                              const float2 *__restrict__ gbin, float2 *__restrict__ Y,
                                              float2 *__restrict__ bout, const unsigned char *__restrict__ bank,
                                              const TileMap &map, int ntiles, int tid) {
  using C = MixCfg<P>;
  using K = MixK<P>;
  using B = MixedBank<P>;
  constexpr int MT = C::MT, KS = C::KS, NT = K::NT, NPL = C::NPL, R = C::R;
  constexpr int kApf = K::kApf, kRing = kApf + 1;
  constexpr bool kF16 = (PREC == FMM2D_F16X3);
  constexpr int cls = CX + 2 * CY;
  constexpr int sx = 1 - 2 * CX, sy = 1 - 2 * CY;  // mirror of class (0, 0)'s offsets
  const int lane = tid & 63, wave = tid >> 6;
  const int j = lane & 15, g = lane >> 4;

  const __amdgpu_buffer_rsrc_t rsrc =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char *>(bank), 0, int(B::total_bytes), 0x00020000);
  const int alane = lane * 16;
  auto frag = [&](size_t byte_off) {
    return __builtin_bit_cast(u32x4_t, __builtin_amdgcn_raw_buffer_load_b128(rsrc, alane, int(byte_off), 0));
  };

  // LDS byte address of this lane's B chunk for k-step ks at window (0, 0);
  // per offset and N tile only an immediate is added
  int abase[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int q = 4 * ks + g, seg = q / NPL;
    const int pl = seg >= 3 ? 0 : ((seg == 1) ? NPL : 0) + q % NPL;  // zero chunk: any finite data (A is 0)
    abase[ks] = (pl * kMPlane + kMRow * (j >> 3) + (j & 7)) * 16;
  }
  auto bimm = [&](int i, int nt) {  // compile-time after unrolling
    const int ox = sx * kOff00.ox[i], oy = sy * kOff00.oy[i];
    return (2 * kMRow * nt + kMRow * ((CY + kHalo + oy) >> 1) + 10 * (((CX + ox) & 1) + 2 * ((CY + oy) & 1)) +
            ((CX + kHalo + ox) >> 1)) *
           16;
  };
  auto lds16 = [&](int byte_off) {
    return *reinterpret_cast<const u32x4_t *>(reinterpret_cast<const char *>(sm.x) + byte_off);
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

  const float ln2 = 0.69314718055994530942f;
  const int G = int(gridDim.x);
  for (int r = 0, t = round_tile(0, int(blockIdx.x), G); t < ntiles; t = round_tile(++r, int(blockIdx.x), G)) {
    const MGeo geo = mgeo(map, t);

    // ---------------- stage the source block: load, (scale,) split, store
    float4 v[K::kItems][2];
    uint32_t ok = 0;
#pragma unroll
    for (int it = 0; it < K::kItems; ++it) {
      const int e = tid + K::kThreads * it;
      const int rb = e / NPL, q = e - rb * NPL;
      const int gx = geo.X0 - kHalo + rb % kMReg, gy = geo.Y0 - kHalo + rb / kMReg;
      const bool in = e < kMRegBoxes * NPL && gx >= 0 && gy >= 0 && gx < geo.nside && gy < geo.nside;
      const int64_t idx = in ? (geo.off + morton2(uint32_t(gx), uint32_t(gy))) * P + 4 * q : 0;
      v[it][0] = *reinterpret_cast<const float4 *>(X + idx);
      v[it][1] = *reinterpret_cast<const float4 *>(X + idx + 2);
      ok |= uint32_t(in) << it;
    }
    float2 gv[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
    if (ADJ && gbin) {
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const int e = tid + K::kThreads * it;
        const int gx = geo.X0 - kHalo + e % kMReg, gy = geo.Y0 - kHalo + e / kMReg;
        const bool in = e < kMRegBoxes && gx >= 0 && gy >= 0 && gx < geo.nside && gy < geo.nside;
        const float2 w = gbin[in ? geo.off + morton2(uint32_t(gx), uint32_t(gy)) : 0];
        gv[it] = in ? w : make_float2(0.f, 0.f);
      }
    }
    int sc = 0;  // FP16: values are stored times 2^sc
    float m = 0.f;
    if (kF16) {
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
    }
    __syncthreads();  // every wave is done with the previous tile's block
    if (kF16) {
      if (lane == 0) sm.wmax[wave] = m;
      __syncthreads();
      m = fmaxf(fmaxf(sm.wmax[0], sm.wmax[1]), fmaxf(sm.wmax[2], sm.wmax[3]));
      sc = (m > 0.f) ? 14 - ilogbf(m) : 0;
    }
#pragma unroll
    for (int it = 0; it < K::kItems; ++it) {
      const int e = tid + K::kThreads * it;
      if (e < kMRegBoxes * NPL) {
        const int rb = e / NPL, q = e - rb * NPL;
        const bool in = (ok >> it) & 1u;
        float w[8] = {v[it][0].x, v[it][0].y, v[it][0].z, v[it][0].w,
                      v[it][1].x, v[it][1].y, v[it][1].z, v[it][1].w};
#pragma unroll
        for (int c = 0; c < 8; ++c) w[c] = in ? (kF16 ? ldexpf(w[c], sc) : w[c]) : 0.f;
        u32x4_t hi, lo;
        split8<PREC>(w, hi, lo);
        const int u = rb % kMReg, vv = rb / kMReg;
        sm.x[munit(q, u, vv)] = hi;
        sm.x[munit(NPL + q, u, vv)] = lo;
      }
    }
    if (ADJ) {
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const int e = tid + K::kThreads * it;
        if (e < kMRegBoxes)
          sm.gb[e] = kF16 ? make_float2(ldexpf(gv[it].x, sc), ldexpf(gv[it].y, sc)) : gv[it];
      }
    }
    __syncthreads();

    // ---------------- products over the 27 offsets of the class
    f4_t acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f4_t{0.f, 0.f, 0.f, 0.f};

    u32x4_t Bf[2][NT][KS];
    auto load_b = [&](int i, int pos) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
          if (C::b_src(ks) == ks) Bf[pos][nt][ks] = lds16(abase[ks] + bimm(i, nt));
    };
    if (!kCarryA)
#pragma unroll
      for (int i = 0; i < kApf; ++i) load_a(i, i);
    if (K::kBpf) load_b(0, 0);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      const int cur = K::kBpf ? (i & 1) : 0;
      if (K::kBpf) {
        if (i + 1 < 27) load_b(i + 1, cur ^ 1);
      } else {
        load_b(i, 0);
      }
      if (kCarryA || i + kApf < 27) load_a((i + kApf) % 27, (i + kApf) % kRing);  // next tile restarts at 0
      const int ap = i % kRing;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int ks = 0; ks < KS; ++ks)
            if (C::a_chunk(ks, 0) >= 0 || C::a_chunk(ks, 1) >= 0 || C::a_chunk(ks, 2) >= 0 || C::a_chunk(ks, 3) >= 0)
              acc[mt][nt] = mfma16<PREC>(A[ap][mt][C::a_src(ks)], Bf[cur][nt][C::b_src(ks)], acc[mt][nt]);
      __builtin_amdgcn_sched_barrier(0);
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
            const float2 z = sm.gb[d < 0 ? kMRegBoxes : d + 2 * kMReg * 2 * nt];
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
          for (int t2 = 0; t2 < 2; ++t2) {
            acc[mt][nt] = mfma16<PREC>(ga[0][mt][t2], ghi[t2], acc[mt][nt]);
            acc[mt][nt] = mfma16<PREC>(ga[0][mt][t2], glo[t2], acc[mt][nt]);
            acc[mt][nt] = mfma16<PREC>(ga[1][mt][t2], ghi[t2], acc[mt][nt]);
          }
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
      const int gx = geo.X0 + 2 * (j & 7) + CX, gy = geo.Y0 + 2 * (2 * nt + (j >> 3)) + CY;
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
  }
}

template <int P, int PREC, bool ADJ>
__global__ __launch_bounds__(256, 2) void m2l_mixed_kernel(const float2 *__restrict__ X,
                                                           const float2 *__restrict__ gbin, float2 *__restrict__ Y,
                                                           float2 *__restrict__ bout,
                                                           const unsigned char *__restrict__ bank, TileMap map,
                                                           int ntiles) {
  __shared__ __attribute__((aligned(16))) LdsMix<P, ADJ> sm;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: the class lives in SGPRs
  if (ADJ && tid == 0) sm.gb[kMRegBoxes] = make_float2(0.f, 0.f);
  // every branch runs the same tile loop, hence the same barriers
  switch (wave) {
    case 0: m2l_mixed_run<P, PREC, ADJ, 0, 0>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
    case 1: m2l_mixed_run<P, PREC, ADJ, 1, 0>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
    case 2: m2l_mixed_run<P, PREC, ADJ, 0, 1>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
    default: m2l_mixed_run<P, PREC, ADJ, 1, 1>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
  }
}

template <int P, int PREC>
void launch_pp(const float *M, const float *gb_in, float *L, float *b, const TileMap &map, int ntiles, bool adjoint,
               const void *ops, hipStream_t s) {
  const int slots = 2 * num_cus();
  const int grid = ntiles < slots ? ntiles : slots;
  const float2 *X = reinterpret_cast<const float2 *>(M);
  float2 *Y = reinterpret_cast<float2 *>(L);
  const unsigned char *bank = static_cast<const unsigned char *>(ops);
  if (adjoint)
    hipLaunchKernelGGL((m2l_mixed_kernel<P, PREC, true>), dim3(grid), dim3(256), 0, s, X,
                       reinterpret_cast<const float2 *>(gb_in), Y, nullptr, bank, map, ntiles);
  else
    hipLaunchKernelGGL((m2l_mixed_kernel<P, PREC, false>), dim3(grid), dim3(256), 0, s, X, nullptr, Y,
                       reinterpret_cast<float2 *>(b), bank, map, ntiles);
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
