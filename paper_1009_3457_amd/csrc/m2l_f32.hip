// FP32 M2L contraction with the fused reduction (Sec. 4.1, steps 2-3 of the
// downward sweep), and its adjoint, on gfx950 matrix cores.
//
// For every target box t of levels lmin..lmax (scaled basis, see fmm2d.h):
//   L~(t) = sum_{o in O_c(t)} A~_o M~(t + o),
//   b(t)  = sum_o [ r_o . M~(t + o) + log(h) M~_0(t + o) ].
//
// Work decomposition (m2l_common.h): 8x8 target tiles.  The 16 boxes of one
// child class of a tile share one list of 27 offsets; for each offset they
// form the 16 columns of one product with a single operator (MFMA rows =
// output orders n, 16 per M tile), run on v_mfma_f32_16x16x4_f32 in Gauss's
// three-real-product form of the complex product (m2l_bank.h).  The
// reduction over the interaction list happens in the MFMA accumulators in a
// fixed offset order and each L~(t) is written once, so results are
// bit-reproducible.
//
// The kernel is persistent: workgroups walk the tiles g, g + G, g + 2G, ...
// A wave's class and offsets never change, so (p <= 16) its operator
// fragments are loaded into registers once and reused for every tile; only
// source expansions move.  The 12x12 source block of the next tile is fetched
// from HBM while the current tile's products run and written to the second
// of two LDS buffers.  Two shapes:
//   * p <= 12: one wave per class holds all 27 operators; four-wave
//     workgroups, two per compute unit, so one workgroup's tile epilogue runs
//     under the other's matrix products;
//   * p = 16, 20: two waves per class split the offset list 14 + 13 (eight-
//     wave workgroups, one per compute unit) and add their partial sums
//     through LDS, always first half + second half.  For p = 20 (two M tiles)
//     the operators are streamed from the L2-resident bank one offset ahead.
//
// Classes (1, .) use the mirror image of class (0, .)'s offset list, so an
// offset is (sx ox0, sy oy0) with signs fixed per wave.
//
// The log row b rides in spare MFMA rows when p is not a multiple of 16
// (m2l_bank.h); for p = 16 it is computed by m2l_logrow.hip.
//
// The adjoint uses the same stencil: since s in IL(t) <=> t in IL(s) and
// A~(d)^T = -A~(-d), the transpose gathers over s's own list with the negated
// forward operator of each offset.  Its log-row part, a contraction of gb
// over the offset list, runs as seven more MFMA k-steps (m2l_bank.h).
#include "fmm2d_internal.h"
#include "m2l_bank.h"
#include "m2l_common.h"
#include "m2l_stage.h"

namespace fmm2d {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));

template <int P>
struct F32Cfg {
  using B = F32Bank<P>;
  static constexpr int S = B::S, MT = B::MT, LS = B::LS;
  static constexpr int NA = 2 * S;                 // floats of an A or B fragment (Re, Im)
  static constexpr bool kRegBank = (MT == 1);      // operators held in registers
  static constexpr bool kLogInRows = B::kLogInRows;
  static constexpr int WPC = (P <= 12) ? 1 : 2;    // waves per class
  static constexpr int kThreads = 256 * WPC;
  static constexpr int kWgPerCu = (WPC == 1) ? 2 : 1;
  static constexpr int kChunks = StageCfg<P, kThreads>::kChunks;  // float4 chunks of a source block
  static constexpr int kPf = StageCfg<P, kThreads>::kPf;           // chunks per thread
  static constexpr int kPfA = (WPC == 1) ? (kPf + 1) / 2 : kPf;  // chunks of the first fetch batch
};

// Offset-list slice and adjoint log-row k-steps of a wave.
template <int P, int HALF>
struct Slice {
  static constexpr int WPC = F32Cfg<P>::WPC;
  static constexpr int I0 = (WPC == 1) ? 0 : HALF * 14;
  static constexpr int NI = (WPC == 1) ? 27 : (HALF ? 13 : 14);
  static constexpr int G0 = (WPC == 1) ? 0 : HALF * 4;
  static constexpr int NG = (WPC == 1) ? 7 : (HALF ? 3 : 4);
};

template <int P, bool ADJ>
struct LdsF32 {
  using C = F32Cfg<P>;
  static constexpr int MT = C::MT;
  // values one offset half hands to the other (two waves per class): the 3
  // Gauss products of the 2 accumulator registers the other half writes out,
  // per M tile, plus (adjoint) the second half's share of sum_o gb
  static constexpr bool kGbSumLanes = ADJ && !F32Bank<P>::kGbSumRow;
  static constexpr int kN = MT * 6 + (ADJ ? (kGbSumLanes ? 2 : 3) : 0);
  static constexpr int kRed = (C::WPC == 2) ? 2 * 2 * 4 * kN * 64 : 1;  // [parity][half][class][value][lane]
  float x[2][XLayout<P>::kFloats];
  float2 gb[2][ADJ ? kRegBoxes + 1 : 1];
  float red[kRed];
};

// First tile of this workgroup.  Workgroups go to the 8 XCDs in turn
// (b mod 8); XCD x's workgroups start on the x-th contiguous run of tiles
// (G/8 of them, one more when x < G mod 8) and step by G, so in every round
// the tiles that share halo boxes are fetched into one L2.
__device__ inline int f32_first_tile() {
  const int b = int(blockIdx.x), G = int(gridDim.x), x = b % 8, q = G / 8, rem = G % 8;
  return x * q + (x < rem ? x : rem) + b / 8;
}

template <int P, bool ADJ, int CX, int CY, int HALF>
__device__ __forceinline__ void m2l_f32_run(LdsF32<P, ADJ> &sm, const float2 *__restrict__ X,
                                            const float2 *__restrict__ gbin, float2 *__restrict__ Y,
                                            float2 *__restrict__ bout, const float *__restrict__ bank,
                                            const TileMap &map, int ntiles, int tid) {
  using C = F32Cfg<P>;
  using B = F32Bank<P>;
  using XL = XLayout<P>;
  using SL = Slice<P, HALF>;
  constexpr int S = C::S, MT = C::MT, LS = C::LS, NA = C::NA, WPC = C::WPC;
  constexpr int I0 = SL::I0, NI = SL::NI, G0 = SL::G0, NG = SL::NG;
  constexpr int kN = LdsF32<P, ADJ>::kN;
  constexpr bool kGbSumLanes = LdsF32<P, ADJ>::kGbSumLanes;

  constexpr int cls = CX + 2 * CY;
  constexpr int sx = 1 - 2 * CX, sy = 1 - 2 * CY;  // mirror of class (0, 0)'s offsets
  const int lane = tid & 63;
  const int j = lane & 15, kk = lane >> 4;
  const int tx = 2 * (j & 3) + CX, ty = 2 * (j >> 2) + CY;

  // The bank is read through a buffer descriptor: one per-lane VGPR offset
  // plus a scalar offset per fragment, so no per-offset vector addresses stay
  // live; reads past the bank's end would return zero.
  const __amdgpu_buffer_rsrc_t rsrc =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(bank), 0, int(B::total_floats * 4), 0x00020000);
  const int alane = lane * LS * 4;
  auto bank_frag = [&](int slot, int mt, int e) {
    const int soff = int((B::a_off + (size_t(slot) * MT + mt) * 64 * LS) * 4) + 16 * e;
    // explicitly typed result, cast whole: subscripting the builtin's
    // deduced result type compiles to a single-dword load here
    const u32x4_t u = __builtin_amdgcn_raw_buffer_load_b128(rsrc, alane, soff, 0);
    return __builtin_bit_cast(float4, u);
  };

  // operator fragments of this wave's offsets, held for the whole kernel (p <= 16)
  float areg[C::kRegBank ? NI : 1][NA];
  if (C::kRegBank) {
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int slot = slot_of(sx * kOff00.ox[I0 + i], sy * kOff00.oy[I0 + i]);
#pragma unroll
      for (int e = 0; e < LS / 4; ++e) {
        const float4 v = bank_frag(slot, 0, e);
        if (4 * e < NA) areg[i][4 * e] = v.x;
        if (4 * e + 1 < NA) areg[i][4 * e + 1] = v.y;
        if (4 * e + 2 < NA) areg[i][4 * e + 2] = v.z;
        if (4 * e + 3 < NA) areg[i][4 * e + 3] = v.w;
      }
    }
  }
  // adjoint log-row fragments (A) and this lane's gb source entries (B)
  float2 ga[ADJ ? NG : 1][MT];
  int gbo[ADJ ? NG : 1];
  if (ADJ) {
    const int glane = lane * 8;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int soff = int((B::ga_off + ((size_t(cls) * B::kGbSteps + G0 + g) * MT + mt) * 64 * 2) * 4);
        const u32x2_t u = __builtin_amdgcn_raw_buffer_load_b64(rsrc, glane, soff, 0);
        ga[g][mt] = __builtin_bit_cast(float2, u);
      }
      const int kap = 4 * (G0 + g) + kk;  // entry of the class's offset list
      int o = kRegBoxes;                  // the zero entry
#pragma unroll
      for (int q = 0; q < 27; ++q)
        if (q == kap) o = (ty + kHalo + sy * kOff00.oy[q]) * kReg + (tx + kHalo + sx * kOff00.ox[q]);
      gbo[g] = o;
    }
  }

  // this lane's unit in the staged block for offset (0, 0) minus the class
  // part; per offset only a compile-time constant is added
  const int lbase = (kk * XL::NE * XL::kPlane + XL::kRow * (j >> 2) + (j & 3)) * 4;
  auto xoff = [&](int i) {  // compile-time after unrolling
    const int ox = sx * kOff00.ox[I0 + i], oy = sy * kOff00.oy[I0 + i];
    const int cu = CX + kHalo + ox, cv = CY + kHalo + oy;  // >= 0
    return (XL::kRow * (cv >> 1) + 6 * ((cu & 1) + 2 * (cv & 1)) + (cu >> 1)) * 4;
  };
  const float ln2 = 0.69314718055994530942f;
  // The next tile's source block is fetched in two batches while this tile's
  // products run; each batch is written to the other LDS buffer (released by
  // every wave at the previous tile's barrier) a few offsets after its loads.
  constexpr int kIssueA = 1, kStoreA = (WPC == 1) ? 12 : NI - 3;
  constexpr int kIssueB = (WPC == 1) ? 13 : NI, kStoreB = (WPC == 1) ? 24 : NI;

  int t = f32_first_tile();  // the tile the kernel's prologue staged
  TileGeo geo = tile_geo(map, t);
  int cur = 0;
  for (;;) {
    // LDS contents change every tile: keep the compiler from caching LDS
    // reads in registers across tiles
    asm volatile("" ::: "memory");
    const int tn = t + int(gridDim.x);
    const bool has_next = tn < ntiles;
    const TileGeo ngeo = has_next ? tile_geo(map, tn) : geo;
    Prefetch<P, C::kThreads> pf;
    // opaque copy of the thread index: the fetch addresses derived from it
    // are recomputed where used instead of being kept live across the tile
    int ftid = tid;
    asm volatile("" : "+v"(ftid));

    const float *L = sm.x[cur];
    f4_t acc[MT][3];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[mt][q] = f4_t{0.f, 0.f, 0.f, 0.f};

    float bcur[LS], bnxt[LS];
    constexpr int AM = C::kRegBank ? 1 : MT, AL = C::kRegBank ? 1 : LS;
    float acur[AM][AL], anxt[AM][AL];
    auto load_b = [&](float (&dst)[LS], int i) {
      const float *bs = L + lbase + xoff(i);
#pragma unroll
      for (int e = 0; e < LS / 4; ++e) {
        const float4 v = *reinterpret_cast<const float4 *>(bs + e * XL::kPlane * 4);
        dst[4 * e] = v.x;
        dst[4 * e + 1] = v.y;
        dst[4 * e + 2] = v.z;
        dst[4 * e + 3] = v.w;
      }
    };
    auto load_a = [&](float (&dst)[AM][AL], int i) {
      if (!C::kRegBank) {
        const int slot = slot_of(sx * kOff00.ox[I0 + i], sy * kOff00.oy[I0 + i]);
#pragma unroll
        for (int mt = 0; mt < AM; ++mt)
#pragma unroll
          for (int e = 0; e < AL / 4; ++e) {
            const float4 v = bank_frag(slot, mt, e);
            dst[mt][4 * e] = v.x;
            dst[mt][4 * e + 1] = v.y;
            dst[mt][4 * e + 2] = v.z;
            dst[mt][4 * e + 3] = v.w;
          }
      }
    };

    load_b(bcur, 0);
    load_a(acur, 0);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      if (i + 1 < NI) {
        load_b(bnxt, i + 1);
        load_a(anxt, i + 1);
      }
      // the loads above stay ahead of this offset's products (the scheduler
      // would otherwise sink them next to their first use)
      __builtin_amdgcn_sched_barrier(0);
      // each accumulator takes a chain of S products (chained accumulation
      // issues faster than rotating accumulators)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const float a0 = C::kRegBank ? areg[i][s] : acur[mt % AM][s % AL];
          acc[mt][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, bcur[s], acc[mt][0], 0, 0, 0);
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const float a1 = C::kRegBank ? areg[i][S + s] : acur[mt % AM][(S + s) % AL];
          acc[mt][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, bcur[S + s], acc[mt][1], 0, 0, 0);
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const float a0 = C::kRegBank ? areg[i][s] : acur[mt % AM][s % AL];
          const float a1 = C::kRegBank ? areg[i][S + s] : acur[mt % AM][(S + s) % AL];
          const float a2 = a0 + a1, b2 = bcur[s] + bcur[S + s];  // third Gauss operands
          acc[mt][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, b2, acc[mt][2], 0, 0, 0);
        }
      }
      if (has_next) {
        if (i == kIssueA) prefetch_issue<P, C::kThreads, ADJ>(pf, ngeo, X, gbin, ftid, 0, C::kPfA);
        if (i == kStoreA) prefetch_store<P, C::kThreads, ADJ>(pf, sm.x[cur ^ 1], sm.gb[cur ^ 1], ftid, 0, C::kPfA);
        if (i == kIssueB) prefetch_issue<P, C::kThreads, ADJ>(pf, ngeo, X, gbin, ftid, C::kPfA, C::kPf);
        if (i == kStoreB) prefetch_store<P, C::kThreads, ADJ>(pf, sm.x[cur ^ 1], sm.gb[cur ^ 1], ftid, C::kPfA, C::kPf);
      }
      // FP32 matrix products and vector instructions do not run concurrently
      // on gfx950, and each switch between them within a wave costs cycles:
      // the offset's vector work (the third Gauss operands, which feed its
      // products, and any block fetch) goes first, then its products as one
      // group.
      __builtin_amdgcn_sched_group_barrier(0x002, 1 << 12, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 3 * S * MT, 0);
      // keep the software pipeline as written: operands of offset i+1 are
      // loaded during offset i, not hoisted further (register pressure)
      __builtin_amdgcn_sched_barrier(0);
      if (i + 1 < NI) {
#pragma unroll
        for (int e = 0; e < LS; ++e) bcur[e] = bnxt[e];
#pragma unroll
        for (int mt = 0; mt < AM; ++mt)
#pragma unroll
          for (int e = 0; e < AL; ++e) acur[mt][e] = anxt[mt][e];
      }
    }
    if (has_next && kIssueB >= NI) {  // second batch not yet issued (short slices)
      prefetch_issue<P, C::kThreads, ADJ>(pf, ngeo, X, gbin, ftid, C::kPfA, C::kPf);
      prefetch_store<P, C::kThreads, ADJ>(pf, sm.x[cur ^ 1], sm.gb[cur ^ 1], ftid, C::kPfA, C::kPf);
    }

    // adjoint log-row part: k-steps over the offset list (B operand = gb)
    float gsr = 0.f, gsi = 0.f;
    if (ADJ) {
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const float2 gv = sm.gb[cur][gbo[g]];
        if (kGbSumLanes) {
          gsr += gv.x;
          gsi += gv.y;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const float2 a = ga[g][mt];
          acc[mt][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, gv.x, acc[mt][0], 0, 0, 0);
          acc[mt][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, gv.y, acc[mt][1], 0, 0, 0);
          acc[mt][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x + a.y, gv.x + gv.y, acc[mt][2], 0, 0, 0);
        }
      }
    }

    const int gx = geo.X0 + tx, gy = geo.Y0 + ty;
    const bool valid = gx < geo.nside && gy < geo.nside;
    const int64_t gbox = geo.off + morton2(uint32_t(gx), uint32_t(gy));
    const float logh = -float(geo.level) * ln2;

    if (WPC == 1) {
      // ---- one wave per class: its accumulators are the whole sum.  The
      // output goes out first; the barrier that follows only orders the LDS
      // buffers (the next tile's block is complete; this tile's block is no
      // longer read).
      float sgr = 0.f, sgi = 0.f;  // adjoint: sum of gb over the list, for n = 0
      if (ADJ) {
        if (kGbSumLanes) {
          sgr = gsr + __shfl_xor(gsr, 16);
          sgi = gsi + __shfl_xor(gsi, 16);
          sgr += __shfl_xor(sgr, 32);
          sgi += __shfl_xor(sgi, 32);
        } else {  // row p + 2 holds -sum gb: fetch it from the lane that owns it
          constexpr int row = P + 2, mtr = row / 16, kkr = (row % 16) / 4, er = row % 4;
          const float t1 = acc[mtr][0][er], t2 = acc[mtr][1][er], t3 = acc[mtr][2][er];
          sgr = -__shfl(t1 - t2, j + 16 * kkr);
          sgi = -__shfl(t3 - t1 - t2, j + 16 * kkr);
        }
      }
      if (valid) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int n0 = 16 * mt + 4 * kk;
          float yr[4], yi[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float t1 = acc[mt][0][q], t2 = acc[mt][1][q], t3 = acc[mt][2][q];
            yr[q] = ADJ ? t2 - t1 : t1 - t2;
            yi[q] = ADJ ? t1 + t2 - t3 : t3 - t1 - t2;
          }
          if (n0 < P) {
            if (ADJ && n0 == 0) {
              yr[0] += logh * sgr;
              yi[0] += logh * sgi;
            }
            float4 *dst = reinterpret_cast<float4 *>(Y + gbox * P + n0);
            dst[0] = make_float4(yr[0], yi[0], yr[1], yi[1]);
            dst[1] = make_float4(yr[2], yi[2], yr[3], yi[3]);
          } else if (!ADJ && C::kLogInRows && n0 == P && bout) {
            bout[gbox] = make_float2(yr[0] + logh * yr[1], yi[0] + logh * yi[1]);
          }
        }
      }
      __syncthreads();
    } else {
      // ---- two waves per class: both publish their partial sums; then each
      // writes half of the output rows (accumulator registers 2h, 2h + 1 of
      // every lane), always adding first half + second half.  One barrier per
      // tile: the partials are double buffered, and the source buffer read in
      // this tile is rewritten only after the next tile's barrier.
      float *red = sm.red + size_t(cur) * (2 * 4 * kN * 64);
      float *pub = red + (HALF * 4 + cls) * kN * 64;
      const float *oth = red + ((1 - HALF) * 4 + cls) * kN * 64;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int g = 0; g < 3; ++g)
#pragma unroll
          for (int h = 0; h < 2; ++h) pub[((mt * 3 + g) * 2 + h) * 64 + lane] = acc[mt][g][2 * (1 - HALF) + h];
      if (ADJ && HALF == 1) {
        if (kGbSumLanes) {
          pub[(MT * 6) * 64 + lane] = gsr;
          pub[(MT * 6 + 1) * 64 + lane] = gsi;
        } else {
          constexpr int row = P + 2, mtr = row / 16, er = row % 4;
#pragma unroll
          for (int g = 0; g < 3; ++g) pub[(MT * 6 + g) * 64 + lane] = acc[mtr][g][er];
        }
      }
      __syncthreads();
      // combined Gauss product g of accumulator register 2 HALF + h (first + second half)
      auto comb = [&](int mt, int g, int h) {
        const float own = acc[mt][g][2 * HALF + h], other = oth[((mt * 3 + g) * 2 + h) * 64 + lane];
        return HALF == 0 ? own + other : other + own;
      };
      float sgr = 0.f, sgi = 0.f;
      if (ADJ && HALF == 0) {
        if (kGbSumLanes) {
          sgr = gsr + oth[(MT * 6) * 64 + lane];
          sgi = gsi + oth[(MT * 6 + 1) * 64 + lane];
          sgr += __shfl_xor(sgr, 16);
          sgi += __shfl_xor(sgi, 16);
          sgr += __shfl_xor(sgr, 32);
          sgi += __shfl_xor(sgi, 32);
        } else {
          constexpr int row = P + 2, mtr = row / 16, kkr = (row % 16) / 4, er = row % 4;
          const float t1 = acc[mtr][0][er] + oth[(MT * 6) * 64 + lane];
          const float t2 = acc[mtr][1][er] + oth[(MT * 6 + 1) * 64 + lane];
          const float t3 = acc[mtr][2][er] + oth[(MT * 6 + 2) * 64 + lane];
          sgr = -__shfl(t1 - t2, j + 16 * kkr);
          sgi = -__shfl(t3 - t1 - t2, j + 16 * kkr);
        }
      }
      if (valid) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int n0 = 16 * mt + 4 * kk;  // rows n0 .. n0 + 3 live in this lane
          if (n0 < P || (!ADJ && C::kLogInRows && HALF == 0 && n0 == P && bout)) {
            float yr[2], yi[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const float t1 = comb(mt, 0, h), t2 = comb(mt, 1, h), t3 = comb(mt, 2, h);
              yr[h] = ADJ ? t2 - t1 : t1 - t2;
              yi[h] = ADJ ? t1 + t2 - t3 : t3 - t1 - t2;
            }
            if (n0 < P) {
              if (ADJ && HALF == 0 && n0 == 0) {
                yr[0] += logh * sgr;
                yi[0] += logh * sgi;
              }
              *reinterpret_cast<float4 *>(Y + gbox * P + n0 + 2 * HALF) = make_float4(yr[0], yi[0], yr[1], yi[1]);
            } else {  // rows p, p + 1: log row and the sum of M~_0
              bout[gbox] = make_float2(yr[0] + logh * yr[1], yi[0] + logh * yi[1]);
            }
          }
        }
      }
    }
    if (!has_next) break;
    // Opaque per tile: stops the per-use sums Ar + Ai from being hoisted out
    // of the tile loop into extra registers (emits no instructions).  It sits
    // at the end of the tile, where the operators are in use anyway, so the
    // first tile still waits for each operator only at its first use.
    if (C::kRegBank) {
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int e = 0; e < NA; ++e) asm volatile("" : "+v"(areg[i][e]));
    }
    cur ^= 1;
    t = tn;
    geo = ngeo;
  }
}

template <int P, bool ADJ>
__global__ __launch_bounds__(F32Cfg<P>::kThreads, F32Cfg<P>::kWgPerCu) void m2l_f32_kernel(
    const float2 *__restrict__ X, const float2 *__restrict__ gbin, float2 *__restrict__ Y, float2 *__restrict__ bout,
    const float *__restrict__ bank, TileMap map, int ntiles) {
  using C = F32Cfg<P>;
  __shared__ __attribute__((aligned(16))) LdsF32<P, ADJ> sm;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: class and half in SGPRs
  if (int(blockIdx.x) >= ntiles) return;
  {
    Prefetch<P, C::kThreads> pf;
    const TileGeo g = tile_geo(map, f32_first_tile());
    prefetch_issue<P, C::kThreads, ADJ>(pf, g, X, gbin, tid, 0, C::kPf);
    prefetch_store<P, C::kThreads, ADJ>(pf, sm.x[0], sm.gb[0], tid, 0, C::kPf);
    if (ADJ && tid == 0) sm.gb[1][kRegBoxes] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  // Every branch executes the same sequence of barriers (the tile loop is
  // identical); the branch is uniform per wave.
  if constexpr (C::WPC == 1) {
    switch (wave) {
      case 0: m2l_f32_run<P, ADJ, 0, 0, 0>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
      case 1: m2l_f32_run<P, ADJ, 1, 0, 0>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
      case 2: m2l_f32_run<P, ADJ, 0, 1, 0>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
      default: m2l_f32_run<P, ADJ, 1, 1, 0>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
    }
  } else {
    switch (wave) {
      case 0: m2l_f32_run<P, ADJ, 0, 0, 0>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
      case 1: m2l_f32_run<P, ADJ, 1, 0, 0>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
      case 2: m2l_f32_run<P, ADJ, 0, 1, 0>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
      case 3: m2l_f32_run<P, ADJ, 1, 1, 0>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
      case 4: m2l_f32_run<P, ADJ, 0, 0, 1>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
      case 5: m2l_f32_run<P, ADJ, 1, 0, 1>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
      case 6: m2l_f32_run<P, ADJ, 0, 1, 1>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
      default: m2l_f32_run<P, ADJ, 1, 1, 1>(sm, X, gbin, Y, bout, bank, map, ntiles, tid); break;
    }
  }
}

int num_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cached[dev] = v;
  }
  return cached[dev];
}

template <int P>
static void launch_p(const float *M, const float *gb_in, float *L, float *b, const TileMap &map, int ntiles,
                     bool adjoint, const void *ops, hipStream_t s) {
  using C = F32Cfg<P>;
  const int slots = C::kWgPerCu * num_cus();
  const int grid = ntiles < slots ? ntiles : slots;
  const float2 *X = reinterpret_cast<const float2 *>(M);
  float2 *Y = reinterpret_cast<float2 *>(L);
  const float *bank = static_cast<const float *>(ops);
  if (adjoint)
    hipLaunchKernelGGL((m2l_f32_kernel<P, true>), dim3(grid), dim3(C::kThreads), 0, s, X,
                       reinterpret_cast<const float2 *>(gb_in), Y, nullptr, bank, map, ntiles);
  else
    hipLaunchKernelGGL((m2l_f32_kernel<P, false>), dim3(grid), dim3(C::kThreads), 0, s, X, nullptr, Y,
                       reinterpret_cast<float2 *>(b), bank, map, ntiles);
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
  int rc = check_launch(adjoint ? "m2l_backward (f32)" : "m2l (f32)");
  if (rc == FMM2D_OK && !adjoint && b && (p % 16) == 0)  // no spare rows: separate log-row pass
    rc = launch_m2l_logrow_fwd(M, b, p, lmin, lmax, static_cast<const float *>(ops) + F32Bank<16>::r_off, s);
  return rc;
}

}  // namespace fmm2d
