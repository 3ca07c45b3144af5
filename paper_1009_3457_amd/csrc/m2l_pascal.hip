// FP32 M2L in the Pascal form, with the fused reduction (Sec. 4.1), and its
// adjoint, on gfx950 matrix cores.
//
// The scaled operator factorises exactly (m2l_pascal_bank.h):
//     A~(d) = D1(d) B D2(d),  B[n][k] = C(n+k, k),  D1 = diag((-1)^n d^-(n+1)),  D2 = diag(d^-k).
// For each offset of the interaction list the wave scales its staged source
// coefficients by D2 (VALU), multiplies them by the constant real B (two
// MFMA chains, one for the real and one for the imaginary parts, on
// v_mfma_f32_16x16x4_f32 with B's fragments resident in registers for the
// whole kernel), and adds D1 times the product into the running local
// expansion (VALU), one offset behind so that it runs under the next
// offset's matrix products.  Per offset this is 2 p/4 MFMA k-steps per M
// tile, against 3 p/4 for the Gauss form of the complex product, and the
// operator occupies p/4 registers per M tile instead of 27 p/2.
//
// Work decomposition, staging and prefetch are those of the Gauss-form
// kernel (m2l_common.h, m2l_stage.h): persistent workgroups of four waves,
// one per child class, over 8x8 target tiles, three per compute unit for
// p <= 16 and two for p = 20 (PascalTab below).  The reduction over the list runs in a fixed offset
// order and each L~(t) is written once, so results are bit-reproducible.
//
// Offsets o and -o of a class's list are taken together (8 pairs of the 27):
// A~(-d) = D1(d) B' D2(d) with the constant B' = S1 B S2 (m2l_pascal_bank.h),
// so a pair costs the two products of its offsets but one D1 accumulation.
//
// The log row b rides in rows p .. p+3 of the product when p is not a
// multiple of 16 (m2l_pascal_bank.h); for p = 16 the loop forms it on the
// vector ALU from the D2-scaled sources it already holds.  The adjoint applies A~(d)^T = D2(d) B D1(d) over the
// class's own list with d = +o, and adds the log row's transpose per offset
// on the VALU: gM~_k += d^-k (Y_k - gb / k) for k >= 1 and
// gM~_0 += Y_0 + (log d + log h) gb.
#include "fmm2d_internal.h"
#include "m2l_bank.h"
#include "m2l_common.h"
#include "m2l_pascal_bank.h"
#include "m2l_stage.h"

namespace fmm2d {

namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int kPThreads = 256;  // one wave per child class

// The scaling tables of one direction (all four classes: 27 KB for p <= 16,
// 48 KB for p = 20) sit in LDS.  A table read is then a broadcast to each
// lane group of 16, and it stays out of the vector-memory counter, which
// retires loads in issue order: a table load issued behind the next tile's
// HBM prefetch would otherwise wait for the whole prefetch.  To fit the
// tables, the source block is single-buffered: the next tile's block is
// fetched into registers during the tile and stored between two barriers at
// its end.  Three workgroups fit per compute unit for p <= 16, two for
// p = 20 (163.6 of the 160 KiB).
template <int P>
struct PascalTab {
  using C = PascalCfg<P>;
  static constexpr int kIn4 = 27 * 4 * C::LI / 4;          // float4 of one class's "in" records
  static constexpr int kOut4 = 27 * C::MT * 4 * C::LO / 4;  // float4 of one class's "out" records
};

template <int P, bool ADJ>
struct LdsPascal {
  float x[XLayout<P>::kFloats];
  float2 gb[ADJ ? kRegBoxes + 1 : 1];
  float4 tab[4 * (PascalTab<P>::kIn4 + PascalTab<P>::kOut4)];
};

template <int P, bool WB = false>
constexpr int kPascalWgPerCu = P <= 16 && !WB ? 3 : 2;  // WB: the in-loop log row's registers

// Symmetric offsets taken in pairs (m2l_pascal_bank.h).  A pair holds two
// staged sources and B' in registers.  Every form takes them; the p = 16
// adjoint then spills a few registers at three workgroups per compute unit
// and is still 5-9% faster than taking every offset alone (6% at p = 20).
template <int P, bool ADJ>
constexpr bool kPascalPairs = true;

// ---------------------------------------------------- source block fetch --
// Target tiles are aligned 8x8 blocks of their level, so every box of a
// tile's 12x12 source block lies in one of the 3x3 aligned blocks around the
// tile, at a position inside that block fixed by the box's place in the
// source block.  The block is fetched in batches (G, q): chunk q (the float4
// of coefficients 2q, 2q+1) of every box of group G, one box per lane, with
//   G = 0  the central 8x8 boxes (lane = 8 ly + lx),
//   G = 1  the four 2x8 edge strips (16 lanes each),
//   G = 2  the four 2x2 corners (lanes 0..15).
// A lane's source address is then a wave-uniform block base, formed once per
// tile on the scalar unit, plus a per-lane constant, with q as an immediate
// offset; its LDS address is a per-lane constant plus an immediate.  Boxes
// outside the level read the bank's zero record.  Each wave (one per child
// class) takes a fixed range of the 3 p / 2 batches, and the adjoint's
// per-box log-row gradients of group G are fetched by the wave whose range
// starts group G.
template <int P>
struct BlockFetch {
  static constexpr int Q = P / 2;              // chunks per box record
  static constexpr int NB = 3 * Q;             // batches per block
  static constexpr int lo(int w) { return w * NB / 4; }
  static constexpr int hi(int w) { return (w + 1) * NB / 4; }
  static constexpr int kMaxB = (NB + 3) / 4;
  static constexpr bool touches(int w, int g) { return lo(w) < (g + 1) * Q && hi(w) > g * Q; }
  static constexpr bool owns_gb(int w, int g) { return lo(w) <= g * Q && hi(w) > g * Q; }
};

// Position (u, v) in the 12x12 source block of the box lane `lane` takes in
// group g (lanes 16..63 of the corner group repeat lanes 0..15).
__device__ inline void group_box(int g, int lane, int &u, int &v) {
  if (g == 0) {
    u = 2 + (lane & 7);
    v = 2 + (lane >> 3);
  } else if (g == 1) {
    const int e = lane >> 4, a = lane & 1, b = (lane >> 1) & 7;
    u = e == 0 ? a : e == 1 ? 10 + a : 2 + b;
    v = e == 0 || e == 1 ? 2 + b : e == 2 ? a : 10 + a;
  } else {
    const int c = (lane >> 2) & 3;
    u = ((c & 1) ? 10 : 0) + (lane & 1);
    v = ((c >> 1) ? 10 : 0) + ((lane >> 1) & 1);
  }
}

// Per-lane constants of the groups a wave fetches.
template <int P>
struct LaneBoxes {
  uint32_t m[3];     // Morton position of the lane's box in its aligned 8x8 block
  uint32_t lds[3];   // float index in the staged block of the lane's box, unit (kk 0, e 0)
  uint32_t slot[3];  // v * 12 + u
  int lx0, ly0;      // the central box's position in its aligned block
};

template <int P>
__device__ inline LaneBoxes<P> lane_boxes(int lane) {
  LaneBoxes<P> c;
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    int u, v;
    group_box(g, lane, u, v);
    c.m[g] = morton2(uint32_t((u + 6) & 7), uint32_t((v + 6) & 7));
    c.lds[g] = uint32_t(XLayout<P>::kRow * (v >> 1) + 6 * ((u & 1) + 2 * (v & 1)) + (u >> 1)) * 4u;
    c.slot[g] = uint32_t(v * kReg + u);
  }
  c.lx0 = lane & 7;
  c.ly0 = lane >> 3;
  return c;
}

template <int P, int W, bool ADJ>
struct Fetched {
  static constexpr int B0 = BlockFetch<P>::lo(W), NBW = BlockFetch<P>::hi(W) - B0;
  float4 v[NBW];
  float2 g[3];
};

// Issues the loads of wave W's batches of the block of tile `geo`.
template <int P, int W, bool ADJ>
__device__ __forceinline__ void fetch_issue(Fetched<P, W, ADJ> &f, const TileGeo &geo, const float2 *__restrict__ X,
                                            const float2 *__restrict__ gbin, const float *__restrict__ zero,
                                            const LaneBoxes<P> &lc, int lane) {
  using BF = BlockFetch<P>;
  using F = Fetched<P, W, ADJ>;
  // wave-uniform: the first box of each of the 3x3 aligned blocks around the
  // tile, with the neighbours' Morton codes formed from the tile's own by
  // dilated-integer steps; kNone if the block lies outside the level
  constexpr uint32_t kEven = 0x55555555u, kOdd = 0xAAAAAAAAu, kNone = ~0u;
  const int tX = geo.X0 >> 3, tY = geo.Y0 >> 3, nblk = (geo.nside + 7) >> 3;
  const uint32_t xm = geo.tm & kEven, ym = geo.tm & kOdd;
  const uint32_t xs[3] = {(xm - 1u) & kEven, xm, ((xm | kOdd) + 1u) & kEven};
  const uint32_t ys[3] = {(ym - 2u) & kOdd, ym, ((ym | kEven) + 2u) & kOdd};
  const bool okx[3] = {tX > 0, true, tX + 1 < nblk}, oky[3] = {tY > 0, true, tY + 1 < nblk};
  const uint32_t off = uint32_t(geo.off);
  auto block = [&](int cx, int cy) -> uint32_t {
    return okx[cx + 1] && oky[cy + 1] ? off + ((xs[cx + 1] | ys[cy + 1]) << 6) : kNone;
  };
  // the lane's block for group g: g = 1 by lane / 16 (left, right, bottom,
  // top), g = 2 by (lane / 4) % 4 (the four corners); a level smaller than a
  // tile has boxes past its side in the central block
  auto lane_block = [&](int g) -> uint32_t {
    if (g == 0)
      return geo.nside < kTile && (lc.lx0 >= geo.nside || lc.ly0 >= geo.nside) ? kNone : block(0, 0);
    if (g == 1) {
      const int e = lane >> 4;
      return e == 0 ? block(-1, 0) : e == 1 ? block(1, 0) : e == 2 ? block(0, -1) : block(0, 1);
    }
    const int c = (lane >> 2) & 3;
    return c == 0 ? block(-1, -1) : c == 1 ? block(1, -1) : c == 2 ? block(-1, 1) : block(1, 1);
  };
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    if (!BF::touches(W, g)) continue;
    const uint32_t first = lane_block(g);
    const bool in = first != kNone;
    const uint32_t box = first + lc.m[g];
    const char *a = in ? reinterpret_cast<const char *>(X + size_t(box) * P)
                       : reinterpret_cast<const char *>(zero) + lc.m[g] * (8u * P);
#pragma unroll
    for (int b = F::B0; b < F::B0 + F::NBW; ++b)
      if (b / BF::Q == g) f.v[b - F::B0] = *reinterpret_cast<const float4 *>(a + 16 * (b % BF::Q));
    if (ADJ && BF::owns_gb(W, g))
      f.g[g] = in && gbin ? gbin[box] : *reinterpret_cast<const float2 *>(zero + 2 * lc.m[g]);
  }
}

// Stores wave W's batches into the staged block (and the adjoint's
// gradients of the groups it owns).
template <int P, int W, bool ADJ>
__device__ __forceinline__ void fetch_store(const Fetched<P, W, ADJ> &f, float *__restrict__ lx,
                                            float2 *__restrict__ lgb, const LaneBoxes<P> &lc, int lane) {
  using BF = BlockFetch<P>;
  using F = Fetched<P, W, ADJ>;
  using XL = XLayout<P>;
  constexpr int S = P / 4;
#pragma unroll
  for (int b = F::B0; b < F::B0 + F::NBW; ++b) {
    const int g = b / BF::Q, q = b % BF::Q;
    if (g == 2 && lane >= 16) continue;
    float *dst = lx + lc.lds[g];
    const float4 c = f.v[b - F::B0];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = 2 * q + h, kk = k / S, sk = k - kk * S;
      dst[((kk * XL::NE + (sk >> 2)) * XL::kPlane) * 4 + (sk & 3)] = h ? c.z : c.x;
      dst[((kk * XL::NE + ((S + sk) >> 2)) * XL::kPlane) * 4 + ((S + sk) & 3)] = h ? c.w : c.y;
    }
  }
  if (ADJ) {
#pragma unroll
    for (int g = 0; g < 3; ++g)
      if (BF::owns_gb(W, g) && (g < 2 || lane < 16)) lgb[lc.slot[g]] = f.g[g];
  }
}

template <int P>
constexpr int kTabPer = (4 * (PascalTab<P>::kIn4 + PascalTab<P>::kOut4) + kPThreads - 1) / kPThreads;

// WB: the forward's log row b formed in the loop, for orders whose MFMA
// tiles have no spare rows (p = 16): from the D2-scaled sources each lane
// already holds, b gets -1/k (a pair's second offset: -(-1)^k / k) times
// scaled coefficient k >= 1, log d times coefficient 0, and log h times the
// sum of coefficient 0.
template <int P, bool ADJ, int CX, int CY, bool WB>
__device__ __forceinline__ void pascal_run(LdsPascal<P, ADJ> &sm, const float2 *__restrict__ X,
                                           const float2 *__restrict__ gbin, float2 *__restrict__ Y,
                                           float2 *__restrict__ bout, const float *__restrict__ bank,
                                           const TileMap &map, int ntiles, int tid,
                                           const float4 (&tv)[kTabPer<P>]) {
  using C = PascalCfg<P>;
  using B = PascalBank<P>;
  using XL = XLayout<P>;
  using Tb = PascalTab<P>;
  constexpr int S = C::S, MT = C::MT, LI = C::LI, LO = C::LO, NE = XL::NE;
  constexpr int cls = CX + 2 * CY, dir = ADJ ? 1 : 0;
  constexpr int sx = 1 - 2 * CX, sy = 1 - 2 * CY;  // mirror of class (0, 0)'s offsets
  const int lane = tid & 63;
  const int j = lane & 15, kk = lane >> 4;
  const int tx = 2 * (j & 3) + CX, ty = 2 * (j >> 2) + CY;


  // fragments of B and of B' (pairs only), held for the whole kernel
  constexpr int SP = kPascalPairs<P, ADJ> ? S : 1;
  float bf[MT][S], bfp[MT][SP];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
    for (int s = 0; s < S; ++s) bf[mt][s] = bank[B::bf_off + (mt * S + s) * 64 + lane];
#pragma unroll
    for (int s = 0; s < SP; ++s) bfp[mt][s] = bank[B::bfp_off + (mt * S + s) * 64 + lane];
  }

  // adjoint: -1/k for this lane's output rows k = 16 mt + 4 kk + r (k = 0: the
  // log d + log h term is added per offset; rows >= p: zero)
  // WB: this lane's log-row weights -1/k, k = S kk + s.  S is even, so the
  // parity of k is that of s, and a pair's second offset takes the same
  // weights with the sign of (-1)^s.
  static_assert(!WB || S % 2 == 0, "in-loop log row: p a multiple of 8");
  float wb1[WB ? S : 1];
  if constexpr (WB) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int k = S * kk + s;
      wb1[s] = k >= 1 ? -1.f / float(k) : 0.f;
    }
  }
  float cm[ADJ ? MT : 1][4], cm2[ADJ ? MT : 1][4];  // cm2: the negative offset's, -(-1)^k / k
  if (ADJ) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = 16 * mt + 4 * kk + r;
        cm[mt][r] = (k >= 1 && k < P) ? -1.f / float(k) : 0.f;
        cm2[mt][r] = (k & 1) ? -cm[mt][r] : cm[mt][r];
      }
  }

  // this lane's unit in the staged block for offset (0, 0) minus the class part
  const int lbase = (kk * NE * XL::kPlane + XL::kRow * (j >> 2) + (j & 3)) * 4;
  auto xoff = [&](int i) {  // compile-time after unrolling
    const int ox = sx * kOff00.ox[i], oy = sy * kOff00.oy[i];
    const int cu = CX + kHalo + ox, cv = CY + kHalo + oy;  // >= 0
    return (XL::kRow * (cv >> 1) + 6 * ((cu & 1) + 2 * (cv & 1)) + (cu >> 1)) * 4;
  };
  auto gbidx = [&](int i) {
    return (ty + kHalo + sy * kOff00.oy[i]) * kReg + (tx + kHalo + sx * kOff00.ox[i]);
  };
  const float ln2 = 0.69314718055994530942f;
  constexpr int kIssue = 1;  // offset at which the next tile's block is requested

  const LaneBoxes<P> lb = lane_boxes<P>(lane);
  const float *zero = bank + B::zero_off;
  // Forward map at p = 12 and 20: workgroups go to the 8 XCDs in turn
  // (b mod 8), and each XCD's workgroups start on a contiguous run of tiles
  // (XCD x holds G/8 of them, one more when x < G mod 8, after those of XCDs
  // 0..x-1), so neighbouring tiles, which share halo boxes, are fetched into
  // one L2; every workgroup then steps by G, which keeps the runs contiguous
  // in every round.  At 2^20 points, depth 8, p = 12 this halves the HBM
  // fetch (21.5 -> 10.2 MB per launch) and runs 0.6% faster.  Elsewhere each
  // workgroup starts on tile b: at p = 16 this order was 7.7% slower in both
  // directions, and the adjoint gained nothing measurable at p = 12 and 20.
  constexpr bool kXcdRuns = !ADJ && (P == 12 || P == 20);
  int t = int(blockIdx.x);
  if constexpr (kXcdRuns) {
    const int b = int(blockIdx.x), G = int(gridDim.x), x = b % 8, q = G / 8, rem = G % 8;
    t = x * q + (x < rem ? x : rem) + b / 8;
  }
  TileGeo geo = tile_geo(map, t);
  {
    // this wave's share of the first block, requested behind the scaling
    // tables; both are stored once both have arrived
    Fetched<P, cls, ADJ> f0;
    fetch_issue<P, cls, ADJ>(f0, geo, X, gbin, zero, lb, lane);
    constexpr int kAll = 4 * (Tb::kIn4 + Tb::kOut4);
#pragma unroll
    for (int r = 0; r < kTabPer<P>; ++r) {
      const int e = tid + r * kPThreads;
      if (e < kAll) sm.tab[e] = tv[r];
    }
    if constexpr (ADJ) {
      if (cls == 0 && lane == 0) sm.gb[kRegBoxes] = make_float2(0.f, 0.f);  // the empty slot
    }
    fetch_store<P, cls, ADJ>(f0, sm.x, sm.gb, lb, lane);
  }
  __syncthreads();
  for (;;) {
    asm volatile("" ::: "memory");  // LDS contents change every tile
    const int tn = t + int(gridDim.x);
    const bool has_next = tn < ntiles;
    const TileGeo ngeo = has_next ? tile_geo(map, tn) : geo;
    Fetched<P, cls, ADJ> pf;
    // The scaling tables are the same for every tile; opaque per-tile copies
    // of the lane group's record index keep the compiler from hoisting all
    // 27 offsets' table reads out of the tile loop.
    int qin = kk * (LI / 4), qout = kk * (LO / 4);
    asm volatile("" : "+v"(qin), "+v"(qout));
    // the adjoint's log d per offset, read with scalar loads: an opaque base
    // per tile keeps the 27 pairs from being hoisted into scalar registers
    const float *lgt = bank + B::lg_rec(dir, cls, 0);
    asm volatile("" : "+s"(lgt));
    const float logh = -float(geo.level) * ln2;

    const float *Lb = sm.x;
    f4_t accr[MT], acci[MT];  // the local expansion (rows 16 mt + 4 kk + r)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) accr[mt] = acci[mt] = f4_t{0.f, 0.f, 0.f, 0.f};

    // A step is one offset, or an offset and its negative (a pair): both
    // sources are scaled by the same D2 record, their products with B and B'
    // are summed in the MFMA accumulator, and the step's D1 record is applied
    // once.  xc/xc2: staged sources of the current step, xn/xn2 of the next.
    constexpr const PascalSteps &ST = kPascalPairs<P, ADJ> ? kPascalSteps : kPascalSingles;
    constexpr int NST = ST.n;
    float xc[4 * NE], xn[4 * NE], xc2[4 * NE], xn2[4 * NE];
    float ic[LI], in_[LI];                 // input scalings of step 0, of step j + 1
    float oc[MT][LO], on[MT][LO];          // output scalings of step j - 1, j
    // adjoint: gb of the step's offsets (x, y: first; z, w: second) and their log d
    float4 gbc = {0.f, 0.f, 0.f, 0.f}, gbn = gbc, lgc = gbc, lgn = gbc;
    f4_t pr[2][MT], pim[2][MT];            // products of steps j (slot j % 2) and j - 1

    auto load_x = [&](float (&dst)[4 * NE], int i) {
      const float *src = Lb + lbase + xoff(i);
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const float4 v = *reinterpret_cast<const float4 *>(src + e * XL::kPlane * 4);
        dst[4 * e] = v.x;
        dst[4 * e + 1] = v.y;
        dst[4 * e + 2] = v.z;
        dst[4 * e + 3] = v.w;
      }
    };
    auto load_in = [&](float (&dst)[LI], int i) {
#pragma unroll
      for (int e = 0; e < LI / 4; ++e) {
        const float4 v = sm.tab[cls * Tb::kIn4 + (i * 4) * (LI / 4) + qin + e];
        dst[4 * e] = v.x;
        dst[4 * e + 1] = v.y;
        dst[4 * e + 2] = v.z;
        dst[4 * e + 3] = v.w;
      }
    };
    auto load_out = [&](float (&dst)[MT][LO], int i) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int e = 0; e < LO / 4; ++e) {
          const float4 v = sm.tab[4 * Tb::kIn4 + cls * Tb::kOut4 + (i * MT + mt) * 4 * (LO / 4) + qout + e];
          dst[mt][4 * e] = v.x;
          dst[mt][4 * e + 1] = v.y;
          dst[mt][4 * e + 2] = v.z;
          dst[mt][4 * e + 3] = v.w;
        }
    };
    auto load_gb = [&](int i) {
      const float2 g = sm.gb[gbidx(i)];
      const float *lgp = lgt + 2 * i;  // uniform: scalar loads
      return make_float4(g.x, g.y, lgp[0], lgp[1]);
    };
    // running sum += D1 (product) for the step whose scalings are in o
    auto accumulate = [&](const f4_t (&yr)[MT], const f4_t (&yi)[MT], const float (&o)[MT][LO], float4 g,
                          float4 lg, bool pair) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float vr = yr[mt][r], vi = yi[mt][r];
          if (ADJ) {  // log rows' transposes: + c gb, c = -1/k (k >= 1), (log d + log h) at k = 0
            vr = fmaf(cm[mt][r], g.x, vr);
            vi = fmaf(cm[mt][r], g.y, vi);
            if (pair) {  // the negative offset's row: -(-1)^k / k
              vr = fmaf(cm2[mt][r], g.z, vr);
              vi = fmaf(cm2[mt][r], g.w, vi);
            }
            if (mt == 0 && r == 0 && kk == 0) {
              const float cr = lg.x + logh, ci = lg.y;
              vr = fmaf(cr, g.x, fmaf(-ci, g.y, vr));
              vi = fmaf(cr, g.y, fmaf(ci, g.x, vi));
              if (pair) {
                const float cr2 = lg.z + logh, ci2 = lg.w;
                vr = fmaf(cr2, g.z, fmaf(-ci2, g.w, vr));
                vi = fmaf(cr2, g.w, fmaf(ci2, g.z, vi));
              }
            }
          }
          const float dr = o[mt][2 * r], di = o[mt][2 * r + 1];
          accr[mt][r] = fmaf(dr, vr, fmaf(-di, vi, accr[mt][r]));
          acci[mt][r] = fmaf(dr, vi, fmaf(di, vr, acci[mt][r]));
        }
    };

    // scaled sources of a step: Re and Im of (input scaling) x, s < S
    float sr[S], si[S], sr2[S], si2[S];
    auto scale = [&](const float (&x)[4 * NE], const float (&c)[LI], float (&yr)[S], float (&yi)[S]) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float xr = x[s], xi = x[S + s];
        const float cr = c[2 * s], ci = c[2 * s + 1];
        yr[s] = fmaf(xr, cr, -xi * ci);
        yi[s] = fmaf(xr, ci, xi * cr);
      }
    };

    // WB: the log row's parts: the k >= 1 sum, and (log d + log h) times
    // coefficient 0, used by the lanes that hold k = 0
    float lbr = 0.f, lbi = 0.f, c0r = 0.f, c0i = 0.f;
    load_x(xc, ST.q1[0]);
    if (ST.q2[0] >= 0) load_x(xc2, ST.q2[0]);
    load_in(ic, ST.q1[0]);
    scale(xc, ic, sr, si);
    if (ST.q2[0] >= 0) scale(xc2, ic, sr2, si2);
#pragma unroll
    for (int j = 0; j < NST; ++j) {
      const int q1 = ST.q1[j], q2 = ST.q2[j];
      const bool pair = q2 >= 0;
      if (j + 1 < NST) {
        load_x(xn, ST.q1[j + 1]);
        if (ST.q2[j + 1] >= 0) load_x(xn2, ST.q2[j + 1]);
        load_in(in_, ST.q1[j + 1]);
      }
      load_out(on, q1);
      if (ADJ) {
        const float4 g = load_gb(q1);
        gbn = make_float4(g.x, g.y, 0.f, 0.f);
        lgn = make_float4(g.z, g.w, 0.f, 0.f);
        if (pair) {
          const float4 g2 = load_gb(q2);
          gbn.z = g2.x;
          gbn.w = g2.y;
          lgn.z = g2.z;
          lgn.w = g2.w;
        }
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        f4_t a = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[mt][0], sr[0], f4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
        for (int s = 1; s < S; ++s) a = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[mt][s], sr[s], a, 0, 0, 0);
        if (pair) {
#pragma unroll
          for (int s = 0; s < S; ++s) a = __builtin_amdgcn_mfma_f32_16x16x4f32(bfp[mt][s], sr2[s], a, 0, 0, 0);
        }
        pr[j & 1][mt] = a;
        f4_t b = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[mt][0], si[0], f4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
        for (int s = 1; s < S; ++s) b = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[mt][s], si[s], b, 0, 0, 0);
        if (pair) {
#pragma unroll
          for (int s = 0; s < S; ++s) b = __builtin_amdgcn_mfma_f32_16x16x4f32(bfp[mt][s], si2[s], b, 0, 0, 0);
        }
        pim[j & 1][mt] = b;
      }
      if (j > 0) accumulate(pr[(j - 1) & 1], pim[(j - 1) & 1], oc, gbc, lgc, ST.q2[j > 0 ? j - 1 : 0] >= 0);
      if constexpr (WB) {  // this step's log-row terms, from the sources its products read
        const float lr1 = lgt[2 * q1] + logh, li1 = lgt[2 * q1 + 1];
#pragma unroll
        for (int s = 0; s < S; ++s) {
          lbr = fmaf(wb1[s], sr[s], lbr);
          lbi = fmaf(wb1[s], si[s], lbi);
        }
        c0r = fmaf(lr1, sr[0], fmaf(-li1, si[0], c0r));
        c0i = fmaf(lr1, si[0], fmaf(li1, sr[0], c0i));
        if (pair) {
          const float lr2 = lgt[2 * q2] + logh, li2 = lgt[2 * q2 + 1];
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const float w = (s & 1) ? -wb1[s] : wb1[s];
            lbr = fmaf(w, sr2[s], lbr);
            lbi = fmaf(w, si2[s], lbi);
          }
          c0r = fmaf(lr2, sr2[0], fmaf(-li2, si2[0], c0r));
          c0i = fmaf(lr2, si2[0], fmaf(li2, sr2[0], c0i));
        }
      }
      // the next step's operands, under this step's products
      if (j + 1 < NST) {
        scale(xn, in_, sr, si);
        if (ST.q2[j + 1] >= 0) scale(xn2, in_, sr2, si2);
      }
      if (has_next) {
        // the whole next block at once, stored at the end of the tile
        if (j == kIssue) fetch_issue<P, cls, ADJ>(pf, ngeo, X, gbin, zero, lb, lane);
      }
      // FP32 matrix products and vector instructions do not run concurrently
      // on gfx950, and each switch from one to the other within a wave costs
      // cycles: the step's products go first, as one group, then the vector
      // work.  The step's LDS reads (the next step's sources and input
      // scalings, this step's output scalings) issue one after each product:
      // the wave issues in order, and a burst of them ahead of the products
      // would hold the matrix pipe while the LDS queue accepts them.
      // (Not for the p = 20 adjoint: its registers are taken, and the longer
      // live ranges would spill.)
      if constexpr (!(ADJ && P > 16)) {
        constexpr int kMaxDs = 2 * XL::NE + LI / 4 + MT * (LO / 4);
        const int nds = (j + 1 < NST ? XL::NE * (ST.q2[j + 1] >= 0 ? 2 : 1) + LI / 4 : 0) + MT * (LO / 4);
#pragma unroll
        for (int q = 0; q < kMaxDs; ++q) {
          if (q < nds) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
          }
        }
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 4 * S * MT, 0);  // at most: a pair's
      __builtin_amdgcn_sched_group_barrier(0x002, 1 << 12, 0);
      __builtin_amdgcn_sched_barrier(0);
      // The running sums feed only the epilogue: without this the compiler
      // sinks every step's accumulation toward it, keeping all the products
      // and their scalings live.  Opaque per step, they are formed here.
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) asm volatile("" : "+v"(accr[mt]), "+v"(acci[mt]));
      if constexpr (WB) asm volatile("" : "+v"(lbr), "+v"(lbi), "+v"(c0r), "+v"(c0i));
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int e = 0; e < LO; ++e) oc[mt][e] = on[mt][e];
      gbc = gbn;
      lgc = lgn;
    }
    accumulate(pr[(NST - 1) & 1], pim[(NST - 1) & 1], oc, gbc, lgc, ST.q2[NST - 1] >= 0);

    const int gx = geo.X0 + tx, gy = geo.Y0 + ty;
    const bool valid = gx < geo.nside && gy < geo.nside;
    const int64_t gbox = geo.off + morton2(uint32_t(gx), uint32_t(gy));
    if constexpr (WB) {  // the four lane groups of box j hold its k ranges
      lbr += __shfl_xor(lbr, 16);
      lbi += __shfl_xor(lbi, 16);
      lbr += __shfl_xor(lbr, 32);
      lbi += __shfl_xor(lbi, 32);
      if (valid && kk == 0) bout[gbox] = make_float2(lbr + c0r, lbi + c0i);
    }
    if (valid) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int n0 = 16 * mt + 4 * kk;
        if (n0 < P) {
          float4 *dst = reinterpret_cast<float4 *>(Y + gbox * P + n0);
          dst[0] = make_float4(accr[mt][0], acci[mt][0], accr[mt][1], acci[mt][1]);
          dst[1] = make_float4(accr[mt][2], acci[mt][2], accr[mt][3], acci[mt][3]);
        } else if (!ADJ && C::kLogInRows && n0 == P && bout) {
          bout[gbox] = make_float2(accr[mt][0] + accr[mt][1] + accr[mt][3] + logh * accr[mt][2],
                                   acci[mt][0] + acci[mt][1] + acci[mt][3] + logh * acci[mt][2]);
        }
      }
    }
    // every wave is done with this tile's block: replace it with the next
    __syncthreads();
    if (!has_next) break;
    fetch_store<P, cls, ADJ>(pf, sm.x, sm.gb, lb, lane);
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
      for (int s = 0; s < S; ++s) asm volatile("" : "+v"(bf[mt][s]));
#pragma unroll
      for (int s = 0; s < SP; ++s) asm volatile("" : "+v"(bfp[mt][s]));
    }
    t = tn;
    geo = ngeo;
  }
}

template <int P, bool ADJ, bool WB>
__global__ __launch_bounds__(kPThreads, (kPascalWgPerCu<P, WB>)) void m2l_pascal_kernel(const float2 *__restrict__ X,
                                                                  const float2 *__restrict__ gbin,
                                                                  float2 *__restrict__ Y, float2 *__restrict__ bout,
                                                                  const float *__restrict__ bank, TileMap map,
                                                                  int ntiles) {
  __shared__ __attribute__((aligned(16))) LdsPascal<P, ADJ> sm;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: the class
  if (int(blockIdx.x) >= ntiles) return;
  // this direction's scaling tables, all classes: requested here and stored
  // by pascal_run together with the first block
  using B = PascalBank<P>;
  using Tb = PascalTab<P>;
  constexpr int dir = ADJ ? 1 : 0, kIn = 4 * Tb::kIn4, kAll = kIn + 4 * Tb::kOut4;
  const float4 *tin = reinterpret_cast<const float4 *>(bank + B::tin_rec(dir, 0, 0));
  const float4 *tout = reinterpret_cast<const float4 *>(bank + B::tout_rec(dir, 0, 0, 0));
  float4 tv[kTabPer<P>];
#pragma unroll
  for (int r = 0; r < kTabPer<P>; ++r) {
    const int e = tid + r * kPThreads;
    tv[r] = e < kIn ? tin[e] : tout[e < kAll ? e - kIn : 0];
  }
  // every branch executes the same sequence of barriers; the branch is uniform per wave
  switch (wave) {
    case 0: pascal_run<P, ADJ, 0, 0, WB>(sm, X, gbin, Y, bout, bank, map, ntiles, tid, tv); break;
    case 1: pascal_run<P, ADJ, 1, 0, WB>(sm, X, gbin, Y, bout, bank, map, ntiles, tid, tv); break;
    case 2: pascal_run<P, ADJ, 0, 1, WB>(sm, X, gbin, Y, bout, bank, map, ntiles, tid, tv); break;
    default: pascal_run<P, ADJ, 1, 1, WB>(sm, X, gbin, Y, bout, bank, map, ntiles, tid, tv); break;
  }
}

template <int P>
void launch_pascal_p(const float *M, const float *gb_in, float *L, float *b, const TileMap &map, int ntiles,
                     bool adjoint, const void *ops, hipStream_t s) {
  constexpr bool kWB = !PascalCfg<P>::kLogInRows;  // the in-loop log row exists for this order
  const bool wb = kWB && !adjoint && b;              // no spare rows: b formed in the loop
  const int slots = (wb ? kPascalWgPerCu<P, kWB> : kPascalWgPerCu<P>) * num_cus();
  const int grid = ntiles < slots ? ntiles : slots;
  const float2 *X = reinterpret_cast<const float2 *>(M);
  float2 *Y = reinterpret_cast<float2 *>(L);
  const float *bank = static_cast<const float *>(ops);
  if (adjoint)
    hipLaunchKernelGGL((m2l_pascal_kernel<P, true, false>), dim3(grid), dim3(kPThreads), 0, s, X,
                       reinterpret_cast<const float2 *>(gb_in), Y, nullptr, bank, map, ntiles);
  else if (wb)
    hipLaunchKernelGGL((m2l_pascal_kernel<P, false, kWB>), dim3(grid), dim3(kPThreads), 0, s, X, nullptr, Y,
                       reinterpret_cast<float2 *>(b), bank, map, ntiles);
  else
    hipLaunchKernelGGL((m2l_pascal_kernel<P, false, false>), dim3(grid), dim3(kPThreads), 0, s, X, nullptr, Y,
                       reinterpret_cast<float2 *>(b), bank, map, ntiles);
}

}  // namespace

int launch_m2l_pascal(const float *M, const float *gb_in, float *L, float *b, int depth, int p, int lmin, int lmax,
                      bool adjoint, const void *ops, hipStream_t s) {
  (void)depth;
  TileMap map = make_tile_map(lmin, lmax);
  const int ntiles = map.first[map.nlev];
  switch (p) {
    case 8: launch_pascal_p<8>(M, gb_in, L, b, map, ntiles, adjoint, ops, s); break;
    case 12: launch_pascal_p<12>(M, gb_in, L, b, map, ntiles, adjoint, ops, s); break;
    case 16: launch_pascal_p<16>(M, gb_in, L, b, map, ntiles, adjoint, ops, s); break;
    case 20: launch_pascal_p<20>(M, gb_in, L, b, map, ntiles, adjoint, ops, s); break;
  }
  return check_launch(adjoint ? "m2l_backward (f32, Pascal form)" : "m2l (f32, Pascal form)");
}

}  // namespace fmm2d
