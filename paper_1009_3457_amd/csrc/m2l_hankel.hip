// M2L in the Hankel form (m2l_hankel_bank.h), with the fused reduction over
// the interaction list (Sec. 4.1), and its adjoint, in FP64 arithmetic.
//
// Every translation of Eq. (eq:M2Lmat) is a Hankel product between two
// diagonal scalings, so the sum over a target's 27 offsets is taken in the
// frequency domain: per target and frequency, 27 complex multiply-adds of an
// operator spectrum with a source spectrum, instead of a p x p product per
// translation.  One workgroup per 8x8 target tile (persistent over tiles; the
// next tile's source block is fetched into registers while one is computed):
//   1. stage the 12x12 source block, scaled (rho^k / k!) and reversed, in LDS;
//   2. transform each of its 144 records (DFT of length N = 2p by Horner's
//      rule at the N roots of unity) into LDS;
//   3. accumulate each target's spectrum over its class's 27 offsets, a lane
//      per (frequency, class, block of targets), reading each operator
//      spectrum once per offset for all its targets;
//   4. evaluate the inverse transform at the p outputs n + p - 1 (Horner
//      again), scale by (-1)^n rho^n / (n! N) and write the local expansion.
// The adjoint runs the same steps with the roles of the two scalings
// exchanged, over each source's own list with the mirrored operator.
// Arithmetic and intermediate storage are FP64; inputs and outputs are the
// library's complex float expansions.  The sums run in a fixed order, so
// results are bit-reproducible.
#include "fmm2d_internal.h"
#include "m2l_bank.h"
#include "m2l_common.h"
#include "m2l_hankel_bank.h"

namespace fmm2d {

namespace {

__device__ inline cd cfma(cd a, cd b, cd c) {  // a b + c
  return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}

constexpr int kThreads = 512;  // 8 waves: two per SIMD

template <int P>
struct HankelLds {
  static constexpr int N = 2 * P;
  cd zb[kRegBoxes * P];  // scaled, reversed source records; then the 64 target spectra [64][N]
  cd zs[kRegBoxes * N];  // source spectra
  cd tw[N];              // exp(-2 pi i j / N)
  double s_in[P];        // input scaling (rho^k / k!, or (-1)^k rho^k / k! in the adjoint)
  double s_out[P];       // output scaling, divided by N
};
static_assert(64 * 2 <= kRegBoxes, "the 64 target spectra (N = 2p each) fit in the records' space");
static_assert(kTile == 8, "step 3 splits each class's 16 targets of an 8x8 tile");

// Workgroups that fit on a compute unit side by side (LDS bound).
template <int P>
constexpr int kHankelWgPerCu = (160 * 1024) / int(sizeof(HankelLds<P>)) > 0 ? (160 * 1024) / int(sizeof(HankelLds<P>)) : 1;

// The records of tile t (complex float, unscaled), kIt per lane, zero
// outside the level or past the tile count.
template <int P, int kIt>
__device__ inline void fetch_records(const float2 *__restrict__ X, const TileMap &map, int t, int ntiles, int tid,
                                     float2 (&m)[kIt]) {
  constexpr int kRec = kRegBoxes * P;
#pragma unroll
  for (int it = 0; it < kIt; ++it) m[it] = make_float2(0.f, 0.f);
  if (t >= ntiles) return;
  int level, tile;
  tile_of(map, t, level, tile);
  const int nside = 1 << level;
  uint32_t tX, tY;
  unmorton2(uint32_t(tile), tX, tY);
  const int X0 = int(tX) * kTile - kHalo, Y0 = int(tY) * kTile - kHalo;
  const int64_t off = level_off(level);
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int e = tid + it * kThreads;
    const int u = e / P, k = e % P;
    const int gx = X0 + u % kReg, gy = Y0 + u / kReg;
    if (e < kRec && gx >= 0 && gy >= 0 && gx < nside && gy < nside)
      m[it] = X[(off + morton2(uint32_t(gx), uint32_t(gy))) * P + k];
  }
}

template <int P, bool ADJ>
__global__ __launch_bounds__(kThreads) void m2l_hankel_kernel(const float2 *__restrict__ X, float2 *__restrict__ Y,
                                                              const unsigned char *__restrict__ bank, TileMap map,
                                                              int ntiles) {
  using B = HankelBank<P>;
  constexpr int N = 2 * P;
  constexpr int kRec = kRegBoxes * P, kIt = (kRec + kThreads - 1) / kThreads;
  __shared__ HankelLds<P> sm;
  const int tid = threadIdx.x;
  const cd *ghat = reinterpret_cast<const cd *>(bank + B::ghat_off);
  const double *dr = reinterpret_cast<const double *>(bank + B::dr_off);
  const double *dl = reinterpret_cast<const double *>(bank + B::dl_off);
  const cd *twg = reinterpret_cast<const cd *>(bank + B::tw_off);
  for (int e = tid; e < N; e += kThreads) sm.tw[e] = twg[e];
  for (int e = tid; e < P; e += kThreads) {
    sm.s_in[e] = ADJ ? dl[e] : dr[e];
    sm.s_out[e] = (ADJ ? dr[e] : dl[e]) / double(N);
  }

  // step 3 lanes: (frequency f, class c, block jb of the class's 16 targets),
  // kTB blocks of kTPB targets each
  constexpr int kTB = 4 * N * 8 <= kThreads ? 8 : 4 * N * 4 <= kThreads ? 4 : 4 * N * 2 <= kThreads ? 2 : 1;
  constexpr int kTPB = 16 / kTB;
  const bool bact = tid < 4 * N * kTB;
  const int bf = tid % N, bc = (tid / N) % 4, bjb = tid / (4 * N);
  const int bcx = bc & 1, bcy = bc >> 1;
  const int bsx = 1 - 2 * bcx, bsy = 1 - 2 * bcy;
  const cd *gl = ghat + bf;  // this lane's frequency of every operator spectrum

  constexpr int FQ = (N % 8 == 0) ? N / 8 : N / 4;  // frequencies per step-2 item
  constexpr int NQ = N / FQ;
  float2 m[kIt];
  fetch_records<P>(X, map, blockIdx.x, ntiles, tid, m);
  for (int t = blockIdx.x; t < ntiles; t += int(gridDim.x)) {
    int level, tile;
    tile_of(map, t, level, tile);
    const int nside = 1 << level;
    uint32_t tX, tY;
    unmorton2(uint32_t(tile), tX, tY);
    const int X0 = int(tX) * kTile, Y0 = int(tY) * kTile;
    const int64_t off = level_off(level);

    __syncthreads();  // the previous tile's readers are done
    // 1. scaled, reversed source records; then the next tile's records are
    //    fetched while this one is computed
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int e = tid + it * kThreads;
      if (e < kRec) {
        const int u = e / P, k = e % P;
        const double sc = sm.s_in[k];
        sm.zb[u * P + (P - 1 - k)] = {sc * double(m[it].x), sc * double(m[it].y)};
      }
    }
    __syncthreads();
    fetch_records<P>(X, map, t + int(gridDim.x), ntiles, tid, m);
    // 2. source spectra: Z^[f] = sum_j zb[j] w^(f j), w = exp(-2 pi i / N)
    for (int e = tid; e < kRegBoxes * NQ; e += kThreads) {
      const int u = e / NQ, fq = e % NQ;
      cd z[P];
#pragma unroll
      for (int j = 0; j < P; ++j) z[j] = sm.zb[u * P + j];
#pragma unroll
      for (int i = 0; i < FQ; ++i) {
        const int f = fq * FQ + i;
        const cd x = sm.tw[f];
        cd acc = z[P - 1];
#pragma unroll
        for (int j = P - 2; j >= 0; --j) acc = cfma(acc, x, z[j]);
        sm.zs[u * N + f] = acc;
      }
    }
    __syncthreads();
    // 3. target spectra: the lane's kTPB targets as independent sums over the
    //    class's 27 offsets, in a fixed order
    cd *yh = sm.zb;
    if (bact) {
      cd acc[kTPB];
#pragma unroll
      for (int jj = 0; jj < kTPB; ++jj) acc[jj] = {0.0, 0.0};
#pragma unroll 3
      for (int q = 0; q < 27; ++q) {
        const int ox = bsx * kOff00.ox[q], oy = bsy * kOff00.oy[q];
        const cd gq = gl[(ADJ ? slot_of(-ox, -oy) : slot_of(ox, oy)) * N];
#pragma unroll
        for (int jj = 0; jj < kTPB; ++jj) {
          const int j = bjb * kTPB + jj;  // class-local target 0..15
          const int tx = 2 * (j & 3) + bcx, ty = 2 * (j >> 2) + bcy;
          const int u = (ty + kHalo + oy) * kReg + (tx + kHalo + ox);
          acc[jj] = cfma(gq, sm.zs[u * N + bf], acc[jj]);
        }
      }
#pragma unroll
      for (int jj = 0; jj < kTPB; ++jj) {
        const int j = bjb * kTPB + jj;
        const int tx = 2 * (j & 3) + bcx, ty = 2 * (j >> 2) + bcy;
        yh[(ty * kTile + tx) * N + bf] = acc[jj];
      }
    }
    __syncthreads();
    // 4. the p outputs i = n + p - 1 of the inverse transform:
    //    sum_f Y^[f] v^f, v = exp(+2 pi i i / N), then the output scaling
    for (int e = tid; e < 64 * P; e += kThreads) {
      const int tb = e / P, n = e % P;
      const int gx = X0 + (tb & 7), gy = Y0 + (tb >> 3);
      const cd w0 = sm.tw[(n + P - 1) % N];
      const cd v = {w0.re, -w0.im};
      cd acc = yh[tb * N + N - 1];
#pragma unroll 8
      for (int f = N - 2; f >= 0; --f) acc = cfma(acc, v, yh[tb * N + f]);
      if (gx < nside && gy < nside) {
        const double sc = sm.s_out[n];
        Y[(off + morton2(uint32_t(gx), uint32_t(gy))) * P + n] = make_float2(float(sc * acc.re), float(sc * acc.im));
      }
    }
  }
}

template <int P>
void launch_hankel_p(const float *M, float *L, const TileMap &map, int ntiles, bool adjoint, const void *ops,
                     hipStream_t s) {
  const int slots = kHankelWgPerCu<P> * num_cus();
  const int grid = ntiles < slots ? ntiles : slots;
  const float2 *X = reinterpret_cast<const float2 *>(M);
  float2 *Y = reinterpret_cast<float2 *>(L);
  const unsigned char *bank = static_cast<const unsigned char *>(ops);
  if (adjoint)
    hipLaunchKernelGGL((m2l_hankel_kernel<P, true>), dim3(grid), dim3(kThreads), 0, s, X, Y, bank, map, ntiles);
  else
    hipLaunchKernelGGL((m2l_hankel_kernel<P, false>), dim3(grid), dim3(kThreads), 0, s, X, Y, bank, map, ntiles);
}

size_t hankel_r_off(int p) {
  switch (p) {
    case 8: return HankelBank<8>::r_off;
    case 12: return HankelBank<12>::r_off;
    case 16: return HankelBank<16>::r_off;
    case 20: return HankelBank<20>::r_off;
  }
  return 0;
}

}  // namespace

int launch_m2l_hankel(const float *M, const float *gb_in, float *L, float *b, int depth, int p, int lmin, int lmax,
                      bool adjoint, const void *ops, hipStream_t s) {
  (void)depth;
  const TileMap map = make_tile_map(lmin, lmax);
  const int ntiles = map.first[map.nlev];
  switch (p) {
    case 8: launch_hankel_p<8>(M, L, map, ntiles, adjoint, ops, s); break;
    case 12: launch_hankel_p<12>(M, L, map, ntiles, adjoint, ops, s); break;
    case 16: launch_hankel_p<16>(M, L, map, ntiles, adjoint, ops, s); break;
    case 20: launch_hankel_p<20>(M, L, map, ntiles, adjoint, ops, s); break;
  }
  int rc = check_launch(adjoint ? "m2l_backward (Hankel form)" : "m2l (Hankel form)");
  if (rc != FMM2D_OK) return rc;
  // the log-potential row, in its own pass (it is not a Hankel product)
  const float *r = reinterpret_cast<const float *>(static_cast<const unsigned char *>(ops) + hankel_r_off(p));
  if (!adjoint && b) rc = launch_m2l_logrow_fwd(M, b, p, lmin, lmax, r, s);
  if (adjoint && gb_in) rc = launch_m2l_logrow_bwd(gb_in, L, p, lmin, lmax, r, s);
  return rc;
}

}  // namespace fmm2d
