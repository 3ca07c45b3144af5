// M2L operator generation (Sec. 4.1, Eq. (eq:M2Lmat)): every entry of every
// offset's scaled operator is computed in FP64 on the device (exact binomial,
// power by repeated complex multiplication of d^-1) and rounded once to the
// storage precision.  The paper builds the entries on the fly inside each
// translation; here the 40 distinct operators of a given p are built once and
// reused by every level, every launch and the adjoint.
#include <cmath>

#include "fmm2d_internal.h"
#include "m2l_bank.h"
#include "m2l_hankel_bank.h"
#include "m2l_mixed_bank.h"
#include "m2l_pascal_bank.h"

namespace fmm2d {

// C(a, b) in FP64: the running product c * (a - b + i) / i stays an exact
// integer below 2^53 for a <= 40.
__device__ inline double binom_f64(int a, int b) {
  double c = 1.0;
  for (int i = 1; i <= b; ++i) c = c * double(a - b + i) / double(i);
  return c;
}

// d^-m for a complex d with |d| >= 2, by m - 1 multiplications of d^-1.
__device__ inline cd cpow_neg(cd d, int m) {
  double den = d.re * d.re + d.im * d.im;
  cd inv = {d.re / den, -d.im / den};
  cd r = {1.0, 0.0};
  for (int i = 0; i < m; ++i) r = cmul(r, inv);
  return r;
}

// Entry (n, k) of the scaled operator for offset (ox, oy): d = -(ox + i oy).
__device__ inline cd m2l_entry(int ox, int oy, int n, int k) {
  cd d = {double(-ox), double(-oy)};
  cd v = cpow_neg(d, n + k + 1);
  double c = binom_f64(n + k, k) * ((n & 1) ? -1.0 : 1.0);
  return {c * v.re, c * v.im};
}

// Log-potential row entry k for a given d: log d (k = 0), -d^-k / k.
__device__ inline cd log_row_entry(double dre, double dim, int k) {
  if (k == 0) return {0.5 * log(dre * dre + dim * dim), atan2(dim, dre)};
  cd v = cpow_neg(cd{dre, dim}, k);
  return {-v.re / double(k), -v.im / double(k)};
}

__device__ inline bool slot_used(int slot, int &ox, int &oy) {
  ox = slot % 7 - 3;
  oy = slot / 7 - 3;
  return (ox < -1 || ox > 1 || oy < -1 || oy > 1);
}

template <int P>
__global__ void f32_bank_kernel(float *bank) {
  using B = F32Bank<P>;
  const size_t total = B::total_floats;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < total; i += size_t(gridDim.x) * blockDim.x) {
    float v = 0.0f;
    if (i < B::a_off + B::a_floats) {
      size_t e = i - B::a_off;
      int pos = int(e % B::LS);
      size_t r = e / B::LS;
      int lane = int(r % 64);
      r /= 64;
      int mt = int(r % B::MT);
      int slot = int(r / B::MT);
      int ox, oy;
      if (pos < 2 * B::S && slot_used(slot, ox, oy)) {
        int part = pos / B::S, s = pos % B::S;
        int n = 16 * mt + lane % 16;
        int k = B::S * (lane / 16) + s;
        cd a = {0.0, 0.0};
        if (n < P) a = m2l_entry(ox, oy, n, k);
        else if (B::kLogInRows && n == P) a = log_row_entry(double(-ox), double(-oy), k);
        else if (B::kLogInRows && n == P + 1) a = {k == 0 ? 1.0 : 0.0, 0.0};
        v = float(part == 0 ? a.re : a.im);
      }
    } else if (i >= B::r_off && i < B::r_off + B::r_floats) {
      size_t e = i - B::r_off;
      int ri = int(e % 2);
      size_t r = e / 2;
      int k = int(r % P);
      int slot = int(r / P);
      int ox, oy;
      if (slot_used(slot, ox, oy)) {
        // d = -o, negated as integers: a zero component must be +0 so that the
        // principal branch of log d is taken (arg d = +pi on the negative axis)
        cd rv = log_row_entry(double(-ox), double(-oy), k);
        v = float(ri ? rv.im : rv.re);
      }
    } else if (i >= B::ga_off && i < B::ga_off + B::ga_floats) {
      size_t e = i - B::ga_off;
      int ri = int(e % 2);
      size_t r = e / 2;
      int lane = int(r % 64);
      r /= 64;
      int mt = int(r % B::MT);
      r /= B::MT;
      int g = int(r % B::kGbSteps);
      int cls = int(r / B::kGbSteps);
      int kappa = 4 * g + lane / 16;  // entry of the class's offset list
      int n = 16 * mt + lane % 16;
      if (kappa < 27) {
        int ox = (1 - 2 * (cls & 1)) * kOff00.ox[kappa];
        int oy = (1 - 2 * (cls >> 1)) * kOff00.oy[kappa];
        if (n < P) {
          cd rv = log_row_entry(double(ox), double(oy), n);  // row at d = +o
          v = -float(ri ? rv.im : rv.re);
        } else if (B::kGbSumRow && n == P + 2) {
          v = ri ? 0.0f : -1.0f;
        }
      }
    }
    bank[i] = v;
  }
}

// ------------------------------------------------------- Pascal-form bank --
// d of offset q of class cls for the forward (dir 0: d = -o) or adjoint
// (dir 1: d = +o) translation; the negation is done on the integers so a zero
// component is +0 (principal branch of log d).
__device__ inline cd pascal_d(int dir, int cls, int q) {
  const int ox = (1 - 2 * (cls & 1)) * kOff00.ox[q], oy = (1 - 2 * (cls >> 1)) * kOff00.oy[q];
  return dir == 0 ? cd{double(-ox), double(-oy)} : cd{double(ox), double(oy)};
}

template <int P>
__global__ void pascal_bank_kernel(float *bank) {
  using B = PascalBank<P>;
  using C = PascalCfg<P>;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < B::total_floats; i += stride) {
    double v = 0.0;
    if (i < B::bf_off + B::bf_floats || (i >= B::bfp_off && i < B::bfp_off + B::bfp_floats)) {
      // B, or B' = S1 B S2 for the negative of an offset
      const bool neg = i >= B::bfp_off;
      const size_t e = i - (neg ? B::bfp_off : B::bf_off);
      const int lane = int(e % 64), s = int((e / 64) % C::S), mt = int(e / 64 / C::S);
      const int n = 16 * mt + lane % 16, k = C::S * (lane / 16) + s;
      const double sk = (k & 1) ? -1.0 : 1.0;
      if (n < P) v = neg ? -sk * ((n & 1) ? -1.0 : 1.0) * binom_f64(n + k, k) : binom_f64(n + k, k);
      else if (C::kLogInRows && n == P) v = k == 0 ? 0.0 : (neg ? sk : 1.0) * (-1.0 / double(k));
      else if (C::kLogInRows && (n == P + 1 || n == P + 2)) v = k == 0 ? 1.0 : 0.0;
      else if (C::kLogInRows && n == P + 3) v = neg && k == 0 ? 1.0 : 0.0;
    } else if (i >= B::tin_off && i < B::tin_off + B::tin_floats) {
      size_t e = i - B::tin_off;
      const int pos = int(e % C::LI);
      e /= C::LI;
      const int kk = int(e % 4), q = int((e / 4) % 27), cls = int((e / 108) % 4), dir = int(e / 432);
      if (pos < 2 * C::S) {
        const int k = C::S * kk + pos / 2;
        const cd d = pascal_d(dir, cls, q);
        cd w = cpow_neg(d, dir == 0 ? k : k + 1);
        if (dir == 1 && (k & 1)) w = {-w.re, -w.im};
        v = (pos & 1) ? w.im : w.re;
      }
    } else if (i >= B::tout_off && i < B::tout_off + B::tout_floats) {
      size_t e = i - B::tout_off;
      const int pos = int(e % C::LO);
      e /= C::LO;
      const int kk = int(e % 4);
      e /= 4;
      const int mt = int(e % C::MT);
      e /= C::MT;
      const int q = int(e % 27), cls = int((e / 27) % 4), dir = int(e / 108);
      const int n = 16 * mt + 4 * kk + pos / 2;
      const cd d = pascal_d(dir, cls, q);
      cd w = {0.0, 0.0};
      if (n < P) {
        w = cpow_neg(d, dir == 0 ? n + 1 : n);
        if (dir == 0 && (n & 1)) w = {-w.re, -w.im};
      } else if (dir == 0 && C::kLogInRows) {
        if (n == P || n == P + 2) {
          w = {1.0, 0.0};
        } else if (n == P + 1) {
          w = log_row_entry(d.re, d.im, 0);
        } else if (n == P + 3 && pascal_partner(q) > q) {
          // the pair's second offset: log(-d) - log d, +-i pi.  -d is taken
          // from the partner's own entry, formed from integers like d, so a
          // zero component is +0 and log(-d) is on the principal branch.
          const cd d2 = pascal_d(dir, cls, pascal_partner(q));
          const cd a = log_row_entry(d2.re, d2.im, 0), b = log_row_entry(d.re, d.im, 0);
          w = {a.re - b.re, a.im - b.im};
        }
      }
      v = (pos & 1) ? w.im : w.re;
    } else if (i >= B::lg_off && i < B::lg_off + B::lg_floats) {
      const size_t e = i - B::lg_off;
      const int ri = int(e % 2), q = int((e / 2) % 27), cls = int((e / 54) % 4), dir = int(e / 216);
      const cd d = pascal_d(dir, cls, q);
      const cd w = log_row_entry(d.re, d.im, 0);
      v = ri ? w.im : w.re;
    }
    bank[i] = float(v);
  }
}

// ---------------------------------------------------- split-precision bank --
// Entry of the interleaved real embedding of a complex value (m2l_mixed_bank.h).
__device__ inline double embed(cd a, int pr, int pc) {
  return pr == 0 ? (pc == 0 ? a.re : -a.im) : (pc == 0 ? a.im : a.re);
}

template <int PREC>
__device__ inline uint16_t round16(double v) {
  if constexpr (PREC == FMM2D_BF16X3) return __builtin_bit_cast(uint16_t, __bf16(float(v)));
  else return __builtin_bit_cast(uint16_t, _Float16(float(v)));
}

template <int PREC>
__device__ inline double widen16(uint16_t h) {
  if constexpr (PREC == FMM2D_BF16X3) return double(float(__builtin_bit_cast(__bf16, h)));
  else return double(float(__builtin_bit_cast(_Float16, h)));
}

// hi (part 0) or lo (part 1) of the two-term split of v
template <int PREC>
__device__ inline uint16_t split16(double v, int part) {
  const uint16_t hi = round16<PREC>(v);
  return part == 0 ? hi : round16<PREC>(v - widen16<PREC>(hi));
}

template <int P, int PREC>
__global__ void mixed_bank_kernel(unsigned char *bank) {
  using B = MixedBank<P>;
  using C = MixCfg<P>;
  constexpr int R = C::R;
  uint16_t *h = reinterpret_cast<uint16_t *>(bank);
  const size_t n16 = B::r_off / 2;  // sections a and ga with their padding
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n16; i += stride) {
    uint16_t out = 0;
    const size_t byte = 2 * i;
    if (byte < B::a_off + B::a_bytes) {
      size_t e16 = i - B::a_off / 2;
      const int e = int(e16 % 8), lane = int((e16 / 8) % 64);
      size_t rest = e16 / 512;
      const int ks = int(rest % C::KS);
      rest /= C::KS;
      const int mt = int(rest % C::MT), slot = int(rest / C::MT);
      const int rho = 16 * mt + lane % 16, kap = 32 * ks + 8 * (lane / 16) + e;
      const int seg = kap / R, c = kap % R;
      int ox, oy;
      if (seg < 3 && slot_used(slot, ox, oy)) {
        double v = 0.0;
        if (rho < R) {
          v = embed(m2l_entry(ox, oy, rho / 2, c / 2), rho % 2, c % 2);
        } else if (C::kLogRows && rho < R + 2) {
          v = embed(log_row_entry(double(-ox), double(-oy), c / 2), rho - R, c % 2);
        } else if (C::kLogRows && rho < R + 4) {
          v = (c == rho - R - 2) ? 1.0 : 0.0;  // Re / Im of M~_0
        }
        out = split16<PREC>(v, seg == 2 ? 1 : 0);
      }
    } else if (byte >= B::ga_off && byte < B::ga_off + B::ga_bytes) {
      size_t e16 = i - B::ga_off / 2;
      const int e = int(e16 % 8), lane = int((e16 / 8) % 64);
      size_t rest = e16 / 512;
      const int t = int(rest % 2);
      rest /= 2;
      const int mt = int(rest % C::MT);
      rest /= C::MT;
      const int part = int(rest % 2), cls = int(rest / 2);
      const int rho = 16 * mt + lane % 16, kap = 32 * t + 8 * (lane / 16) + e;
      const int q = kap / 2, pc = kap % 2;  // entry of the class's offset list, Re / Im of gb
      if (q < 27 && rho < R) {
        const int ox = (1 - 2 * (cls & 1)) * kOff00.ox[q];
        const int oy = (1 - 2 * (cls >> 1)) * kOff00.oy[q];
        const cd rv = log_row_entry(double(ox), double(oy), rho / 2);  // row at d = +o
        out = split16<PREC>(-embed(rv, rho % 2, pc), part);
      }
    }
    h[i] = out;
  }
  float *r = reinterpret_cast<float *>(bank + B::r_off);
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < size_t(kSlots) * P * 2; i += stride) {
    const int ri = int(i % 2), k = int((i / 2) % P), slot = int(i / 2 / P);
    int ox, oy;
    float v = 0.f;
    if (slot_used(slot, ox, oy)) {
      const cd rv = log_row_entry(double(-ox), double(-oy), k);
      v = float(ri ? rv.im : rv.re);
    }
    r[i] = v;
  }
}

// Hankel-form bank (m2l_hankel_bank.h), all in FP64 except the FP32 log rows.
// G^_o[f] = sum_m g_m(d) exp(-2 pi i f m / N) with g_m(d) = m! rho^-m d^-(m+1),
// d = -o; the angle of each term is reduced exactly, (f m) mod N.
template <int P>
__global__ void hankel_bank_kernel(unsigned char *bank) {
  using B = HankelBank<P>;
  constexpr int N = B::N;
  const double rho = HankelCfg<P>::rho();
  const double two_pi = 6.283185307179586476925286766559;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  const size_t i0 = blockIdx.x * size_t(blockDim.x) + threadIdx.x;
  cd *ghat = reinterpret_cast<cd *>(bank + B::ghat_off);
  for (size_t i = i0; i < size_t(kSlots) * N; i += stride) {
    const int f = int(i % N), slot = int(i / N);
    int ox, oy;
    cd acc = {0.0, 0.0};
    if (slot_used(slot, ox, oy)) {
      const cd d = {double(-ox), double(-oy)};
      const double den = d.re * d.re + d.im * d.im;
      const cd dinv = {d.re / den, -d.im / den};
      cd dp = dinv;      // d^-(m+1)
      double c = 1.0;    // m! rho^-m
      for (int m = 0; m <= 2 * P - 2; ++m) {
        if (m > 0) {
          c *= double(m) / rho;
          dp = cmul(dp, dinv);
        }
        const double ang = -two_pi * double((f * m) % N) / double(N);
        const cd w = {cos(ang), sin(ang)};
        const cd t = cmul(dp, w);
        acc.re += c * t.re;
        acc.im += c * t.im;
      }
    }
    ghat[i] = acc;
  }
  double *dr = reinterpret_cast<double *>(bank + B::dr_off);
  double *dl = reinterpret_cast<double *>(bank + B::dl_off);
  if (i0 == 0) {
    double c = 1.0;  // rho^k / k!
    for (int k = 0; k < P; ++k) {
      if (k > 0) c *= rho / double(k);
      dr[k] = c;
      dl[k] = (k & 1) ? -c : c;
    }
  }
  cd *tw = reinterpret_cast<cd *>(bank + B::tw_off);
  for (size_t i = i0; i < size_t(N); i += stride) {
    const double ang = -two_pi * double(i) / double(N);
    tw[i] = {cos(ang), sin(ang)};
  }
  float *r = reinterpret_cast<float *>(bank + B::r_off);
  for (size_t i = i0; i < size_t(kSlots) * P * 2; i += stride) {
    const int ri = int(i % 2), k = int((i / 2) % P), slot = int(i / 2 / P);
    int ox, oy;
    float v = 0.f;
    if (slot_used(slot, ox, oy)) {
      const cd rv = log_row_entry(double(-ox), double(-oy), k);
      v = float(ri ? rv.im : rv.re);
    }
    r[i] = v;
  }
}

size_t mixed_bank_bytes(int p, int precision) {
  if (precision != FMM2D_BF16X3 && precision != FMM2D_F16X3) return 0;
  switch (p) {
    case 8: return MixedBank<8>::total_bytes;
    case 12: return MixedBank<12>::total_bytes;
    case 16: return MixedBank<16>::total_bytes;
    case 20: return MixedBank<20>::total_bytes;
  }
  return 0;
}

template <int PREC>
static void launch_mixed_bank(int p, unsigned char *bank, hipStream_t s) {
  dim3 grid(512), block(256);
  switch (p) {
    case 8: hipLaunchKernelGGL((mixed_bank_kernel<8, PREC>), grid, block, 0, s, bank); break;
    case 12: hipLaunchKernelGGL((mixed_bank_kernel<12, PREC>), grid, block, 0, s, bank); break;
    case 16: hipLaunchKernelGGL((mixed_bank_kernel<16, PREC>), grid, block, 0, s, bank); break;
    case 20: hipLaunchKernelGGL((mixed_bank_kernel<20, PREC>), grid, block, 0, s, bank); break;
  }
}

int launch_mixed_ops(int p, int precision, void *ops, hipStream_t s) {
  unsigned char *bank = static_cast<unsigned char *>(ops);
  if (precision == FMM2D_BF16X3) launch_mixed_bank<FMM2D_BF16X3>(p, bank, s);
  else launch_mixed_bank<FMM2D_F16X3>(p, bank, s);
  return check_launch("m2l split-precision operator bank");
}

size_t m2l_ops_bytes(int p, int precision) {
  if (!p_supported(p)) return 0;
  if (precision == FMM2D_F32) return f32_bank_bytes(p);
  if (precision == FMM2D_F32_PASCAL) return pascal_bank_bytes(p);
  if (precision == FMM2D_F64_HANKEL) return hankel_bank_bytes(p);
  return mixed_bank_bytes(p, precision);
}

int launch_m2l_ops(int p, int precision, void *ops, hipStream_t s) {
  if (precision == FMM2D_F64_HANKEL) {
    unsigned char *bank = static_cast<unsigned char *>(ops);
    dim3 grid(64), block(256);
    switch (p) {
      case 8: hipLaunchKernelGGL(hankel_bank_kernel<8>, grid, block, 0, s, bank); break;
      case 12: hipLaunchKernelGGL(hankel_bank_kernel<12>, grid, block, 0, s, bank); break;
      case 16: hipLaunchKernelGGL(hankel_bank_kernel<16>, grid, block, 0, s, bank); break;
      case 20: hipLaunchKernelGGL(hankel_bank_kernel<20>, grid, block, 0, s, bank); break;
    }
    return check_launch("m2l Hankel-form operator bank");
  }
  if (precision == FMM2D_F32_PASCAL) {
    float *bank = static_cast<float *>(ops);
    dim3 grid(512), block(256);
    switch (p) {
      case 8: hipLaunchKernelGGL(pascal_bank_kernel<8>, grid, block, 0, s, bank); break;
      case 12: hipLaunchKernelGGL(pascal_bank_kernel<12>, grid, block, 0, s, bank); break;
      case 16: hipLaunchKernelGGL(pascal_bank_kernel<16>, grid, block, 0, s, bank); break;
      case 20: hipLaunchKernelGGL(pascal_bank_kernel<20>, grid, block, 0, s, bank); break;
    }
    return check_launch("m2l Pascal-form operator bank");
  }
  if (precision != FMM2D_F32) return launch_mixed_ops(p, precision, ops, s);
  float *bank = static_cast<float *>(ops);
  dim3 grid(512), block(256);
  switch (p) {
    case 8: hipLaunchKernelGGL(f32_bank_kernel<8>, grid, block, 0, s, bank); break;
    case 12: hipLaunchKernelGGL(f32_bank_kernel<12>, grid, block, 0, s, bank); break;
    case 16: hipLaunchKernelGGL(f32_bank_kernel<16>, grid, block, 0, s, bank); break;
    case 20: hipLaunchKernelGGL(f32_bank_kernel<20>, grid, block, 0, s, bank); break;
  }
  return check_launch("m2l operator bank");
}

}  // namespace fmm2d
