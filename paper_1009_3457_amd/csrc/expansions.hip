// Upward sweep (P2M, M2M), L2L and L2P (Sec. 2.1, stages 2-4) in the scaled
// basis of fmm2d.h, and the plain transposes of each for gradients.
//
// These stages are O(N p) or O(boxes p^2) and not the hot path: one thread
// per box or per point.  M2M and L2L shift coefficient vectors held in
// registers by repeated Horner steps; L2P finds a target's leaf from its
// coordinates.  L2L and L2P run in FP64 (the
// deep-level accumulation of local expansions).
#include "fmm2d_internal.h"

namespace fmm2d {

// Find the leaf of sorted item i: the largest m with ls[m] <= i.
__device__ inline int64_t leaf_of(const int32_t *__restrict__ ls, int64_t nleaf, int64_t i) {
  int64_t lo = 0, hi = nleaf;  // invariant: ls[lo] <= i < ls[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (int64_t(ls[mid]) <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Leaf of sorted target t at `z`: the leaf the tree build assigns to z
// (floor of z 2^depth, clamped), confirmed against the leaf ranges; a search
// of the ranges when they disagree.
__device__ inline int64_t leaf_of_point(float2 z, const int32_t *__restrict__ ls, int64_t nleaf, int depth,
                                        int64_t t) {
  const float side = float(1 << depth);  // z 2^depth is exact in FP32
  const int lim = (1 << depth) - 1;
  const int ix = min(max(int(floorf(z.x * side)), 0), lim), iy = min(max(int(floorf(z.y * side)), 0), lim);
  const int64_t m = morton2(uint32_t(ix), uint32_t(iy));
  if (int64_t(ls[m]) <= t && t < int64_t(ls[m + 1])) return m;
  return leaf_of(ls, nleaf, t);
}

// (x - c)/h for a point and the centre of leaf m at level `depth`.
__device__ inline float2 scaled_offset(float2 p, uint32_t m, int depth) {
  uint32_t ix, iy;
  unmorton2(m, ix, iy);
  const float h = ldexpf(1.f, -depth);
  const float cx = (float(ix) + 0.5f) * h, cy = (float(iy) + 0.5f) * h;
  return make_float2((p.x - cx) * float(1 << depth), (p.y - cy) * float(1 << depth));
}

// ------------------------------------------------------------------ P2M --

template <int P>
__global__ void p2m_kernel(const float2 *__restrict__ xy, const float *__restrict__ q, const int32_t *__restrict__ ls,
                           int depth, float2 *__restrict__ M) {
  const int64_t nleaf = int64_t(1) << (2 * depth);
  const int64_t m = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (m >= nleaf) return;
  float ar[P], ai[P];
#pragma unroll
  for (int k = 0; k < P; ++k) ar[k] = ai[k] = 0.f;
  for (int32_t s = ls[m]; s < ls[m + 1]; ++s) {
    const float2 w = scaled_offset(xy[s], uint32_t(m), depth);
    float pr = q[s], pi = 0.f;  // q w^k
#pragma unroll
    for (int k = 0; k < P; ++k) {
      ar[k] += pr;
      ai[k] += pi;
      const float tr = pr * w.x - pi * w.y;
      pi = pr * w.y + pi * w.x;
      pr = tr;
    }
  }
  float2 *out = M + (level_off(depth) + m) * P;
#pragma unroll
  for (int k = 0; k < P; ++k) out[k] = make_float2(ar[k], ai[k]);
}

// P2M^T and its z-derivative for every sorted source.
template <int P>
__global__ void p2m_backward_kernel(const float2 *__restrict__ xy, const float *__restrict__ q,
                                    const int32_t *__restrict__ ls, int64_t n, int depth,
                                    const float2 *__restrict__ gM, float *__restrict__ gq, float2 *__restrict__ G) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int64_t nleaf = int64_t(1) << (2 * depth);
  if (i >= n || i >= int64_t(ls[nleaf])) return;
  const int64_t m = leaf_of(ls, nleaf, i);
  const float2 w = scaled_offset(xy[i], uint32_t(m), depth);
  const float2 *g = gM + (level_off(depth) + m) * P;
  float qr = 0.f, qi = 0.f, dr = 0.f, di = 0.f;
  float pr = 1.f, pi = 0.f;  // w^k
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const float2 gk = g[k];
    qr += gk.x * pr - gk.y * pi;
    qi += gk.x * pi + gk.y * pr;
    if (k + 1 < P) {  // d/dz of gM_{k+1} w^{k+1} = (k+1) gM_{k+1} w^k
      const float2 g1 = g[k + 1];
      dr += float(k + 1) * (g1.x * pr - g1.y * pi);
      di += float(k + 1) * (g1.x * pi + g1.y * pr);
    }
    const float tr = pr * w.x - pi * w.y;
    pi = pr * w.y + pi * w.x;
    pr = tr;
  }
  (void)qi;
  const float sc = q[i] * float(1 << depth);  // q / h
  gq[i] = qr;
  G[i] = make_float2(sc * dr, sc * di);
}

// ------------------------------------------------------- shifts by u --
// A shift between a box and its parent applies the binomial matrix of the
// offset u = (+-1 +- i)/2 (child centre minus parent centre, in child
// widths) to a coefficient vector held in registers, by repeated Horner
// steps: p(p-1)/2 complex multiply-adds, no binomial or power tables.

// a_n <- sum_{m>=n} C(m,n) u^(m-n) a_m  (re-expanding a Taylor series about a point shifted by u)
template <int P, typename T>
__device__ inline void shift_down(T (&ar)[P], T (&ai)[P], T ur, T ui) {
#pragma unroll
  for (int k = 0; k < P - 1; ++k)
#pragma unroll
    for (int j = P - 2; j >= k; --j) {
      ar[j] += ur * ar[j + 1] - ui * ai[j + 1];
      ai[j] += ur * ai[j + 1] + ui * ar[j + 1];
    }
}

// a_k <- sum_{j<=k} C(k,j) u^(k-j) a_j  (the transpose of shift_down)
template <int P, typename T>
__device__ inline void shift_up(T (&ar)[P], T (&ai)[P], T ur, T ui) {
#pragma unroll
  for (int k = P - 2; k >= 0; --k)
#pragma unroll
    for (int j = k; j <= P - 2; ++j) {
      ar[j + 1] += ur * ar[j] - ui * ai[j];
      ai[j + 1] += ur * ai[j] + ui * ar[j];
    }
}

// ------------------------------------------------------------------ M2M --
// M~_k(parent) = 2^-k sum_children sum_{j<=k} C(k,j) u^(k-j) M~_j(child):
// one thread per parent box.

template <int P>
__global__ __launch_bounds__(256) void m2m_kernel(float2 *__restrict__ M, int lpar) {
  const int64_t npar = int64_t(1) << (2 * lpar);
  const int64_t par = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (par >= npar) return;
  uint32_t px, py;
  unmorton2(uint32_t(par), px, py);
  float sr[P], si[P];
#pragma unroll
  for (int k = 0; k < P; ++k) sr[k] = si[k] = 0.f;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const uint32_t ch = morton2(2 * px + (c & 1), 2 * py + (c >> 1));
    const float4 *Mc = reinterpret_cast<const float4 *>(M + (level_off(lpar + 1) + ch) * P);
    float ar[P], ai[P];
#pragma unroll
    for (int j = 0; j < P / 2; ++j) {
      const float4 v = Mc[j];
      ar[2 * j] = v.x, ai[2 * j] = v.y, ar[2 * j + 1] = v.z, ai[2 * j + 1] = v.w;
    }
    shift_up<P>(ar, ai, (c & 1) ? 0.5f : -0.5f, (c >> 1) ? 0.5f : -0.5f);
#pragma unroll
    for (int k = 0; k < P; ++k) sr[k] += ar[k], si[k] += ai[k];
  }
  float4 *out = reinterpret_cast<float4 *>(M + (level_off(lpar) + par) * P);
  float sc = 1.f;  // 2^-k
#pragma unroll
  for (int j = 0; j < P / 2; ++j) {
    const float s0 = sc, s1 = 0.5f * sc;
    out[j] = make_float4(s0 * sr[2 * j], s0 * si[2 * j], s1 * sr[2 * j + 1], s1 * si[2 * j + 1]);
    sc *= 0.25f;
  }
}

// gM~_j(child) += sum_{k>=j} C(k,j) u^(k-j) 2^-k gM~_k(parent): one thread per child box.
template <int P>
__global__ __launch_bounds__(256) void m2m_backward_kernel(float2 *__restrict__ gM, int lchild) {
  const int64_t nch = int64_t(1) << (2 * lchild);
  const int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (c >= nch) return;
  uint32_t ix, iy;
  unmorton2(uint32_t(c), ix, iy);
  const uint32_t par = morton2(ix >> 1, iy >> 1);
  const float4 *gp = reinterpret_cast<const float4 *>(gM + (level_off(lchild - 1) + par) * P);
  float ar[P], ai[P];
  float sc = 1.f;  // 2^-k
#pragma unroll
  for (int j = 0; j < P / 2; ++j) {
    const float4 v = gp[j];
    ar[2 * j] = sc * v.x, ai[2 * j] = sc * v.y;
    ar[2 * j + 1] = 0.5f * sc * v.z, ai[2 * j + 1] = 0.5f * sc * v.w;
    sc *= 0.25f;
  }
  shift_down<P>(ar, ai, (ix & 1) ? 0.5f : -0.5f, (iy & 1) ? 0.5f : -0.5f);
  float4 *dst = reinterpret_cast<float4 *>(gM + (level_off(lchild) + c) * P);
#pragma unroll
  for (int j = 0; j < P / 2; ++j) {
    const float4 o = dst[j];
    dst[j] = make_float4(o.x + ar[2 * j], o.y + ai[2 * j], o.z + ar[2 * j + 1], o.w + ai[2 * j + 1]);
  }
}

// ------------------------------------------------------------------ L2L --
// L~_n(child) = Lm2l_n(child) + sum_{m>=n} C(m,n) u^(m-n) 2^-(m+1) L~_m(parent)
// b(child)    = bm2l(child) + b(parent) + sum_m 2^-(m+1) L~_m(parent) u^(m+1)/(m+1)

__global__ void zero_f64_kernel(double *__restrict__ a, int64_t n) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

// One thread per child box at level l.
template <int P>
__global__ __launch_bounds__(256) void l2l_kernel(const float2 *__restrict__ Lm2l, const float2 *__restrict__ bm2l,
                                                  double2 *__restrict__ L, double2 *__restrict__ b, int l) {
  const int64_t nb = int64_t(1) << (2 * l);
  const int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (c >= nb) return;
  const bool has_parent = l >= 3;  // levels 0-1 carry no local expansion
  uint32_t ix, iy;
  unmorton2(uint32_t(c), ix, iy);
  const int64_t gc = level_off(l) + c;
  const double ur = (ix & 1) ? 0.5 : -0.5, ui = (iy & 1) ? 0.5 : -0.5;
  double ar[P], ai[P];
  double br = 0.0, bi = 0.0;
  if (has_parent) {
    const int64_t gp = level_off(l - 1) + morton2(ix >> 1, iy >> 1);
    const double2 *Lp = L + gp * P;
    double sc = 0.5;  // 2^-(m+1)
#pragma unroll
    for (int m = 0; m < P; ++m) {
      const double2 v = Lp[m];
      ar[m] = sc * v.x, ai[m] = sc * v.y;
      sc *= 0.5;
    }
    if (b) {
      // b(parent) + sum_m a_m u^(m+1)/(m+1), Horner in u
#pragma unroll
      for (int m = P - 1; m >= 0; --m) {
        constexpr double one = 1.0;
        const double inv = one / double(m + 1);
        const double tr = br + inv * ar[m], ti = bi + inv * ai[m];
        br = tr * ur - ti * ui;
        bi = tr * ui + ti * ur;
      }
      const double2 bp = b[gp];
      br += bp.x;
      bi += bp.y;
    }
    shift_down<P>(ar, ai, ur, ui);
  } else {
#pragma unroll
    for (int m = 0; m < P; ++m) ar[m] = ai[m] = 0.0;
  }
  const float4 *own = reinterpret_cast<const float4 *>(Lm2l + gc * P);
  double2 *out = L + gc * P;
#pragma unroll
  for (int j = 0; j < P / 2; ++j) {
    const float4 o = own[j];
    out[2 * j] = make_double2(ar[2 * j] + o.x, ai[2 * j] + o.y);
    out[2 * j + 1] = make_double2(ar[2 * j + 1] + o.z, ai[2 * j + 1] + o.w);
  }
  if (b) {
    const float2 bo = bm2l[gc];
    b[gc] = make_double2(br + bo.x, bi + bo.y);
  }
}

// L2L^T, one thread per parent box at level lp:
//   gL~_m(parent) = 2^-(m+1) sum_children [sum_{n<=m} C(m,n) u^(m-n) gL~_n(child) + gb(child) u^(m+1)/(m+1)]
//   gb(parent)    = sum_children gb(child)
template <int P>
__global__ __launch_bounds__(256) void l2l_backward_kernel(double2 *__restrict__ gL, double2 *__restrict__ gb, int lp) {
  const int64_t npar = int64_t(1) << (2 * lp);
  const int64_t par = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (par >= npar) return;
  uint32_t px, py;
  unmorton2(uint32_t(par), px, py);
  double sr[P], si[P];
#pragma unroll
  for (int m = 0; m < P; ++m) sr[m] = si[m] = 0.0;
  double gbr = 0.0, gbi = 0.0;
#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    const int64_t ch = level_off(lp + 1) + morton2(2 * px + (c & 1), 2 * py + (c >> 1));
    const double ur = (c & 1) ? 0.5 : -0.5, ui = (c >> 1) ? 0.5 : -0.5;
    const double2 *gc = gL + ch * P;
    double ar[P], ai[P];
#pragma unroll
    for (int n = 0; n < P; ++n) {
      const double2 v = gc[n];
      ar[n] = v.x, ai[n] = v.y;
    }
    shift_up<P>(ar, ai, ur, ui);
#pragma unroll
    for (int m = 0; m < P; ++m) sr[m] += ar[m], si[m] += ai[m];
    if (gb) {
      const double2 g = gb[ch];
      double wr = ur * g.x - ui * g.y, wi = ur * g.y + ui * g.x;  // gb u^(m+1)
#pragma unroll
      for (int m = 0; m < P; ++m) {
        constexpr double one = 1.0;
        const double inv = one / double(m + 1);
        sr[m] += inv * wr, si[m] += inv * wi;
        const double tr = wr * ur - wi * ui;
        wi = wr * ui + wi * ur;
        wr = tr;
      }
      gbr += g.x, gbi += g.y;
    }
  }
  double2 *out = gL + (level_off(lp) + par) * P;
  double sc = 0.5;  // 2^-(m+1)
#pragma unroll
  for (int m = 0; m < P; ++m) {
    out[m] = make_double2(sc * sr[m], sc * si[m]);
    sc *= 0.5;
  }
  if (gb) gb[level_off(lp) + par] = make_double2(gbr, gbi);
}

__global__ void f64_to_f32_kernel(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) b[i] = float(a[i]);
}

// ------------------------------------------------------------------ L2P --

template <int P>
__global__ void l2p_kernel(const float2 *__restrict__ txy, const int32_t *__restrict__ tls, int64_t nt, int depth,
                           const double2 *__restrict__ L, const double2 *__restrict__ b, float2 *__restrict__ phi,
                           float2 *__restrict__ field) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int64_t nleaf = int64_t(1) << (2 * depth);
  if (t >= nt || t >= int64_t(tls[nleaf])) return;
  const float2 z = txy[t];
  const int64_t m = leaf_of_point(z, tls, nleaf, depth, t);
  uint32_t ix, iy;
  unmorton2(uint32_t(m), ix, iy);
  const double h = ldexp(1.0, -depth), ih = ldexp(1.0, depth);  // exact
  const double wr = (double(z.x) - (double(ix) + 0.5) * h) * ih;
  const double wi = (double(z.y) - (double(iy) + 0.5) * h) * ih;
  const double2 *Ll = L + (level_off(depth) + m) * P;
  double fr = 0.0, fi = 0.0, pr = 0.0, pi = 0.0;
  double cr = 1.0, ci = 0.0;  // w^n
#pragma unroll
  for (int n = 0; n < P; ++n) {
    const double2 ln = Ll[n];
    const double ar = ln.x * cr - ln.y * ci, ai = ln.x * ci + ln.y * cr;  // L_n w^n
    fr += ar;
    fi += ai;
    const double inv = 1.0 / double(n + 1);
    pr += inv * (ar * wr - ai * wi);  // L_n w^(n+1)/(n+1)
    pi += inv * (ar * wi + ai * wr);
    const double tr = cr * wr - ci * wi;
    ci = cr * wi + ci * wr;
    cr = tr;
  }
  if (b) {
    const double2 bb = b[level_off(depth) + m];
    pr += bb.x;
    pi += bb.y;
  }
  if (field) {
    const float2 o = field[t];
    field[t] = make_float2(o.x + float(fr * ih), o.y + float(fi * ih));
  }
  if (phi) {
    const float2 o = phi[t];
    phi[t] = make_float2(o.x + float(pr), o.y + float(pi));
  }
}

// L2P^T on one leaf per thread: gL_n = sum_t [cphi w^(n+1)/(n+1) + cfield w^n / h], gb = sum_t cphi.
template <int P>
__global__ void l2p_backward_kernel(const float2 *__restrict__ txy, const int32_t *__restrict__ tls, int depth,
                                    const float2 *__restrict__ cphi, const float2 *__restrict__ cfield,
                                    double2 *__restrict__ gL, double2 *__restrict__ gb) {
  const int64_t nleaf = int64_t(1) << (2 * depth);
  const int64_t m = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (m >= nleaf) return;
  uint32_t ix, iy;
  unmorton2(uint32_t(m), ix, iy);
  const double h = ldexp(1.0, -depth), ih = ldexp(1.0, depth);  // exact
  const double cx = (double(ix) + 0.5) * h, cy = (double(iy) + 0.5) * h;
  double ar[P], ai[P];
#pragma unroll
  for (int n = 0; n < P; ++n) ar[n] = ai[n] = 0.0;
  double sbr = 0.0, sbi = 0.0;
  for (int32_t t = tls[m]; t < tls[m + 1]; ++t) {
    const float2 z = txy[t];
    const double wr = (double(z.x) - cx) * ih, wi = (double(z.y) - cy) * ih;
    const float2 cp = cphi ? cphi[t] : make_float2(0.f, 0.f);
    const float2 cf = cfield ? cfield[t] : make_float2(0.f, 0.f);
    const double fr = double(cf.x) * ih, fi = double(cf.y) * ih;  // cfield / h
    sbr += cp.x;
    sbi += cp.y;
    double cr = 1.0, ci = 0.0;  // w^n
#pragma unroll
    for (int n = 0; n < P; ++n) {
      ar[n] += fr * cr - fi * ci;
      ai[n] += fr * ci + fi * cr;
      const double tr = cr * wr - ci * wi;
      ci = cr * wi + ci * wr;
      cr = tr;
      constexpr double one = 1.0;
      const double inv = one / double(n + 1);
      ar[n] += inv * (cp.x * cr - cp.y * ci);
      ai[n] += inv * (cp.x * ci + cp.y * cr);
    }
  }
  double2 *o = gL + (level_off(depth) + m) * P;
#pragma unroll
  for (int n = 0; n < P; ++n) o[n] = make_double2(ar[n], ai[n]);
  if (gb) gb[level_off(depth) + m] = make_double2(sbr, sbi);
}

// ------------------------------------------------------------- launchers --

static inline unsigned blocks_for(int64_t n, int bs = 256) { return unsigned((n + bs - 1) / bs); }

int launch_p2m(const float *xy, const float *q, const int32_t *ls, int depth, int p, float *M, hipStream_t s) {
  const int64_t nleaf = int64_t(1) << (2 * depth);
  const float2 *x = reinterpret_cast<const float2 *>(xy);
  float2 *Mo = reinterpret_cast<float2 *>(M);
  dim3 g(blocks_for(nleaf)), bl(256);
  switch (p) {
    case 8: hipLaunchKernelGGL(p2m_kernel<8>, g, bl, 0, s, x, q, ls, depth, Mo); break;
    case 12: hipLaunchKernelGGL(p2m_kernel<12>, g, bl, 0, s, x, q, ls, depth, Mo); break;
    case 16: hipLaunchKernelGGL(p2m_kernel<16>, g, bl, 0, s, x, q, ls, depth, Mo); break;
    case 20: hipLaunchKernelGGL(p2m_kernel<20>, g, bl, 0, s, x, q, ls, depth, Mo); break;
  }
  return check_launch("p2m");
}

int launch_p2m_backward(const float *xy, const float *q, const int32_t *ls, int64_t n, int depth, int p,
                        const float *gM, float *gq, float *G, hipStream_t s) {
  if (n == 0) return FMM2D_OK;
  const float2 *x = reinterpret_cast<const float2 *>(xy);
  const float2 *g = reinterpret_cast<const float2 *>(gM);
  float2 *Go = reinterpret_cast<float2 *>(G);
  dim3 gr(blocks_for(n)), bl(256);
  switch (p) {
    case 8: hipLaunchKernelGGL(p2m_backward_kernel<8>, gr, bl, 0, s, x, q, ls, n, depth, g, gq, Go); break;
    case 12: hipLaunchKernelGGL(p2m_backward_kernel<12>, gr, bl, 0, s, x, q, ls, n, depth, g, gq, Go); break;
    case 16: hipLaunchKernelGGL(p2m_backward_kernel<16>, gr, bl, 0, s, x, q, ls, n, depth, g, gq, Go); break;
    case 20: hipLaunchKernelGGL(p2m_backward_kernel<20>, gr, bl, 0, s, x, q, ls, n, depth, g, gq, Go); break;
  }
  return check_launch("p2m_backward");
}

int launch_m2m(float *M, int depth, int p, hipStream_t s) {
  float2 *Mo = reinterpret_cast<float2 *>(M);
  for (int lp = depth - 1; lp >= 0; --lp) {
    const dim3 g(blocks_for(int64_t(1) << (2 * lp))), bl(256);
    switch (p) {
      case 8: hipLaunchKernelGGL(m2m_kernel<8>, g, bl, 0, s, Mo, lp); break;
      case 12: hipLaunchKernelGGL(m2m_kernel<12>, g, bl, 0, s, Mo, lp); break;
      case 16: hipLaunchKernelGGL(m2m_kernel<16>, g, bl, 0, s, Mo, lp); break;
      case 20: hipLaunchKernelGGL(m2m_kernel<20>, g, bl, 0, s, Mo, lp); break;
    }
  }
  return check_launch("m2m");
}

int launch_m2m_backward(float *gM, int depth, int p, hipStream_t s) {
  float2 *g = reinterpret_cast<float2 *>(gM);
  for (int lc = 3; lc <= depth; ++lc) {
    const dim3 gr(blocks_for(int64_t(1) << (2 * lc))), bl(256);
    switch (p) {
      case 8: hipLaunchKernelGGL(m2m_backward_kernel<8>, gr, bl, 0, s, g, lc); break;
      case 12: hipLaunchKernelGGL(m2m_backward_kernel<12>, gr, bl, 0, s, g, lc); break;
      case 16: hipLaunchKernelGGL(m2m_backward_kernel<16>, gr, bl, 0, s, g, lc); break;
      case 20: hipLaunchKernelGGL(m2m_backward_kernel<20>, gr, bl, 0, s, g, lc); break;
    }
  }
  return check_launch("m2m_backward");
}

int launch_l2l(const float *Lm2l, const float *bm2l, double *L, double *b, int depth, int p, hipStream_t s) {
  const float2 *Lm = reinterpret_cast<const float2 *>(Lm2l);
  const float2 *bm = reinterpret_cast<const float2 *>(bm2l);
  double2 *Lo = reinterpret_cast<double2 *>(L);
  double2 *bo = reinterpret_cast<double2 *>(b);
  // levels 0 and 1 have empty interaction lists: their local expansions are zero
  const int64_t low = level_off(2);
  hipLaunchKernelGGL(zero_f64_kernel, dim3(blocks_for(low * p * 2)), dim3(256), 0, s, L, low * p * 2);
  if (b) hipLaunchKernelGGL(zero_f64_kernel, dim3(blocks_for(low * 2)), dim3(256), 0, s, b, low * 2);
  for (int l = 2; l <= depth; ++l) {
    const dim3 g(blocks_for(int64_t(1) << (2 * l))), bl(256);
    switch (p) {
      case 8: hipLaunchKernelGGL(l2l_kernel<8>, g, bl, 0, s, Lm, bm, Lo, bo, l); break;
      case 12: hipLaunchKernelGGL(l2l_kernel<12>, g, bl, 0, s, Lm, bm, Lo, bo, l); break;
      case 16: hipLaunchKernelGGL(l2l_kernel<16>, g, bl, 0, s, Lm, bm, Lo, bo, l); break;
      case 20: hipLaunchKernelGGL(l2l_kernel<20>, g, bl, 0, s, Lm, bm, Lo, bo, l); break;
    }
  }
  return check_launch("l2l");
}

int launch_l2l_backward(double *gL, double *gb, float *gLm2l, float *gbm2l, int depth, int p, hipStream_t s) {
  double2 *g = reinterpret_cast<double2 *>(gL);
  double2 *gbb = reinterpret_cast<double2 *>(gb);
  for (int lp = depth - 1; lp >= 2; --lp) {
    const dim3 gr(blocks_for(int64_t(1) << (2 * lp))), bl(256);
    switch (p) {
      case 8: hipLaunchKernelGGL(l2l_backward_kernel<8>, gr, bl, 0, s, g, gbb, lp); break;
      case 12: hipLaunchKernelGGL(l2l_backward_kernel<12>, gr, bl, 0, s, g, gbb, lp); break;
      case 16: hipLaunchKernelGGL(l2l_backward_kernel<16>, gr, bl, 0, s, g, gbb, lp); break;
      case 20: hipLaunchKernelGGL(l2l_backward_kernel<20>, gr, bl, 0, s, g, gbb, lp); break;
    }
  }
  const int64_t o = level_off(2), e = level_off(depth + 1);
  const int64_t nl = (e - o) * p * 2;
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(blocks_for(nl)), dim3(256), 0, s, gL + o * p * 2, gLm2l + o * p * 2,
                     nl);
  if (gb)
    hipLaunchKernelGGL(f64_to_f32_kernel, dim3(blocks_for((e - o) * 2)), dim3(256), 0, s, gb + o * 2, gbm2l + o * 2,
                       (e - o) * 2);
  return check_launch("l2l_backward");
}

int launch_l2p(const float *txy, const int32_t *tls, int64_t nt, const double *L, const double *b, int depth, int p,
               float *phi, float *field, hipStream_t s) {
  if (nt == 0) return FMM2D_OK;
  const float2 *t = reinterpret_cast<const float2 *>(txy);
  const double2 *Li = reinterpret_cast<const double2 *>(L);
  const double2 *bi = reinterpret_cast<const double2 *>(b);
  float2 *ph = reinterpret_cast<float2 *>(phi);
  float2 *fi = reinterpret_cast<float2 *>(field);
  dim3 g(blocks_for(nt)), bl(256);
  switch (p) {
    case 8: hipLaunchKernelGGL(l2p_kernel<8>, g, bl, 0, s, t, tls, nt, depth, Li, bi, ph, fi); break;
    case 12: hipLaunchKernelGGL(l2p_kernel<12>, g, bl, 0, s, t, tls, nt, depth, Li, bi, ph, fi); break;
    case 16: hipLaunchKernelGGL(l2p_kernel<16>, g, bl, 0, s, t, tls, nt, depth, Li, bi, ph, fi); break;
    case 20: hipLaunchKernelGGL(l2p_kernel<20>, g, bl, 0, s, t, tls, nt, depth, Li, bi, ph, fi); break;
  }
  return check_launch("l2p");
}

int launch_l2p_backward(const float *txy, const int32_t *tls, const float *cphi, const float *cfield, int depth,
                        int p, double *gL, double *gb, hipStream_t s) {
  const int64_t nleaf = int64_t(1) << (2 * depth);
  const float2 *t = reinterpret_cast<const float2 *>(txy);
  const float2 *cp = reinterpret_cast<const float2 *>(cphi);
  const float2 *cf = reinterpret_cast<const float2 *>(cfield);
  double2 *g = reinterpret_cast<double2 *>(gL);
  double2 *gbo = reinterpret_cast<double2 *>(gb);
  dim3 gr(blocks_for(nleaf)), bl(256);
  switch (p) {
    case 8: hipLaunchKernelGGL(l2p_backward_kernel<8>, gr, bl, 0, s, t, tls, depth, cp, cf, g, gbo); break;
    case 12: hipLaunchKernelGGL(l2p_backward_kernel<12>, gr, bl, 0, s, t, tls, depth, cp, cf, g, gbo); break;
    case 16: hipLaunchKernelGGL(l2p_backward_kernel<16>, gr, bl, 0, s, t, tls, depth, cp, cf, g, gbo); break;
    case 20: hipLaunchKernelGGL(l2p_backward_kernel<20>, gr, bl, 0, s, t, tls, depth, cp, cf, g, gbo); break;
  }
  return check_launch("l2p_backward");
}

}  // namespace fmm2d
