// extern "C" entry points of libfmm2d.so (include/fmm2d.h): argument
// validation on the host, before any HIP call, then the launchers.
#include <cstdarg>
#include <string>

#include "fmm2d_internal.h"

namespace fmm2d {

static thread_local std::string g_last_error;

int set_error(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

void clear_error() { g_last_error.clear(); }

int check_launch(const char *what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(FMM2D_EHIP, "%s: %s", what, hipGetErrorString(e));
  return FMM2D_OK;
}

static int check_depth(const char *fn, int depth) {
  if (depth < 2 || depth > kMaxDepth) return set_error(FMM2D_EDEPTH, "%s: depth %d outside 2..%d", fn, depth, kMaxDepth);
  return FMM2D_OK;
}

static int check_p(const char *fn, int p) {
  if (!p_supported(p)) return set_error(FMM2D_EUNSUPPORTED_P, "%s: p = %d not in {8, 12, 16, 20}", fn, p);
  return FMM2D_OK;
}

#define FMM2D_NONNULL(fn, ptr)                                                     \
  do {                                                                             \
    if ((ptr) == nullptr) return set_error(FMM2D_EINVAL, "%s: %s is NULL", fn, #ptr); \
  } while (0)

#define FMM2D_TRY(expr)            \
  do {                             \
    const int rc_ = (expr);        \
    if (rc_ != FMM2D_OK) return rc_; \
  } while (0)

static int check_levels(const char *fn, int depth, int lmin, int lmax) {
  if (lmin < 2 || lmax > depth || lmin > lmax)
    return set_error(FMM2D_ELEVEL, "%s: levels %d..%d not within 2..%d", fn, lmin, lmax, depth);
  return FMM2D_OK;
}

static int check_precision(const char *fn, int p, int precision, const void *ops, size_t ops_bytes) {
  if (precision != FMM2D_F32 && precision != FMM2D_BF16X3 && precision != FMM2D_F16X3 &&
      precision != FMM2D_F32_PASCAL && precision != FMM2D_F64_HANKEL)
    return set_error(FMM2D_EINVAL, "%s: unknown precision %d", fn, precision);
  const size_t need = m2l_ops_bytes(p, precision);
  if (need == 0)
    return set_error(FMM2D_EUNSUPPORTED_P, "%s: precision %d is not built for p = %d", fn, precision, p);
  if (ops == nullptr) return set_error(FMM2D_EINVAL, "%s: ops is NULL", fn);
  if (ops_bytes < need)
    return set_error(FMM2D_EWORKSPACE, "%s: operator bank holds %zu bytes, %zu needed", fn, ops_bytes, need);
  return FMM2D_OK;
}

}  // namespace fmm2d

using namespace fmm2d;

extern "C" {

int fmm2d_abi_version(void) { return FMM2D_ABI_VERSION; }

const char *fmm2d_last_error(void) { return g_last_error.c_str(); }

int64_t fmm2d_num_boxes(int depth) {
  if (depth < 0 || depth > kMaxDepth) return -1;
  return level_off(depth + 1);
}

int64_t fmm2d_level_offset(int level) {
  if (level < 0 || level > kMaxDepth + 1) return -1;
  return level_off(level);
}

int64_t fmm2d_translation_count(int lmin, int lmax) {
  if (lmin < 2 || lmax > kMaxDepth || lmin > lmax) return -1;
  int64_t tot = 0;
  for (int l = lmin; l <= lmax; ++l) {
    // ordered pairs of boxes whose parents touch (or coincide), minus pairs that touch
    const int64_t a = 3 * (int64_t(1) << l) - 4, b = 3 * (int64_t(1) << l) - 2;
    tot += 4 * a * a - b * b;
  }
  return tot;
}

size_t fmm2d_build_tree_workspace(int64_t n, int depth) {
  if (n < 0 || n >= (int64_t(1) << 31) || depth < 2 || depth > kMaxDepth) return 0;
  return build_tree_ws_bytes(n, depth);
}

int fmm2d_build_tree(const float *xy, int64_t n, int depth, int32_t *perm, int32_t *leaf_start,
                     uint32_t *domain_flag, void *ws, size_t ws_bytes, hipStream_t stream) {
  const char *fn = "fmm2d_build_tree";
  clear_error();
  FMM2D_TRY(check_depth(fn, depth));
  if (n < 0 || n >= (int64_t(1) << 31)) return set_error(FMM2D_EINVAL, "%s: n = %lld outside [0, 2^31)", fn, (long long)n);
  if (n > 0) {
    FMM2D_NONNULL(fn, xy);
    FMM2D_NONNULL(fn, perm);
  }
  FMM2D_NONNULL(fn, leaf_start);
  FMM2D_NONNULL(fn, domain_flag);
  FMM2D_NONNULL(fn, ws);
  const size_t need = build_tree_ws_bytes(n, depth);
  if (ws_bytes < need) return set_error(FMM2D_EWORKSPACE, "%s: workspace %zu bytes, %zu needed", fn, ws_bytes, need);
  return launch_build_tree(xy, n, depth, perm, leaf_start, domain_flag, ws, stream);
}

int fmm2d_build_tree_noalloc(const float *xy, int64_t n, int depth, int32_t *perm, int32_t *leaf_start,
                             uint32_t *domain_flag, hipStream_t stream) {
  const char *fn = "fmm2d_build_tree_noalloc";
  clear_error();
  FMM2D_TRY(check_depth(fn, depth));
  if (n < 0 || n > kNoAllocMaxPoints)
    return set_error(n < 0 ? FMM2D_EINVAL : FMM2D_EWORKSPACE, "%s: n = %lld outside [0, %lld]", fn, (long long)n,
                     (long long)kNoAllocMaxPoints);
  if (n > 0) {
    FMM2D_NONNULL(fn, xy);
    FMM2D_NONNULL(fn, perm);
  }
  FMM2D_NONNULL(fn, leaf_start);
  FMM2D_NONNULL(fn, domain_flag);
  return launch_build_tree_noalloc(xy, n, depth, perm, leaf_start, domain_flag, stream);
}

static int gather_common(const char *fn, const float *src, const int32_t *perm, int64_t n, int width, float *dst,
                         bool scatter, hipStream_t stream) {
  clear_error();
  if (n < 0 || n >= (int64_t(1) << 31)) return set_error(FMM2D_EINVAL, "%s: n out of range", fn);
  if (width < 1 || width > 64) return set_error(FMM2D_EINVAL, "%s: width %d outside 1..64", fn, width);
  if (n == 0) return FMM2D_OK;
  FMM2D_NONNULL(fn, src);
  FMM2D_NONNULL(fn, perm);
  FMM2D_NONNULL(fn, dst);
  if (src == dst) return set_error(FMM2D_EINVAL, "%s: src and dst must not overlap", fn);
  return launch_gather(src, perm, n, width, dst, scatter, stream);
}

int fmm2d_gather(const float *src, const int32_t *perm, int64_t n, int width, float *dst, hipStream_t stream) {
  return gather_common("fmm2d_gather", src, perm, n, width, dst, false, stream);
}

int fmm2d_scatter(const float *src, const int32_t *perm, int64_t n, int width, float *dst, hipStream_t stream) {
  return gather_common("fmm2d_scatter", src, perm, n, width, dst, true, stream);
}

int fmm2d_p2m(const float *xy_sorted, const float *q_sorted, const int32_t *leaf_start, int depth, int p, float *M,
              hipStream_t stream) {
  const char *fn = "fmm2d_p2m";
  clear_error();
  FMM2D_TRY(check_depth(fn, depth));
  FMM2D_TRY(check_p(fn, p));
  FMM2D_NONNULL(fn, xy_sorted);
  FMM2D_NONNULL(fn, q_sorted);
  FMM2D_NONNULL(fn, leaf_start);
  FMM2D_NONNULL(fn, M);
  return launch_p2m(xy_sorted, q_sorted, leaf_start, depth, p, M, stream);
}

int fmm2d_m2m(float *M, int depth, int p, hipStream_t stream) {
  const char *fn = "fmm2d_m2m";
  clear_error();
  FMM2D_TRY(check_depth(fn, depth));
  FMM2D_TRY(check_p(fn, p));
  FMM2D_NONNULL(fn, M);
  return launch_m2m(M, depth, p, stream);
}

size_t fmm2d_m2l_operators_bytes(int p, int precision) { return m2l_ops_bytes(p, precision); }

int fmm2d_m2l_operators(int p, int precision, void *ops, size_t ops_bytes, hipStream_t stream) {
  const char *fn = "fmm2d_m2l_operators";
  clear_error();
  FMM2D_TRY(check_p(fn, p));
  FMM2D_TRY(check_precision(fn, p, precision, ops, ops_bytes));
  return launch_m2l_ops(p, precision, ops, stream);
}

static int m2l_common(const char *fn, const float *in, const float *gb_in, float *out, float *b, int depth, int p,
                      int lmin, int lmax, int precision, const void *ops, size_t ops_bytes, bool adjoint,
                      hipStream_t stream) {
  clear_error();
  FMM2D_TRY(check_depth(fn, depth));
  FMM2D_TRY(check_p(fn, p));
  FMM2D_TRY(check_levels(fn, depth, lmin, lmax));
  FMM2D_TRY(check_precision(fn, p, precision, ops, ops_bytes));
  FMM2D_NONNULL(fn, in);
  FMM2D_NONNULL(fn, out);
  if (in == out) return set_error(FMM2D_EINVAL, "%s: input and output must not overlap", fn);
  if (precision == FMM2D_F32) return launch_m2l_f32(in, gb_in, out, b, depth, p, lmin, lmax, adjoint, ops, stream);
  if (precision == FMM2D_F32_PASCAL)
    return launch_m2l_pascal(in, gb_in, out, b, depth, p, lmin, lmax, adjoint, ops, stream);
  if (precision == FMM2D_F64_HANKEL)
    return launch_m2l_hankel(in, gb_in, out, b, depth, p, lmin, lmax, adjoint, ops, stream);
  return launch_m2l_mixed(in, gb_in, out, b, depth, p, lmin, lmax, adjoint, precision, ops, stream);
}

int fmm2d_m2l(const float *M, float *L, float *b, int depth, int p, int lmin, int lmax, int precision,
              const void *ops, size_t ops_bytes, hipStream_t stream) {
  return m2l_common("fmm2d_m2l", M, nullptr, L, b, depth, p, lmin, lmax, precision, ops, ops_bytes, false, stream);
}

int fmm2d_m2l_backward(const float *gL, const float *gb, float *gM, int depth, int p, int lmin, int lmax,
                       int precision, const void *ops, size_t ops_bytes, hipStream_t stream) {
  return m2l_common("fmm2d_m2l_backward", gL, gb, gM, nullptr, depth, p, lmin, lmax, precision, ops, ops_bytes, true,
                    stream);
}

int fmm2d_l2l(const float *Lm2l, const float *bm2l, double *L, double *b, int depth, int p, hipStream_t stream) {
  const char *fn = "fmm2d_l2l";
  clear_error();
  FMM2D_TRY(check_depth(fn, depth));
  FMM2D_TRY(check_p(fn, p));
  FMM2D_NONNULL(fn, Lm2l);
  FMM2D_NONNULL(fn, L);
  if ((bm2l == nullptr) != (b == nullptr)) return set_error(FMM2D_EINVAL, "%s: bm2l and b must both be NULL or not", fn);
  return launch_l2l(Lm2l, bm2l, L, b, depth, p, stream);
}

int fmm2d_l2p(const float *txy_sorted, const int32_t *tleaf_start, int64_t nt, const double *L, const double *b,
              int depth, int p, float *phi, float *field, hipStream_t stream) {
  const char *fn = "fmm2d_l2p";
  clear_error();
  FMM2D_TRY(check_depth(fn, depth));
  FMM2D_TRY(check_p(fn, p));
  if (nt < 0 || nt >= (int64_t(1) << 31)) return set_error(FMM2D_EINVAL, "%s: nt out of range", fn);
  FMM2D_NONNULL(fn, tleaf_start);
  FMM2D_NONNULL(fn, L);
  if (nt > 0) FMM2D_NONNULL(fn, txy_sorted);
  return launch_l2p(txy_sorted, tleaf_start, nt, L, b, depth, p, phi, field, stream);
}

int fmm2d_p2p(const float *xy_sorted, const float *q_sorted, const int32_t *leaf_start, const float *txy_sorted,
              const int32_t *tleaf_start, int64_t nt, int depth, float *phi, float *field, hipStream_t stream) {
  const char *fn = "fmm2d_p2p";
  clear_error();
  FMM2D_TRY(check_depth(fn, depth));
  if (nt < 0 || nt >= (int64_t(1) << 31)) return set_error(FMM2D_EINVAL, "%s: nt out of range", fn);
  FMM2D_NONNULL(fn, xy_sorted);
  FMM2D_NONNULL(fn, q_sorted);
  FMM2D_NONNULL(fn, leaf_start);
  FMM2D_NONNULL(fn, tleaf_start);
  if (nt > 0) FMM2D_NONNULL(fn, txy_sorted);
  return launch_p2p(xy_sorted, q_sorted, leaf_start, txy_sorted, tleaf_start, nt, depth, phi, field, stream);
}

int fmm2d_l2p_backward(const float *txy_sorted, const int32_t *tleaf_start, const float *cphi, const float *cfield,
                       int depth, int p, double *gL, double *gb, hipStream_t stream) {
  const char *fn = "fmm2d_l2p_backward";
  clear_error();
  FMM2D_TRY(check_depth(fn, depth));
  FMM2D_TRY(check_p(fn, p));
  FMM2D_NONNULL(fn, txy_sorted);
  FMM2D_NONNULL(fn, tleaf_start);
  FMM2D_NONNULL(fn, gL);
  return launch_l2p_backward(txy_sorted, tleaf_start, cphi, cfield, depth, p, gL, gb, stream);
}

int fmm2d_l2l_backward(double *gL, double *gb, float *gLm2l, float *gbm2l, int depth, int p, hipStream_t stream) {
  const char *fn = "fmm2d_l2l_backward";
  clear_error();
  FMM2D_TRY(check_depth(fn, depth));
  FMM2D_TRY(check_p(fn, p));
  FMM2D_NONNULL(fn, gL);
  FMM2D_NONNULL(fn, gLm2l);
  if ((gb == nullptr) != (gbm2l == nullptr)) return set_error(FMM2D_EINVAL, "%s: gb and gbm2l must both be NULL or not", fn);
  return launch_l2l_backward(gL, gb, gLm2l, gbm2l, depth, p, stream);
}

int fmm2d_m2m_backward(float *gM, int depth, int p, hipStream_t stream) {
  const char *fn = "fmm2d_m2m_backward";
  clear_error();
  FMM2D_TRY(check_depth(fn, depth));
  FMM2D_TRY(check_p(fn, p));
  FMM2D_NONNULL(fn, gM);
  return launch_m2m_backward(gM, depth, p, stream);
}

int fmm2d_p2m_backward(const float *xy_sorted, const float *q_sorted, const int32_t *leaf_start, int64_t n, int depth,
                       int p, const float *gM, float *gq, float *G, hipStream_t stream) {
  const char *fn = "fmm2d_p2m_backward";
  clear_error();
  FMM2D_TRY(check_depth(fn, depth));
  FMM2D_TRY(check_p(fn, p));
  if (n < 0 || n >= (int64_t(1) << 31)) return set_error(FMM2D_EINVAL, "%s: n out of range", fn);
  FMM2D_NONNULL(fn, leaf_start);
  FMM2D_NONNULL(fn, gM);
  if (n > 0) {
    FMM2D_NONNULL(fn, xy_sorted);
    FMM2D_NONNULL(fn, q_sorted);
    FMM2D_NONNULL(fn, gq);
    FMM2D_NONNULL(fn, G);
  }
  return launch_p2m_backward(xy_sorted, q_sorted, leaf_start, n, depth, p, gM, gq, G, stream);
}

int fmm2d_p2p_backward(const float *xy_sorted, const float *q_sorted, const int32_t *leaf_start, int64_t n,
                       const float *txy_sorted, const int32_t *tleaf_start, int depth, const float *cphi,
                       const float *cfield, float *gq, float *G, hipStream_t stream) {
  const char *fn = "fmm2d_p2p_backward";
  clear_error();
  FMM2D_TRY(check_depth(fn, depth));
  if (n < 0 || n >= (int64_t(1) << 31)) return set_error(FMM2D_EINVAL, "%s: n out of range", fn);
  FMM2D_NONNULL(fn, leaf_start);
  FMM2D_NONNULL(fn, tleaf_start);
  FMM2D_NONNULL(fn, txy_sorted);
  if (n > 0) {
    FMM2D_NONNULL(fn, xy_sorted);
    FMM2D_NONNULL(fn, q_sorted);
    FMM2D_NONNULL(fn, gq);
    FMM2D_NONNULL(fn, G);
  }
  return launch_p2p_backward(xy_sorted, q_sorted, leaf_start, n, txy_sorted, tleaf_start, depth, cphi, cfield, gq, G,
                             stream);
}

}  // extern "C"
