/*
 * fmm2d.h -- C ABI of libfmm2d.so: the 2D fast multipole method of
 * Cruz, Layton & Barba, "How to obtain efficient GPU kernels: an illustration
 * using FMM & FGT algorithms" (arXiv:1009.3457), on AMD MI355X (gfx950).
 *
 * The method (Sec. 2.1) evaluates Eq. (eq:n_body) for the logarithmic kernel in
 * complex form,
 *     phi(z) = sum_s q_s log(z - z_s),        f(z) = phi'(z) = sum_s q_s / (z - z_s),
 * (Re phi is the 2D potential; f is the Cauchy / Biot-Savart sum of the vortex
 * method, Sec. 1) through five stages: tree construction, upward sweep (P2M,
 * M2M), downward sweep (M2L over every box's interaction list plus reduction,
 * then L2L), far-field evaluation (L2P) and near-field evaluation (P2P).
 *
 * ---------------------------------------------------------------------------
 * Conventions shared by every entry point
 * ---------------------------------------------------------------------------
 * Tree.  Uniform quadtree over the unit square; level l has 2^l x 2^l boxes of
 *   width h_l = 2^-l.  A point (x, y) in [0,1]^2 lies in leaf
 *   (min(floor(x 2^depth), 2^depth - 1), min(floor(y 2^depth), 2^depth - 1)).
 *   Boxes of level l are numbered level_offset(l) + morton(ix, iy) with
 *   level_offset(l) = (4^l - 1)/3 and bit 2b (2b+1) of the Morton index equal
 *   to bit b of ix (iy).  num_boxes(depth) = (4^(depth+1) - 1)/3.
 * Expansions.  Complex arrays are interleaved (re, im) pairs.  An expansion
 *   array is [num_boxes][p] complex.  Multipole and local coefficients are
 *   stored in a SCALED basis that makes the M2L operators independent of the
 *   level: with c the box centre and h its width,
 *     multipole  M~_k = sum_s q_s ((z_s - c)/h)^k                   k < p
 *     local      f(z)   ~ (1/h) sum_n L~_n ((z - c)/h)^n            n < p
 *                phi(z) ~ b + sum_n L~_n ((z - c)/h)^(n+1)/(n+1)
 *   i.e. M~_k = M_k / h^k and L~_n = L_n h^(n+1) for the unscaled M_k, L_n of
 *   the paper.  b (one complex per box) is the constant term of the local
 *   expansion of phi; it is produced by the log-potential row of the M2L.
 * Points.  xy is [n][2] float (x, y).  Entry points named *_sorted take points
 *   in leaf order, i.e. src_sorted[i] = src[perm[i]] with perm from
 *   fmm2d_build_tree; leaf_start has 4^depth + 1 entries.
 * Memory.  Every pointer argument is DEVICE memory on the current HIP device
 *   unless stated otherwise; the caller allocates and owns it.  No entry point
 *   allocates device memory; fmm2d_build_tree sorts in the caller's workspace
 *   and fmm2d_build_tree_noalloc in a fixed array of the library.  Arrays must
 *   not overlap unless stated.
 * Streams.  Work is enqueued on `stream` (0 = the null stream) and every
 *   entry point returns without synchronising with the host.
 * Errors.  Every entry point returns FMM2D_OK (0) or a negative
 *   fmm2d_status.  Arguments are validated on the host before any HIP call, so
 *   an invalid call enqueues nothing.  fmm2d_last_error() returns a message for
 *   the last failing call on the calling thread.
 * Supported orders p: 8, 12, 16, 20.  Supported depth: 2..12.
 */
#ifndef FMM2D_H
#define FMM2D_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMM2D_ABI_VERSION 2

typedef enum fmm2d_status {
    FMM2D_OK = 0,
    FMM2D_EINVAL = -1,          /* null pointer, bad size or range */
    FMM2D_EUNSUPPORTED_P = -2,  /* p not in {8, 12, 16, 20} (or not built for this precision) */
    FMM2D_EDEPTH = -3,          /* depth outside 2..12 */
    FMM2D_EDOMAIN = -4,         /* a point outside [0,1]^2 or NaN */
    FMM2D_EWORKSPACE = -5,      /* workspace or operator buffer too small */
    FMM2D_EHIP = -6,            /* a HIP runtime call failed */
    FMM2D_ELEVEL = -7           /* lmin/lmax outside 2 <= lmin <= lmax <= depth */
} fmm2d_status;

/* Arithmetic of the M2L contraction.  The operators are always generated in
 * FP64 and rounded once; accumulation is FP32 except in FMM2D_F64_HANKEL. */
typedef enum fmm2d_precision {
    FMM2D_F32 = 0,     /* FP32 products (MFMA f32)                                   */
    FMM2D_BF16X3 = 1,  /* BF16 hi/lo split of both operands, 3 MFMA products (hi*hi,   */
                       /* hi*lo, lo*hi), FP32 accumulation                             */
    FMM2D_F16X3 = 2,   /* the same with FP16 and power-of-two pre-scaling              */
    FMM2D_F32_PASCAL = 3, /* FP32 products on the factorisation                        */
                          /*   A~(d) = diag((-1)^n d^-(n+1)) B diag(d^-k),              */
                          /*   B[n][k] = C(n+k, k): two real MFMA products with the     */
                          /*   constant B per translation, the diagonals on the VALU   */
    FMM2D_F64_HANKEL = 4  /* FP64 arithmetic on the Hankel form of Eq. (eq:M2Lmat)      */
                          /*   (entries depend on n + k between two diagonals): the    */
                          /*   list's translations summed as spectra of length 2p,     */
                          /*   27 complex multiply-adds per target and frequency;      */
                          /*   L~ accumulated in FP64 on the vector ALUs; the log row  */
                          /*   b (and its transpose) in FP32, in a pass of its own     */
} fmm2d_precision;

/* ----------------------------------------------------------- queries ---- */

int fmm2d_abi_version(void);

/* Message describing the last failing call on this thread ("" if none).
 * The pointer stays valid until the next call on this thread. */
const char *fmm2d_last_error(void);

/* (4^(depth+1) - 1)/3, or -1 if depth is outside 0..12. */
int64_t fmm2d_num_boxes(int depth);

/* (4^level - 1)/3, or -1 if level is outside 0..13. */
int64_t fmm2d_level_offset(int level);

/* Exact number of M2L translations (box pairs (t, s) with s in the interaction
 * list of t) over levels lmin..lmax, boundary truncation included (host only).
 * Returns -1 on a bad range. */
int64_t fmm2d_translation_count(int lmin, int lmax);

/* ------------------------------------------------------------- tree ----- */

/* Bytes of device workspace fmm2d_build_tree needs for n points. */
size_t fmm2d_build_tree_workspace(int64_t n, int depth);

/*
 * Initialization stage (Sec. 2.1, stage 1): assign each point to its leaf and
 * stably sort the points by leaf Morton index.
 *   xy          [n][2] float, points in [0,1]^2 (x = 1 or y = 1 is clamped
 *               into the last leaf)
 *   perm        [n] int32 out: perm[i] = original index of the i-th sorted point
 *   leaf_start  [4^depth + 1] int32 out: first sorted index of every leaf;
 *               leaf_start[4^depth] = n
 *   domain_flag [1] uint32 out (device memory, required): 0 when every point
 *               lies in [0,1]^2, nonzero when one lies outside or is NaN (then
 *               perm and leaf_start are unspecified).  It is written on the
 *               stream like the other outputs; the caller reads it when it
 *               chooses, so the call never waits for the device.
 *   ws, ws_bytes  caller workspace of at least fmm2d_build_tree_workspace(n, depth)
 * 0 <= n < 2^31.  Returns without synchronising; FMM2D_EDOMAIN is never
 * returned by this call (the domain check lives in domain_flag).
 */
int fmm2d_build_tree(const float *xy, int64_t n, int depth, int32_t *perm, int32_t *leaf_start,
                     uint32_t *domain_flag, void *ws, size_t ws_bytes, hipStream_t stream);

/* Most points fmm2d_build_tree_noalloc accepts. */
#define FMM2D_NOALLOC_MAX_POINTS 4194304

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * fmm2d_build_tree without a workspace argument.  Same arguments and results
 * as fmm2d_build_tree (perm, leaf_start and domain_flag are still the
 * caller's); the sort's workspace is a fixed device array of the library,
 * sized for FMM2D_NOALLOC_MAX_POINTS points (67,371,264 bytes), of which each device
 * the call runs on holds its own copy until the process ends.  The call
 * allocates nothing.  0 <= n <= FMM2D_NOALLOC_MAX_POINTS, else
 * FMM2D_EWORKSPACE (n too large) or FMM2D_EINVAL (n < 0), on the host before
 * any HIP call.  All calls on one device share its array: calls that overlap
 * on one device (other streams, other host threads) race and give undefined
 * results; calls ordered on one stream are safe.
 */
int fmm2d_build_tree_noalloc(const float *xy, int64_t n, int depth, int32_t *perm, int32_t *leaf_start,
                             uint32_t *domain_flag, hipStream_t stream);

/* dst[i][c] = src[perm[i]][c] for i < n, c < width (float rows). */
int fmm2d_gather(const float *src, const int32_t *perm, int64_t n, int width, float *dst,
                 hipStream_t stream);

/* dst[perm[i]][c] = src[i][c] for i < n, c < width (inverse of fmm2d_gather). */
int fmm2d_scatter(const float *src, const int32_t *perm, int64_t n, int width, float *dst,
                  hipStream_t stream);

/* ---------------------------------------------------- upward sweep ------ */

/*
 * P2M (Sec. 2.1, stage 2): multipole expansion of every leaf,
 *   M~_k(leaf) = sum_{s in leaf} q_s ((z_s - c)/h)^k,  k < p.
 *   xy_sorted [n][2], q_sorted [n] float; leaf_start from fmm2d_build_tree.
 *   M [num_boxes(depth)][p] complex float: the leaf level is overwritten,
 *   other levels are untouched.
 */
int fmm2d_p2m(const float *xy_sorted, const float *q_sorted, const int32_t *leaf_start, int depth,
              int p, float *M, hipStream_t stream);

/*
 * M2M (Sec. 2.1, stage 2): multipole expansions of levels depth-1 .. 0 from
 * their children (exact binomial shift in the scaled basis),
 *   M~_k(parent) = 2^-k sum_children sum_{j<=k} C(k,j) u^(k-j) M~_j(child),
 * u = (c_child - c_parent)/h_child = (+-1 +- i)/2.  M is updated in place.
 */
int fmm2d_m2m(float *M, int depth, int p, hipStream_t stream);

/* --------------------------------------------------- downward sweep ----- */

/* Bytes of the M2L operator bank for (p, precision); 0 if unsupported. */
size_t fmm2d_m2l_operators_bytes(int p, int precision);

/*
 * Generate the M2L operator bank (Sec. 4.1, Eq. (eq:M2Lmat)): for each of the
 * 40 distinct interaction-list offsets o = (ox, oy) (source box minus target
 * box, in box widths, 2 <= max(|ox|, |oy|) <= 3) the scaled matrix
 *   A~_o[n][k] = (-1)^n C(n+k, k) d^-(n+k+1),   d = -(ox + i oy),
 * the log-potential row r_o[0] = log d, r_o[k] = -d^-k / k, and the rows of
 * the transposed (adjoint) form.  Entries are computed in FP64 on the device
 * and rounded once to the precision's storage format, in a layout private to
 * the library.  One bank serves every level and both fmm2d_m2l and
 * fmm2d_m2l_backward.  ops must hold fmm2d_m2l_operators_bytes(p, precision).
 */
int fmm2d_m2l_operators(int p, int precision, void *ops, size_t ops_bytes, hipStream_t stream);

/*
 * M2L plus reduction (Sec. 4.1, steps 1-3 of the downward sweep) on every box
 * of levels lmin..lmax:
 *   L~(t) = sum_{s in IL(t)} A~_(s-t) M~(s)
 *   b(t)  = sum_{s in IL(t)} [ r_(s-t) . M~(s) + log(h_l) M~_0(s) ]
 * where IL(t) is the interaction list: boxes of t's level that are children
 * of the neighbours of t's parent (or of the parent itself) and are not
 * adjacent to t (27 in the interior, fewer at the boundary).  In the unscaled
 * basis this is L_n(t) = sum_s sum_k (-1)^n C(n+k,k) (x_t - x_s)^-(n+k+1) M_k(s).
 *   M  [num_boxes][p] complex float, read on levels lmin..lmax
 *   L  [num_boxes][p] complex float, OVERWRITTEN on levels lmin..lmax
 *   b  [num_boxes] complex float or NULL, overwritten on levels lmin..lmax
 *   ops  bank from fmm2d_m2l_operators(p, precision), ops_bytes its size
 * Each L~(t) is accumulated in registers in a fixed order and written once:
 * results are bit-reproducible from run to run.  M and L must not overlap.
 */
int fmm2d_m2l(const float *M, float *L, float *b, int depth, int p, int lmin, int lmax,
              int precision, const void *ops, size_t ops_bytes, hipStream_t stream);

/*
 * Adjoint M2L (transpose translation): the plain transpose (no conjugation)
 * of fmm2d_m2l as a complex-linear map of M~,
 *   gM~(s) = sum_{t : s in IL(t)} [ A~_(s-t)^T gL~(t) + (r_(s-t) + log(h_l) e_0) gb(t) ].
 * Since the list relation is symmetric and A~(d)^T = -A~(-d), this is a
 * gather over s's own interaction list.
 *   gL [num_boxes][p] complex float, read on levels lmin..lmax
 *   gb [num_boxes] complex float or NULL (treated as zero)
 *   gM [num_boxes][p] complex float, OVERWRITTEN on levels lmin..lmax
 * Same ops bank as the forward call.
 */
int fmm2d_m2l_backward(const float *gL, const float *gb, float *gM, int depth, int p, int lmin,
                       int lmax, int precision, const void *ops, size_t ops_bytes,
                       hipStream_t stream);

/*
 * L2L (Sec. 2.1, stage 3, "aggregation of LEs"), accumulated in FP64:
 *   L(l) = Lm2l(l) + shift(L(l-1)) for l = 1..depth (levels 0-1 of Lm2l are
 *   taken as zero), with the exact re-expansion
 *   L~_n(child) = sum_{m>=n} C(m,n) u^(m-n) 2^-(m+1) L~_m(parent),
 *   b(child)    = b(parent) + sum_m L~_m(parent) (u/2)^(m+1)/(m+1),
 *   u = (c_child - c_parent)/h_child.
 *   Lm2l [num_boxes][p] complex float, bm2l [num_boxes] complex float or NULL
 *   (read on levels 2..depth)
 *   L [num_boxes][p] complex double, b [num_boxes] complex double or NULL:
 *   written on every level.  b and bm2l must be both NULL or both non-NULL.
 */
int fmm2d_l2l(const float *Lm2l, const float *bm2l, double *L, double *b, int depth, int p,
              hipStream_t stream);

/* -------------------------------------------------------- far field ----- */

/*
 * L2P (Sec. 2.1, stage 4): evaluate the leaf local expansions at the targets,
 *   field += (1/h) sum_n L~_n w^n,   phi += b + sum_n L~_n w^(n+1)/(n+1),
 *   w = (z - c_leaf)/h.   Evaluated in FP64, accumulated into FP32 outputs.
 *   txy_sorted [nt][2], tleaf_start [4^depth + 1] (targets' own tree; nt must
 *   equal tleaf_start[4^depth]: targets beyond it are ignored);
 *   L, b from fmm2d_l2l (b may be NULL: phi then omits the constant);
 *   phi, field [nt] complex float, ACCUMULATED into; either may be NULL.
 */
int fmm2d_l2p(const float *txy_sorted, const int32_t *tleaf_start, int64_t nt, const double *L,
              const double *b, int depth, int p, float *phi, float *field, hipStream_t stream);

/* ------------------------------------------------------- near field ----- */

/*
 * P2P (Sec. 2.1, stage 5): direct interaction of every target with the
 * sources of the 3x3 block of leaves around its own leaf (that leaf
 * included), coincident pairs skipped:
 *   phi += q_s log(z - z_s),  field += q_s / (z - z_s)   (principal log branch).
 * Sources and targets are each in their own leaf order (nt = tleaf_start[4^depth]).
 * phi, field [nt] complex float, ACCUMULATED into; either may be NULL.  Sources
 * closer than FP32 can resolve (squared distance 0) count as coincident.
 */
int fmm2d_p2p(const float *xy_sorted, const float *q_sorted, const int32_t *leaf_start,
              const float *txy_sorted, const int32_t *tleaf_start, int64_t nt, int depth,
              float *phi, float *field, hipStream_t stream);

/* ------------------------------------------ transposes (gradients) ------ */
/*
 * The plain transposes of the linear stages above, for the gradient of a real
 * loss l with respect to the charges q and the source positions (x, y) at a
 * frozen tree.  With cphi = conj(dl/dRe phi + i dl/dIm phi) at the targets
 * (and cfield likewise) the chain
 *   l2p_backward -> l2l_backward -> m2l_backward -> m2m_backward -> p2m_backward
 * plus p2p_backward yields dl/dq_s and G_s = sum_t c_t dK_ts/dz_s, from which
 * dl/dx_s = Re G_s and dl/dy_s = -Im G_s.
 */

/* gL~ (leaf level) and gb (leaf level) = L2P^T applied to the cotangents:
 *   gL~_n += sum_t [cphi_t w^(n+1)/(n+1) + cfield_t w^n / h],  gb += sum_t cphi_t.
 * cphi, cfield [nt] complex float in target leaf order (either may be NULL).
 * gL [num_boxes][p] and gb [num_boxes] complex double: the leaf level is
 * OVERWRITTEN, other levels untouched. */
int fmm2d_l2p_backward(const float *txy_sorted, const int32_t *tleaf_start, const float *cphi,
                       const float *cfield, int depth, int p, double *gL, double *gb,
                       hipStream_t stream);

/* L2L^T, an upward sweep in FP64: on entry gL (and gb) hold the cotangents of
 * the accumulated leaf-level L (and b) on the leaf level; levels above are
 * overwritten with the cotangents of the accumulated L of those levels.
 * gLm2l [num_boxes][p] and gbm2l [num_boxes] complex float (gbm2l NULL iff gb
 * NULL) receive the cotangents of the M2L outputs on levels 2..depth. */
int fmm2d_l2l_backward(double *gL, double *gb, float *gLm2l, float *gbm2l, int depth, int p,
                       hipStream_t stream);

/* M2M^T, a downward sweep: gM holds the cotangents produced by
 * fmm2d_m2l_backward on levels 2..depth (levels 0-1 are neither read nor
 * written: no M2L reads them); on return every level l >= 3 additionally holds
 * what reaches it from its ancestors, so the leaf level is the full cotangent
 * of the P2M output. */
int fmm2d_m2m_backward(float *gM, int depth, int p, hipStream_t stream);

/* P2M^T and its derivative in z_s, with w = (z_s - c)/h:
 *   gq_s = Re sum_k gM~_k w^k,  G_s = (q_s/h) sum_{k>=1} k gM~_k w^(k-1).
 * n = leaf_start[4^depth].  gq [n] float and G [n] complex float, OVERWRITTEN
 * (leaf order). */
int fmm2d_p2m_backward(const float *xy_sorted, const float *q_sorted, const int32_t *leaf_start,
                       int64_t n, int depth, int p, const float *gM, float *gq, float *G,
                       hipStream_t stream);

/* P2P^T: for every source s and the targets t of the 3x3 leaf block around it,
 *   gq_s += Re sum_t [cphi_t log(z_t - z_s) + cfield_t / (z_t - z_s)]
 *   G_s  += q_s sum_t [-cphi_t / (z_t - z_s) + cfield_t / (z_t - z_s)^2]
 * gq [n] float and G [n] complex float are ACCUMULATED into (leaf order). */
int fmm2d_p2p_backward(const float *xy_sorted, const float *q_sorted, const int32_t *leaf_start,
                       int64_t n, const float *txy_sorted, const int32_t *tleaf_start, int depth,
                       const float *cphi, const float *cfield, float *gq, float *G,
                       hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* FMM2D_H */
