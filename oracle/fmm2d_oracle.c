/*
 * fmm2d_oracle.c -- plain FP64 CPU oracle for the 2D fast multipole method of
 * Cruz, Layton & Barba, "How to obtain efficient GPU kernels: an illustration
 * using FMM & FGT algorithms" (arXiv:1009.3457).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the package's smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code with the GPU path.
 *
 * What it computes (all in double precision, complex = C99 double complex):
 *   - the N-body sum of Eq. (eq:n_body) for the logarithmic kernel in complex
 *     form, phi(z) = sum_s q_s log(z - z_s), and its derivative, the Cauchy sum
 *     f(z) = sum_s q_s / (z - z_s)  (Sec. 1; the vortex-method velocity);
 *   - the five FMM stages of Sec. 2.1 on a uniform quadtree over [0,1)^2:
 *     initialization (tree), upward sweep (P2M, M2M), downward sweep (M2L over
 *     interaction lists, reduction, L2L), far field (L2P), near field (P2P);
 *   - the M2L matrix entries of Eq. (eq:M2Lmat):
 *         a_nk = (-1)^n C(n+k, k) (x_i - x_j)^(-k-n-1),  n, k = 0..p-1,
 *     with x_i the target-cluster centre and x_j the source-cluster centre,
 *     built per translation exactly as the equation is written;
 *   - the plain transposes of every linear stage, for gradients.
 *
 * Everything is in the UNSCALED basis the paper writes:
 *   multipole  M_k = sum_s q_s (z_s - c)^k                         (k < p)
 *   local      f(z) ~ sum_n L_n (z - c)^n,
 *              phi(z) ~ b + sum_n L_n (z - c)^(n+1) / (n+1)          (n < p)
 * The log-potential constant b is the extra output row that the complex
 * logarithm needs beside Eq. (eq:M2Lmat):
 *   b = M_0 log d - sum_{k>=1} M_k d^(-k) / k,  d = c_target - c_source.
 *
 * Array layouts (shared with the GPU library only by convention):
 *   boxes of level l are stored at offset (4^l - 1)/3, in Morton order
 *   (bit 2b of the index is bit b of ix, bit 2b+1 is bit b of iy); an
 *   expansion array is [box][p] complex; points are [n][2] (x, y).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORA_MAXP 64

/* ---------------------------------------------------------------- tree --- */

static int64_t lvl_off(int l) { return (((int64_t)1 << (2 * l)) - 1) / 3; }

int64_t ora_num_boxes(int depth) { return lvl_off(depth + 1); }
int64_t ora_level_offset(int l) { return lvl_off(l); }

int64_t ora_morton(int64_t ix, int64_t iy, int l)
{
    int64_t m = 0;
    for (int bit = 0; bit < l; ++bit) {
        m |= ((ix >> bit) & 1) << (2 * bit);
        m |= ((iy >> bit) & 1) << (2 * bit + 1);
    }
    return m;
}

void ora_demorton(int64_t m, int l, int64_t *ix, int64_t *iy)
{
    int64_t x = 0, y = 0;
    for (int bit = 0; bit < l; ++bit) {
        x |= ((m >> (2 * bit)) & 1) << bit;
        y |= ((m >> (2 * bit + 1)) & 1) << bit;
    }
    *ix = x;
    *iy = y;
}

/* Centre of box (ix, iy) of level l: ((ix + 1/2) h, (iy + 1/2) h), h = 2^-l. */
static cplx box_centre(int64_t ix, int64_t iy, int l)
{
    double h = ldexp(1.0, -l);
    return ((double)ix + 0.5) * h + I * (((double)iy + 0.5) * h);
}

static cplx box_centre_m(int64_t m, int l)
{
    int64_t ix, iy;
    ora_demorton(m, l, &ix, &iy);
    return box_centre(ix, iy, l);
}

/* Leaf coordinate of x in [0,1]: floor(x 2^L) clamped to 2^L - 1. */
static int64_t leaf_coord(double x, int depth)
{
    int64_t nside = (int64_t)1 << depth;
    int64_t i = (int64_t)floor(x * (double)nside);
    if (i > nside - 1) i = nside - 1;
    return i;
}

/*
 * Initialization stage (Sec. 2.1, stage 1): hierarchical decomposition of
 * [0,1)^2 into a uniform quadtree of the given depth.  Points are assigned to
 * leaves and stably sorted by leaf Morton index.
 *   perm[j]        = original index of the j-th point in sorted order
 *   leaf_start[m]  = first sorted position of leaf m (4^depth + 1 entries)
 * Returns 0, or -4 if a point lies outside [0,1]^2 (or is NaN).
 */
int ora_build_tree(const double *xy, int64_t n, int depth, int32_t *perm,
                   int32_t *leaf_start)
{
    int64_t nleaf = (int64_t)1 << (2 * depth);
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *count = (int64_t *)calloc((size_t)nleaf + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        double x = xy[2 * i], y = xy[2 * i + 1];
        if (!(x >= 0.0 && x <= 1.0 && y >= 0.0 && y <= 1.0)) {
            free(key);
            free(count);
            return -4;
        }
        key[i] = ora_morton(leaf_coord(x, depth), leaf_coord(y, depth), depth);
        count[key[i] + 1]++;
    }
    for (int64_t m = 0; m < nleaf; ++m) count[m + 1] += count[m];
    for (int64_t m = 0; m <= nleaf; ++m) leaf_start[m] = (int32_t)count[m];
    for (int64_t i = 0; i < n; ++i) perm[count[key[i]]++] = (int32_t)i; /* stable */
    free(key);
    free(count);
    return 0;
}

/* ----------------------------------------------------------- binomials --- */

/* C(a, b) for 0 <= b <= a < 2*ORA_MAXP, by Pascal's rule (exact in FP64
 * while the values stay below 2^53, which holds for a <= 2*20). */
static double binom_tab[2 * ORA_MAXP][2 * ORA_MAXP];
static int binom_ready = 0;

static void binom_init(void)
{
    if (binom_ready) return;
    for (int a = 0; a < 2 * ORA_MAXP; ++a) {
        for (int b = 0; b < 2 * ORA_MAXP; ++b) binom_tab[a][b] = 0.0;
        binom_tab[a][0] = 1.0;
        for (int b = 1; b <= a; ++b)
            binom_tab[a][b] = binom_tab[a - 1][b - 1] + binom_tab[a - 1][b];
    }
    binom_ready = 1;
}

static double binom(int a, int b) { return binom_tab[a][b]; }

void ora_init(void) { binom_init(); }

/* Number of OpenMP threads the parallel loops use (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int ora_num_threads(void) { return omp_get_max_threads(); }
#else
int ora_num_threads(void) { return 1; }
#endif

/* ------------------------------------------------------- upward sweep --- */

/*
 * P2M (Sec. 2.1 stage 2, multipole expansion of a cluster about its centre):
 *   M_k(leaf) = sum_{s in leaf} q_s (z_s - c_leaf)^k,   k = 0..p-1.
 * xy, q are in sorted order; writes the leaf level of M, unscaled.
 */
void ora_p2m(const double *xy, const double *q, const int32_t *leaf_start,
             int depth, int p, cplx *M)
{
    int64_t nleaf = (int64_t)1 << (2 * depth);
    cplx *Mleaf = M + lvl_off(depth) * p;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t m = 0; m < nleaf; ++m) {
        cplx c = box_centre_m(m, depth);
        for (int k = 0; k < p; ++k) Mleaf[m * p + k] = 0.0;
        for (int32_t s = leaf_start[m]; s < leaf_start[m + 1]; ++s) {
            cplx w = (xy[2 * s] + I * xy[2 * s + 1]) - c;
            cplx wk = 1.0;
            for (int k = 0; k < p; ++k) {
                Mleaf[m * p + k] += q[s] * wk;
                wk *= w;
            }
        }
    }
}

/*
 * M2M (upward sweep, textbook binomial shift; exact for a truncated series):
 *   M_k(parent) = sum_{children c'} sum_{j<=k} C(k,j) (c' - c)^(k-j) M_j(c').
 * Fills levels depth-1 .. 0 from the leaf level.
 */
void ora_m2m(cplx *M, int depth, int p)
{
    binom_init();
    for (int l = depth; l >= 1; --l) {
        int64_t npar = (int64_t)1 << (2 * (l - 1));
        cplx *Mc = M + lvl_off(l) * p;
        cplx *Mp = M + lvl_off(l - 1) * p;
#pragma omp parallel for schedule(static)
        for (int64_t P = 0; P < npar; ++P) {
            int64_t px, py;
            ora_demorton(P, l - 1, &px, &py);
            cplx cp = box_centre(px, py, l - 1);
            for (int k = 0; k < p; ++k) Mp[P * p + k] = 0.0;
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) {
                    int64_t ix = 2 * px + cx, iy = 2 * py + cy;
                    int64_t ch = ora_morton(ix, iy, l);
                    cplx d = box_centre(ix, iy, l) - cp;
                    cplx dpow[ORA_MAXP];
                    dpow[0] = 1.0;
                    for (int j = 1; j < p; ++j) dpow[j] = dpow[j - 1] * d;
                    for (int k = 0; k < p; ++k)
                        for (int j = 0; j <= k; ++j)
                            Mp[P * p + k] += binom(k, j) * dpow[k - j] * Mc[ch * p + j];
                }
        }
    }
}

/* --------------------------------------------------- downward sweep ----- */

/*
 * The interaction list of box (ix, iy) at level l (Sec. 4.1, downward-sweep
 * step 1): boxes of the same level that are children of the neighbours of
 * the box's parent (neighbours include the parent itself) and are not
 * adjacent to the box (Chebyshev distance >= 2).  At most 27 boxes in 2D.
 * Writes Morton indices of the sources; returns the count.  Levels 0 and 1
 * have empty lists.
 */
int ora_interaction_list(int l, int64_t ix, int64_t iy, int64_t *out)
{
    int cnt = 0;
    if (l < 2) return 0;
    int64_t pside = (int64_t)1 << (l - 1);
    int64_t px = ix >> 1, py = iy >> 1;
    for (int64_t qy = py - 1; qy <= py + 1; ++qy)
        for (int64_t qx = px - 1; qx <= px + 1; ++qx) {
            if (qx < 0 || qy < 0 || qx >= pside || qy >= pside) continue;
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) {
                    int64_t sx = 2 * qx + cx, sy = 2 * qy + cy;
                    int64_t dx = sx - ix, dy = sy - iy;
                    if (dx < 0) dx = -dx;
                    if (dy < 0) dy = -dy;
                    if ((dx > dy ? dx : dy) >= 2) out[cnt++] = ora_morton(sx, sy, l);
                }
        }
    return cnt;
}

/*
 * The M2L matrix of Eq. (eq:M2Lmat) for centre difference d = x_i - x_j
 * (target centre minus source centre): A[n*p + k] = (-1)^n C(n+k,k) d^(-k-n-1).
 */
void ora_m2l_operator(double dre, double dim, int p, cplx *A)
{
    binom_init();
    cplx d = dre + I * dim;
    cplx dinv = 1.0 / d;
    cplx dneg[2 * ORA_MAXP]; /* dneg[j] = d^(-j) */
    dneg[0] = 1.0;
    for (int j = 1; j < 2 * p; ++j) dneg[j] = dneg[j - 1] * dinv;
    for (int n = 0; n < p; ++n)
        for (int k = 0; k < p; ++k) {
            double sign = (n % 2 == 0) ? 1.0 : -1.0;
            A[n * p + k] = sign * binom(n + k, k) * dneg[k + n + 1];
        }
}

/* The log-potential row for the same d: r_0 = log d, r_k = -d^(-k)/k. */
void ora_log_row(double dre, double dim, int p, cplx *r)
{
    cplx d = dre + I * dim;
    cplx dinv = 1.0 / d;
    cplx dk = 1.0;
    r[0] = clog(d);
    for (int k = 1; k < p; ++k) {
        dk *= dinv;
        r[k] = -dk / (double)k;
    }
}

/* One target box: L(t) = sum over its interaction list of A(c_t - c_s) M(s)
 * (step 2), summed into one local expansion (step 3, the reduction). */
static void m2l_one_target(const cplx *Mlev, int l, int64_t t, int p, cplx *Lt,
                           cplx *bt)
{
    int64_t ix, iy, list[32];
    ora_demorton(t, l, &ix, &iy);
    cplx ct = box_centre(ix, iy, l);
    int cnt = ora_interaction_list(l, ix, iy, list);
    cplx A[ORA_MAXP * ORA_MAXP], r[ORA_MAXP];
    for (int n = 0; n < p; ++n) Lt[n] = 0.0;
    if (bt) *bt = 0.0;
    for (int e = 0; e < cnt; ++e) {
        int64_t s = list[e];
        cplx d = ct - box_centre_m(s, l);
        ora_m2l_operator(creal(d), cimag(d), p, A);
        for (int n = 0; n < p; ++n)
            for (int k = 0; k < p; ++k) Lt[n] += A[n * p + k] * Mlev[s * p + k];
        if (bt) {
            ora_log_row(creal(d), cimag(d), p, r);
            for (int k = 0; k < p; ++k) *bt += r[k] * Mlev[s * p + k];
        }
    }
}

/*
 * M2L over every box of levels lmin..lmax (steps 1-3 of the downward sweep).
 * L and b (b may be NULL) are overwritten on those levels, untouched elsewhere.
 */
void ora_m2l(const cplx *M, cplx *L, cplx *b, int depth, int p, int lmin, int lmax)
{
    binom_init();
    (void)depth;
    for (int l = lmin; l <= lmax; ++l) {
        int64_t nb = (int64_t)1 << (2 * l);
        const cplx *Ml = M + lvl_off(l) * p;
        cplx *Ll = L + lvl_off(l) * p;
        cplx *bl = b ? b + lvl_off(l) : NULL;
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t t = 0; t < nb; ++t)
            m2l_one_target(Ml, l, t, p, Ll + t * p, bl ? bl + t : NULL);
    }
}

/* M2L for a sample of target boxes of one level (Morton indices `boxes`).
 * Mlev points at the level's multipoles; outputs are [nb][p] and [nb]. */
void ora_m2l_boxes(const cplx *Mlev, int l, int p, const int64_t *boxes, int64_t nb,
                   cplx *Lout, cplx *bout)
{
    binom_init();
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t e = 0; e < nb; ++e)
        m2l_one_target(Mlev, l, boxes[e], p, Lout + e * p, bout ? bout + e : NULL);
}

/*
 * Plain transpose of ora_m2l (no conjugation):
 *   gM_k(s) += sum_{t : s in IL(t)} [ sum_n A(c_t - c_s)_{nk} gL_n(t) + r_k(c_t - c_s) gb(t) ].
 * Written as the literal scatter over every (t, s) pair of every list.
 * gM is accumulated into; gb may be NULL.
 */
void ora_m2l_transpose(const cplx *gL, const cplx *gb, cplx *gM, int depth, int p,
                       int lmin, int lmax)
{
    binom_init();
    (void)depth;
    for (int l = lmin; l <= lmax; ++l) {
        int64_t nb = (int64_t)1 << (2 * l);
        const cplx *gLl = gL + lvl_off(l) * p;
        const cplx *gbl = gb ? gb + lvl_off(l) : NULL;
        cplx *gMl = gM + lvl_off(l) * p;
        /* serial scatter: every source may be written by up to 27 targets */
        for (int64_t t = 0; t < nb; ++t) {
            int64_t ix, iy, list[32];
            ora_demorton(t, l, &ix, &iy);
            cplx ct = box_centre(ix, iy, l);
            int cnt = ora_interaction_list(l, ix, iy, list);
            cplx A[ORA_MAXP * ORA_MAXP], r[ORA_MAXP];
            for (int e = 0; e < cnt; ++e) {
                int64_t s = list[e];
                cplx d = ct - box_centre_m(s, l);
                ora_m2l_operator(creal(d), cimag(d), p, A);
                for (int k = 0; k < p; ++k)
                    for (int n = 0; n < p; ++n) gMl[s * p + k] += A[n * p + k] * gLl[t * p + n];
                if (gbl) {
                    ora_log_row(creal(d), cimag(d), p, r);
                    for (int k = 0; k < p; ++k) gMl[s * p + k] += r[k] * gbl[t];
                }
            }
        }
    }
}

/*
 * The same transpose for a sample of source boxes of one level, written as a
 * gather over each source's own interaction list.  The list is symmetric at a
 * level (s is in IL(t) exactly when t is in IL(s)), so
 *   gM_k(s) = sum_{t in IL(s)} [ sum_n A(c_t - c_s)_{nk} gL_n(t) + r_k(c_t - c_s) gb(t) ],
 * with the operator built for d = c_t - c_s exactly as in the forward map.
 * gLlev, gblev point at the level's cotangents (gblev may be NULL); gMout is
 * [nb][p], overwritten.
 */
void ora_m2l_transpose_boxes(const cplx *gLlev, const cplx *gblev, int l, int p,
                             const int64_t *boxes, int64_t nb, cplx *gMout)
{
    binom_init();
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t e = 0; e < nb; ++e) {
        int64_t s = boxes[e], sx, sy, list[32];
        ora_demorton(s, l, &sx, &sy);
        cplx cs = box_centre(sx, sy, l);
        int cnt = ora_interaction_list(l, sx, sy, list);
        cplx A[ORA_MAXP * ORA_MAXP], r[ORA_MAXP];
        cplx *g = gMout + e * p;
        for (int k = 0; k < p; ++k) g[k] = 0.0;
        for (int j = 0; j < cnt; ++j) {
            int64_t t = list[j];
            cplx d = box_centre_m(t, l) - cs;
            ora_m2l_operator(creal(d), cimag(d), p, A);
            for (int k = 0; k < p; ++k)
                for (int n = 0; n < p; ++n) g[k] += A[n * p + k] * gLlev[t * p + n];
            if (gblev) {
                ora_log_row(creal(d), cimag(d), p, r);
                for (int k = 0; k < p; ++k) g[k] += r[k] * gblev[t];
            }
        }
    }
}

/* Sets the number of threads the parallel loops use (no-op without OpenMP). */
void ora_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * L2L (downward sweep, "aggregation of LEs"; textbook exact re-expansion of a
 * truncated polynomial), delta = c_child - c_parent:
 *   L_n(child) += sum_{m>=n} C(m,n) delta^(m-n) L_m(parent)
 *   b(child)   += b(parent) + sum_m L_m(parent) delta^(m+1) / (m+1)
 * Inputs: Lm2l, bm2l = the M2L outputs of every level (levels 0-1 zero).
 * Outputs: L, b = accumulated local expansions of every level (bm2l, b may be
 * NULL together).
 */
void ora_l2l(const cplx *Lm2l, const cplx *bm2l, cplx *L, cplx *b, int depth, int p)
{
    binom_init();
    int64_t ntot = lvl_off(depth + 1);
    memcpy(L, Lm2l, sizeof(cplx) * (size_t)(ntot * p));
    if (b) memcpy(b, bm2l, sizeof(cplx) * (size_t)ntot);
    for (int l = 1; l <= depth; ++l) {
        int64_t nb = (int64_t)1 << (2 * l);
        cplx *Lc = L + lvl_off(l) * p;
        const cplx *Lp = L + lvl_off(l - 1) * p;
        cplx *bc = b ? b + lvl_off(l) : NULL;
        const cplx *bp = b ? b + lvl_off(l - 1) : NULL;
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nb; ++c) {
            int64_t ix, iy;
            ora_demorton(c, l, &ix, &iy);
            int64_t P = ora_morton(ix >> 1, iy >> 1, l - 1);
            cplx delta = box_centre(ix, iy, l) - box_centre(ix >> 1, iy >> 1, l - 1);
            cplx dpow[ORA_MAXP + 1];
            dpow[0] = 1.0;
            for (int j = 1; j <= p; ++j) dpow[j] = dpow[j - 1] * delta;
            for (int n = 0; n < p; ++n)
                for (int m = n; m < p; ++m)
                    Lc[c * p + n] += binom(m, n) * dpow[m - n] * Lp[P * p + m];
            if (bc) {
                bc[c] += bp[P];
                for (int m = 0; m < p; ++m) bc[c] += Lp[P * p + m] * dpow[m + 1] / (double)(m + 1);
            }
        }
    }
}

/*
 * Plain transpose of ora_l2l with respect to (Lm2l, bm2l), computed in place:
 * on entry gL, gb hold the cotangents of the accumulated L, b at every level;
 * on exit they hold the cotangents of Lm2l, bm2l (an upward sweep).
 */
void ora_l2l_transpose(cplx *gL, cplx *gb, int depth, int p)
{
    binom_init();
    for (int l = depth; l >= 1; --l) {
        int64_t npar = (int64_t)1 << (2 * (l - 1));
        const cplx *gc = gL + lvl_off(l) * p;
        cplx *gp = gL + lvl_off(l - 1) * p;
        const cplx *gbc = gb ? gb + lvl_off(l) : NULL;
        cplx *gbp = gb ? gb + lvl_off(l - 1) : NULL;
#pragma omp parallel for schedule(static)
        for (int64_t P = 0; P < npar; ++P) {
            int64_t px, py;
            ora_demorton(P, l - 1, &px, &py);
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) {
                    int64_t ix = 2 * px + cx, iy = 2 * py + cy;
                    int64_t c = ora_morton(ix, iy, l);
                    cplx delta = box_centre(ix, iy, l) - box_centre(px, py, l - 1);
                    cplx dpow[ORA_MAXP + 1];
                    dpow[0] = 1.0;
                    for (int j = 1; j <= p; ++j) dpow[j] = dpow[j - 1] * delta;
                    for (int m = 0; m < p; ++m)
                        for (int n = 0; n <= m; ++n)
                            gp[P * p + m] += binom(m, n) * dpow[m - n] * gc[c * p + n];
                    if (gbp) {
                        gbp[P] += gbc[c];
                        for (int m = 0; m < p; ++m)
                            gp[P * p + m] += gbc[c] * dpow[m + 1] / (double)(m + 1);
                    }
                }
        }
    }
}

/*
 * Plain transpose of ora_m2m, in place: on entry gM holds the direct
 * cotangents of M at every level (from M2L^T); on exit the cotangent of the
 * leaf level includes everything that reached it through M2M (a downward
 * sweep: gM(child) += T^T gM(parent)).
 */
void ora_m2m_transpose(cplx *gM, int depth, int p)
{
    binom_init();
    for (int l = 1; l <= depth; ++l) {
        int64_t nb = (int64_t)1 << (2 * l);
        cplx *gc = gM + lvl_off(l) * p;
        const cplx *gp = gM + lvl_off(l - 1) * p;
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nb; ++c) {
            int64_t ix, iy;
            ora_demorton(c, l, &ix, &iy);
            int64_t P = ora_morton(ix >> 1, iy >> 1, l - 1);
            cplx d = box_centre(ix, iy, l) - box_centre(ix >> 1, iy >> 1, l - 1);
            cplx dpow[ORA_MAXP];
            dpow[0] = 1.0;
            for (int j = 1; j < p; ++j) dpow[j] = dpow[j - 1] * d;
            for (int j = 0; j < p; ++j)
                for (int k = j; k < p; ++k) gc[c * p + j] += binom(k, j) * dpow[k - j] * gp[P * p + k];
        }
    }
}

/* ----------------------------------------------------------- far field --- */

/*
 * L2P (Sec. 2.1 stage 4), w = z - c_leaf:
 *   f(z)   += sum_n L_n w^n
 *   phi(z) += b + sum_n L_n w^(n+1)/(n+1)
 * txy in sorted order (tleaf_start); phi, f accumulate; b may be NULL.
 */
void ora_l2p(const double *txy, const int32_t *tleaf_start, const cplx *L, const cplx *b,
             int depth, int p, cplx *phi, cplx *f)
{
    int64_t nleaf = (int64_t)1 << (2 * depth);
    const cplx *Ll = L + lvl_off(depth) * p;
    const cplx *bl = b ? b + lvl_off(depth) : NULL;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t m = 0; m < nleaf; ++m) {
        cplx c = box_centre_m(m, depth);
        for (int32_t t = tleaf_start[m]; t < tleaf_start[m + 1]; ++t) {
            cplx w = (txy[2 * t] + I * txy[2 * t + 1]) - c;
            cplx wn = 1.0, fs = 0.0, ps = bl ? bl[m] : 0.0;
            for (int n = 0; n < p; ++n) {
                fs += Ll[m * p + n] * wn;
                wn *= w;
                ps += Ll[m * p + n] * wn / (double)(n + 1);
            }
            if (f) f[t] += fs;
            if (phi) phi[t] += ps;
        }
    }
}

/* Plain transpose of ora_l2p: gL_n(leaf) += sum_t [cphi_t w^(n+1)/(n+1) + cf_t w^n],
 * gb(leaf) += sum_t cphi_t.  cphi / cf may be NULL. */
void ora_l2p_transpose(const double *txy, const int32_t *tleaf_start, const cplx *cphi,
                       const cplx *cf, int depth, int p, cplx *gL, cplx *gb)
{
    int64_t nleaf = (int64_t)1 << (2 * depth);
    cplx *gLl = gL + lvl_off(depth) * p;
    cplx *gbl = gb ? gb + lvl_off(depth) : NULL;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t m = 0; m < nleaf; ++m) {
        cplx c = box_centre_m(m, depth);
        for (int32_t t = tleaf_start[m]; t < tleaf_start[m + 1]; ++t) {
            cplx w = (txy[2 * t] + I * txy[2 * t + 1]) - c;
            cplx wn = 1.0;
            for (int n = 0; n < p; ++n) {
                if (cf) gLl[m * p + n] += cf[t] * wn;
                wn *= w;
                if (cphi) gLl[m * p + n] += cphi[t] * wn / (double)(n + 1);
            }
            if (gbl && cphi) gbl[m] += cphi[t];
        }
    }
}

/* ---------------------------------------------------------- near field --- */

/*
 * P2P (Sec. 2.1 stage 5): direct sum over the sources of the 3x3 block of
 * leaves around the target's leaf (its own leaf included); coincident pairs
 * are skipped.  phi += q log(z - z_s), f += q / (z - z_s).  Accumulates.
 */
void ora_p2p(const double *xy, const double *q, const int32_t *leaf_start,
             const double *txy, const int32_t *tleaf_start, int depth, cplx *phi, cplx *f)
{
    int64_t nside = (int64_t)1 << depth;
    int64_t nleaf = nside * nside;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t m = 0; m < nleaf; ++m) {
        int64_t ix, iy;
        ora_demorton(m, depth, &ix, &iy);
        for (int32_t t = tleaf_start[m]; t < tleaf_start[m + 1]; ++t) {
            cplx z = txy[2 * t] + I * txy[2 * t + 1];
            cplx ps = 0.0, fs = 0.0;
            for (int64_t sy = iy - 1; sy <= iy + 1; ++sy)
                for (int64_t sx = ix - 1; sx <= ix + 1; ++sx) {
                    if (sx < 0 || sy < 0 || sx >= nside || sy >= nside) continue;
                    int64_t sm = ora_morton(sx, sy, depth);
                    for (int32_t s = leaf_start[sm]; s < leaf_start[sm + 1]; ++s) {
                        cplx r = z - (xy[2 * s] + I * xy[2 * s + 1]);
                        if (r == 0.0) continue;
                        ps += q[s] * clog(r);
                        fs += q[s] / r;
                    }
                }
            if (phi) phi[t] += ps;
            if (f) f[t] += fs;
        }
    }
}

/*
 * Near-field part of the gradient (plain transpose of ora_p2p in q, and its
 * derivative in the source positions).  For every source s, over the targets
 * t of the 3x3 leaf block around s's leaf, with c_t = cphi_t (and cf_t):
 *   gq_s += Re sum_t [cphi_t log(z_t - z_s) + cf_t / (z_t - z_s)]
 *   G_s  += q_s sum_t [cphi_t * (-1/(z_t - z_s)) + cf_t / (z_t - z_s)^2]
 * so that dl/dx_s = Re G_s and dl/dy_s = -Im G_s.  Accumulates.
 */
void ora_p2p_transpose(const double *xy, const double *q, const int32_t *leaf_start,
                       const double *txy, const int32_t *tleaf_start, int depth,
                       const cplx *cphi, const cplx *cf, double *gq, cplx *G)
{
    int64_t nside = (int64_t)1 << depth;
    int64_t nleaf = nside * nside;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t m = 0; m < nleaf; ++m) {
        int64_t ix, iy;
        ora_demorton(m, depth, &ix, &iy);
        for (int32_t s = leaf_start[m]; s < leaf_start[m + 1]; ++s) {
            cplx zs = xy[2 * s] + I * xy[2 * s + 1];
            cplx acc_q = 0.0, acc_G = 0.0;
            for (int64_t ty = iy - 1; ty <= iy + 1; ++ty)
                for (int64_t tx = ix - 1; tx <= ix + 1; ++tx) {
                    if (tx < 0 || ty < 0 || tx >= nside || ty >= nside) continue;
                    int64_t tm = ora_morton(tx, ty, depth);
                    for (int32_t t = tleaf_start[tm]; t < tleaf_start[tm + 1]; ++t) {
                        cplx r = (txy[2 * t] + I * txy[2 * t + 1]) - zs;
                        if (r == 0.0) continue;
                        if (cphi) {
                            acc_q += cphi[t] * clog(r);
                            acc_G += cphi[t] * (-1.0 / r);
                        }
                        if (cf) {
                            acc_q += cf[t] / r;
                            acc_G += cf[t] / (r * r);
                        }
                    }
                }
            gq[s] += creal(acc_q);
            G[s] += q[s] * acc_G;
        }
    }
}

/*
 * Far-field part of the source gradient: plain transpose of ora_p2m in q and
 * its derivative in z_s, with w = z_s - c_leaf and gM the leaf-level
 * multipole cotangent:
 *   gq_s += Re sum_k gM_k w^k
 *   G_s  += q_s sum_{k>=1} gM_k k w^(k-1)
 */
void ora_p2m_transpose(const double *xy, const double *q, const int32_t *leaf_start,
                       int depth, int p, const cplx *gM, double *gq, cplx *G)
{
    int64_t nleaf = (int64_t)1 << (2 * depth);
    const cplx *gMl = gM + lvl_off(depth) * p;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t m = 0; m < nleaf; ++m) {
        cplx c = box_centre_m(m, depth);
        for (int32_t s = leaf_start[m]; s < leaf_start[m + 1]; ++s) {
            cplx w = (xy[2 * s] + I * xy[2 * s + 1]) - c;
            cplx wk = 1.0, accq = 0.0, accG = 0.0;
            for (int k = 0; k < p; ++k) {
                accq += gMl[m * p + k] * wk;
                if (k + 1 < p) accG += gMl[m * p + k + 1] * (double)(k + 1) * wk;
                wk *= w;
            }
            gq[s] += creal(accq);
            G[s] += q[s] * accG;
        }
    }
}

/* ---------------------------------------------------------- direct sum --- */

/*
 * Eq. (eq:n_body) evaluated directly, O(N Nt): for every target z_t,
 *   phi_t = sum_s q_s log(z_t - z_s),  f_t = sum_s q_s / (z_t - z_s),
 * coincident pairs skipped.  Overwrites phi, f (either may be NULL).
 */
void ora_direct(const double *xy, const double *q, int64_t n, const double *txy, int64_t nt,
                cplx *phi, cplx *f)
{
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nt; ++t) {
        cplx z = txy[2 * t] + I * txy[2 * t + 1];
        cplx ps = 0.0, fs = 0.0;
        for (int64_t s = 0; s < n; ++s) {
            cplx r = z - (xy[2 * s] + I * xy[2 * s + 1]);
            if (r == 0.0) continue;
            ps += q[s] * clog(r);
            fs += q[s] / r;
        }
        if (phi) phi[t] = ps;
        if (f) f[t] = fs;
    }
}

/*
 * Exact gradient of a loss l(phi) through the direct sum, for cotangents
 * cphi_t = conj(dl/dRe phi_t + i dl/dIm phi_t):
 *   gq_s = Re sum_t cphi_t log(z_t - z_s),  G_s = q_s sum_t cphi_t (-1/(z_t - z_s)).
 * Overwrites gq, G.
 */
void ora_direct_grad(const double *xy, const double *q, int64_t n, const double *txy,
                     int64_t nt, const cplx *cphi, double *gq, cplx *G)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        cplx zs = xy[2 * s] + I * xy[2 * s + 1];
        cplx aq = 0.0, aG = 0.0;
        for (int64_t t = 0; t < nt; ++t) {
            cplx r = (txy[2 * t] + I * txy[2 * t + 1]) - zs;
            if (r == 0.0) continue;
            aq += cphi[t] * clog(r);
            aG += cphi[t] * (-1.0 / r);
        }
        gq[s] = creal(aq);
        G[s] = q[s] * aG;
    }
}
