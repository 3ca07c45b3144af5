/*
 * fgt2d_oracle.c -- plain FP64 CPU oracle for the Hermite-series evaluation
 * of the fast Gauss transform in Cruz, Layton & Barba, "How to obtain
 * efficient GPU kernels: an illustration using FMM & FGT algorithms"
 * (arXiv:1009.3457), Sec. 2.2 and Sec. 4.2.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests and the CPU baseline leg of the benchmark
 * do.  It shares no code with the GPU path.
 *
 * In two dimensions, with sigma the Gaussian width:
 *   - Eq. (eqn:dgt), the discrete Gauss transform
 *         G(y) = sum_i q_i exp(-|x_i - y|^2 / (2 sigma^2));
 *   - Eq. (eqn:A_alpha), the Hermite coefficients of the sources of box B
 *     about its centre s_B, for the multi-index alpha = (a, b):
 *         A_ab = 1/(a! b!) sum_j q_j s1^a s2^b,   s = (x_j - s_B)/(sqrt(2) sigma);
 *   - Eq. (eqn:hermite), their evaluation at a target y,
 *         G(y) ~ sum_B sum_{a,b < p} A_ab(B) h_a(t1) h_b(t2),  t = (y - s_B)/(sqrt(2) sigma),
 *     with h_n(t) = exp(-t^2) H_n(t) and H_n the physicists' Hermite
 *     polynomials (Sec. 2.2).
 *
 * Readings (the paper leaves them open):
 *   - the multi-index runs over the square 0 <= a, b < p (p^2 terms per box);
 *   - the boxes are the 4^depth leaves of the uniform grid over [0,1)^2 that
 *     the tree build uses, each box its own source cluster with s_B its centre;
 *   - a target in box (tx, ty) takes the clusters (bx, by) with
 *     |bx - tx| <= K and |by - ty| <= K (clipped to the grid).
 *
 * Layouts: points [n][2] (x, y); coefficients [4^depth][p][p] indexed
 * [morton box][a][b]; sources given in leaf order with leaf_start as for the
 * FMM tree.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define FGT_MAXP 64

int64_t ora_morton(int64_t ix, int64_t iy, int l);
void ora_demorton(int64_t m, int l, int64_t *ix, int64_t *iy);

static int64_t fgt_box_coord(double x, int depth)
{
    int64_t nside = (int64_t)1 << depth;
    int64_t i = (int64_t)floor(x * (double)nside);
    if (i < 0) i = 0;
    if (i > nside - 1) i = nside - 1;
    return i;
}

/* h_n(t) = exp(-t^2) H_n(t) for n < p, from H_0 = 1, H_1 = 2t and
 * H_{n+1} = 2t H_n - 2n H_{n-1} (the physicists' Hermite polynomials). */
void ora_hermite_functions(double t, int p, double *h)
{
    double e = exp(-t * t);
    double hm = 0.0, hn = 1.0; /* H_{n-1}, H_n */
    for (int n = 0; n < p; ++n) {
        h[n] = e * hn;
        double next = 2.0 * t * hn - 2.0 * (double)n * hm;
        hm = hn;
        hn = next;
    }
}

/* Eq. (eqn:dgt) by direct summation, every source against every target. */
void ora_fgt_direct(const double *xy, const double *q, int64_t n, const double *txy,
                    int64_t nt, double sigma, double *G)
{
    double c = 1.0 / (2.0 * sigma * sigma);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nt; ++t) {
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double dx = xy[2 * i] - txy[2 * t], dy = xy[2 * i + 1] - txy[2 * t + 1];
            acc += q[i] * exp(-(dx * dx + dy * dy) * c);
        }
        G[t] = acc;
    }
}

/* Eq. (eqn:dgt) restricted to the sources of the (2K+1)^2 boxes around each
 * target's box: the quantity the Hermite evaluation approximates. */
void ora_fgt_direct_boxes(const double *xy_sorted, const double *q_sorted,
                          const int32_t *leaf_start, int depth, const double *txy,
                          int64_t nt, double sigma, int K, double *G)
{
    int64_t nside = (int64_t)1 << depth;
    double c = 1.0 / (2.0 * sigma * sigma);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nt; ++t) {
        double y1 = txy[2 * t], y2 = txy[2 * t + 1];
        int64_t tx = fgt_box_coord(y1, depth), ty = fgt_box_coord(y2, depth);
        double acc = 0.0;
        for (int64_t by = ty - K; by <= ty + K; ++by) {
            if (by < 0 || by >= nside) continue;
            for (int64_t bx = tx - K; bx <= tx + K; ++bx) {
                if (bx < 0 || bx >= nside) continue;
                int64_t m = ora_morton(bx, by, depth);
                for (int32_t j = leaf_start[m]; j < leaf_start[m + 1]; ++j) {
                    double dx = xy_sorted[2 * j] - y1, dy = xy_sorted[2 * j + 1] - y2;
                    acc += q_sorted[j] * exp(-(dx * dx + dy * dy) * c);
                }
            }
        }
        G[t] = acc;
    }
}

/* Eq. (eqn:A_alpha) for every box of the grid at `depth`. */
void ora_fgt_hermite_coeffs(const double *xy_sorted, const double *q_sorted,
                            const int32_t *leaf_start, int depth, int p, double sigma,
                            double *A)
{
    int64_t nbox = (int64_t)1 << (2 * depth);
    double w = ldexp(1.0, -depth), scale = 1.0 / (sqrt(2.0) * sigma);
    double fact[FGT_MAXP];
    fact[0] = 1.0;
    for (int n = 1; n < p; ++n) fact[n] = fact[n - 1] * (double)n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t m = 0; m < nbox; ++m) {
        int64_t bx, by;
        ora_demorton(m, depth, &bx, &by);
        double c1 = ((double)bx + 0.5) * w, c2 = ((double)by + 0.5) * w;
        double *Am = A + m * p * p;
        for (int i = 0; i < p * p; ++i) Am[i] = 0.0;
        for (int32_t j = leaf_start[m]; j < leaf_start[m + 1]; ++j) {
            double s1 = (xy_sorted[2 * j] - c1) * scale, s2 = (xy_sorted[2 * j + 1] - c2) * scale;
            double pa = 1.0; /* s1^a */
            for (int a = 0; a < p; ++a) {
                double pb = 1.0; /* s2^b */
                for (int b = 0; b < p; ++b) {
                    Am[a * p + b] += q_sorted[j] * pa * pb;
                    pb *= s2;
                }
                pa *= s1;
            }
        }
        for (int a = 0; a < p; ++a)
            for (int b = 0; b < p; ++b) Am[a * p + b] /= fact[a] * fact[b];
    }
}

/* Eq. (eqn:hermite) at every target, summed over the (2K+1)^2 boxes around
 * the target's box (clipped to the grid).  Targets in any order. */
void ora_fgt_hermite_eval(const double *txy, int64_t nt, int depth, int p, double sigma, int K,
                          const double *A, double *G)
{
    int64_t nside = (int64_t)1 << depth;
    double w = ldexp(1.0, -depth), scale = 1.0 / (sqrt(2.0) * sigma);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nt; ++t) {
        double y1 = txy[2 * t], y2 = txy[2 * t + 1];
        int64_t tx = fgt_box_coord(y1, depth), ty = fgt_box_coord(y2, depth);
        double h1[FGT_MAXP], h2[FGT_MAXP];
        double acc = 0.0;
        for (int64_t by = ty - K; by <= ty + K; ++by) {
            if (by < 0 || by >= nside) continue;
            ora_hermite_functions((y2 - ((double)by + 0.5) * w) * scale, p, h2);
            for (int64_t bx = tx - K; bx <= tx + K; ++bx) {
                if (bx < 0 || bx >= nside) continue;
                ora_hermite_functions((y1 - ((double)bx + 0.5) * w) * scale, p, h1);
                const double *Am = A + ora_morton(bx, by, depth) * p * p;
                for (int a = 0; a < p; ++a)
                    for (int b = 0; b < p; ++b) acc += Am[a * p + b] * h1[a] * h2[b];
            }
        }
        G[t] = acc;
    }
}
