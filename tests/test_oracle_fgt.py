"""Pins of the FP64 fast-Gauss-transform oracle (Hermite evaluation,
Sec. 2.2 and Sec. 4.2) against facts fixed outside it: numpy's Hermite
polynomials, the Hermite generating function, convergence of the series to
the direct Gauss sum, Cramer's bound on the truncation error, the Gaussian
cutoff bound, and the p = 1 special case.

Throughout, boxes have width w = 2^-depth and sigma = sqrt(2) w, i.e. the box
width is r sqrt(2) sigma with r = 1/2, so a source lies within r/2 of its box
centre in each coordinate of s = (x - s_B)/(sqrt(2) sigma)."""
import math

import numpy as np
import pytest
from numpy.polynomial import hermite as npherm

import oracle
import synthetic as sy
from oracle import fgt


def _sigma(depth):
    return math.sqrt(2.0) * 2.0 ** -depth


def _setup(n, nt, depth, seed):
    xy = sy.uniform(n, seed).astype(np.float64)
    q = sy.charges(n, seed + 1).astype(np.float64)
    t = sy.uniform(nt, seed + 2).astype(np.float64)
    perm, ls = oracle.build_tree(xy, depth)
    return xy, q, t, xy[perm], q[perm], ls


def test_hermite_functions_match_numpy():
    """h_n(t) = exp(-t^2) H_n(t) against numpy's physicists' Hermite series."""
    p = 20
    for t in np.linspace(-6.0, 6.0, 25):
        h = fgt.hermite_functions(t, p)
        ref = np.array([npherm.hermval(t, [0.0] * n + [1.0]) for n in range(p)]) * math.exp(-t * t)
        scale = np.maximum(np.abs(ref), 1e-300)
        assert np.all(np.abs(h - ref) <= 1e-12 * scale + 1e-300), t


def test_hermite_generating_function():
    """exp(-(t - s)^2) = sum_n s^n / n! h_n(t): the identity behind the
    Hermite expansion of one Gaussian (Sec. 2.2)."""
    for t in np.linspace(-4.0, 4.0, 17):
        h = fgt.hermite_functions(t, 40)
        for s in np.linspace(-0.5, 0.5, 11):
            series = sum(s ** n / math.factorial(n) * h[n] for n in range(40))
            assert abs(series - math.exp(-(t - s) ** 2)) < 1e-13, (t, s)


def test_coefficients_of_one_source():
    """One source: A_ab = q s1^a s2^b / (a! b!) in its own box, zero elsewhere."""
    depth, p = 3, 6
    x = np.array([[0.61, 0.23]])
    q = np.array([0.7])
    perm, ls = oracle.build_tree(x, depth)
    A = fgt.hermite_coeffs(x[perm], q[perm], ls, depth, p, _sigma(depth))
    bx, by = int(0.61 * 8), int(0.23 * 8)
    m = oracle.morton(bx, by, depth)
    s = (x[0] - (np.array([bx, by]) + 0.5) / 8) / (math.sqrt(2.0) * _sigma(depth))
    ref = np.array([[0.7 * s[0] ** a * s[1] ** b / (math.factorial(a) * math.factorial(b))
                     for b in range(p)] for a in range(p)])
    assert np.allclose(A[m], ref, rtol=1e-14, atol=0)
    others = np.delete(A, m, axis=0)
    assert not others.any()


def test_series_converges_to_box_direct_sum():
    """With p large the Hermite evaluation equals the direct Gauss sum over
    the same (2K+1)^2 boxes (Eq. (eqn:dgt) vs Eq. (eqn:hermite))."""
    depth, K, sigma = 3, 2, _sigma(3)
    xy, q, t, xs, qs, ls = _setup(2000, 500, depth, 5)
    A = fgt.hermite_coeffs(xs, qs, ls, depth, 22, sigma)
    G = fgt.hermite_eval(t, depth, 22, sigma, K, A)
    Gd = fgt.direct_boxes(xs, qs, ls, depth, t, sigma, K)
    assert np.max(np.abs(G - Gd)) < 1e-11 * np.max(np.abs(Gd))


def _cramer_tail(p, smax, kmax=80):
    """rho(p) >= sum_{n>=p} |s|^n/n! |h_n(t)| for |s| <= smax, from Cramer's
    inequality |H_n(t)| exp(-t^2/2) <= k 2^(n/2) sqrt(n!), k < 1.0865."""
    return 1.0865 * sum((math.sqrt(2.0) * smax) ** n / math.sqrt(math.factorial(n)) for n in range(p, kmax))


@pytest.mark.parametrize("p", [3, 5, 9, 12])
def test_truncation_error_within_bound(p):
    """|G_p - G_direct| <= sum |q| (2 rho + rho^2) per target: with
    f = f1 f2 and T = (f1 - R1)(f2 - R2), |f - T| <= |R1| + |R2| + |R1 R2|
    since 0 < f_i <= 1 and |R_i| <= rho(p) for |s_i| <= r/2 = 1/4."""
    depth, K, sigma = 4, 3, _sigma(4)
    xy, q, t, xs, qs, ls = _setup(6000, 800, depth, 11)
    A = fgt.hermite_coeffs(xs, qs, ls, depth, p, sigma)
    G = fgt.hermite_eval(t, depth, p, sigma, K, A)
    Gd = fgt.direct_boxes(xs, qs, ls, depth, t, sigma, K)
    rho = _cramer_tail(p, 0.25)
    qabs = fgt.direct_boxes(xs, np.abs(qs), ls, depth, t, 1e30, K)  # sum |q| over the boxes
    err = np.abs(G - Gd)
    assert np.all(err <= qabs * (2 * rho + rho * rho)), (p, float(np.max(err / qabs)), rho)
    if p >= 9:  # and the series is not merely bounded: it converges
        assert np.max(err) < 1e-5 * np.max(np.abs(Gd))


def test_cutoff_error_within_bound():
    """Sources outside the (2K+1)^2 boxes lie at least K w from the target, so
    each contributes at most exp(-(K w)^2 / (2 sigma^2)) = exp(-K^2 r^2)."""
    depth, K, sigma = 4, 3, _sigma(4)
    xy, q, t, xs, qs, ls = _setup(6000, 800, depth, 13)
    G = fgt.direct(xy, q, t, sigma)
    Gb = fgt.direct_boxes(xs, qs, ls, depth, t, sigma, K)
    bound = np.sum(np.abs(q)) * math.exp(-(K * 0.5) ** 2)
    assert np.max(np.abs(G - Gb)) <= bound
    assert np.max(np.abs(G - Gb)) > 0  # the cut is real at this K


def test_p1_is_gaussians_at_box_centres():
    """p = 1: A_00 is the box's total charge and h_0(t) = exp(-t^2), so the
    evaluation is sum_B Q_B exp(-|y - s_B|^2 / (2 sigma^2))."""
    depth, K, sigma = 3, 2, _sigma(3)
    xy, q, t, xs, qs, ls = _setup(1500, 300, depth, 17)
    A = fgt.hermite_coeffs(xs, qs, ls, depth, 1, sigma)
    G = fgt.hermite_eval(t, depth, 1, sigma, K, A)
    side = 8
    bx = np.minimum((xy[:, 0] * side).astype(int), side - 1)
    by = np.minimum((xy[:, 1] * side).astype(int), side - 1)
    Q = np.zeros((side, side))
    np.add.at(Q, (bx, by), q)
    tx = np.minimum((t[:, 0] * side).astype(int), side - 1)
    ty = np.minimum((t[:, 1] * side).astype(int), side - 1)
    ref = np.zeros(len(t))
    for i in range(side):
        for j in range(side):
            near = (np.abs(tx - i) <= K) & (np.abs(ty - j) <= K)
            d2 = (t[:, 0] - (i + 0.5) / side) ** 2 + (t[:, 1] - (j + 0.5) / side) ** 2
            ref += np.where(near, Q[i, j] * np.exp(-d2 / (2 * sigma * sigma)), 0.0)
    assert np.max(np.abs(G - ref)) < 1e-13 * np.max(np.abs(ref))


def test_whole_grid_matches_full_transform():
    """K spanning the grid and p large: the Hermite evaluation is the whole
    Gauss transform of Eq. (eqn:dgt)."""
    depth, sigma = 2, _sigma(2)
    xy, q, t, xs, qs, ls = _setup(800, 200, depth, 19)
    G, _ = fgt.gauss_transform(xy, q, t, depth, 24, sigma, 3)
    Gd = fgt.direct(xy, q, t, sigma)
    assert np.max(np.abs(G - Gd)) < 1e-11 * np.max(np.abs(Gd))
