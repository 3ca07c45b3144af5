"""Pins for the FP64 oracle: checks against facts fixed by the paper and by
mathematics (closed forms, series, counts, exactness, finite differences), not
against the oracle's own formulas.  CPU only."""
import os

import numpy as np
import pytest

import oracle
import synthetic as sy

HERE = os.path.dirname(os.path.abspath(__file__))


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


# ---------------------------------------------------------- direct sum ---

def test_direct_sum_ngon_closed_form():
    """n equal charges on a circle: sum_s log(z - c - r w^s) = log((z-c)^n - r^n),
    and the Cauchy sum is n (z-c)^(n-1) / ((z-c)^n - r^n)."""
    nside, r, c, qv = 7, 0.1, 0.45 + 0.55j, 0.75
    ang = 2 * np.pi * np.arange(nside) / nside
    src = c + r * np.exp(1j * ang)
    xy = np.stack([src.real, src.imag], 1)
    q = np.full(nside, qv)
    tz = np.array([0.05 + 0.1j, 0.9 + 0.95j, 0.47 + 0.52j, 0.2 + 0.8j])
    phi, f = oracle.direct(xy, q, np.stack([tz.real, tz.imag], 1))
    w = tz - c
    assert np.allclose(phi.real, qv * np.log(np.abs(w ** nside - r ** nside)), atol=1e-13)
    assert np.allclose(f, qv * nside * w ** (nside - 1) / (w ** nside - r ** nside),
                       rtol=1e-12)


def test_direct_skips_coincident_pair():
    xy = np.array([[0.25, 0.25], [0.75, 0.5]])
    q = np.array([1.0, -2.0])
    phi, f = oracle.direct(xy, q, xy)
    d = 0.5 + 0.25j
    assert np.isclose(phi[0], -2.0 * np.log(-d))
    assert np.isclose(f[1], 1.0 / d)


# ------------------------------------------------------------- operator ---

@pytest.mark.parametrize("p", [8, 12, 20])
def test_operator_columns_are_taylor_coefficients(p):
    """Column k of Eq. (eq:M2Lmat) must be the Taylor series about the target
    centre of (z - x_j)^-(k+1): sum_n a_nk w^n = (w + d)^-(k+1) for |w| << |d|."""
    d = 2.0 - 3.0j
    A = oracle.m2l_operator(d, p)
    w = np.array([0.01 + 0.004j, -0.007j, 0.006 - 0.002j])
    for k in range(p):
        series = np.array([np.sum(A[:, k] * wi ** np.arange(p)) for wi in w])
        exact = (w + d) ** (-(k + 1))
        assert np.allclose(series, exact, rtol=1e-12, atol=0)


def test_log_row_is_series_of_log_potential():
    """b from the log row is the value at the target centre of the source
    cluster's log expansion M_0 log(z - x_j) - sum_{k>=1} M_k (z - x_j)^-k / k;
    for one charge at z_s that is q log(x_i - z_s)."""
    p = 24
    cs, ct = 0.3 + 0.2j, 0.9 + 0.7j
    zs, qv = cs + (0.03 - 0.04j), 0.7
    M = qv * (zs - cs) ** np.arange(p)
    r = oracle.log_row(ct - cs, p)
    assert np.isclose(np.sum(r * M), qv * np.log(ct - zs), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("p", [8, 12, 16, 20])
def test_operator_identities(p):
    """A(d)^T = -A(-d) (the Cauchy kernel is odd) and
    A(d) = diag((-1)^n d^-(n+1)) B diag(d^-k), B_nk = C(n+k, k) (Pascal)."""
    from math import comb
    for d in [3.0 + 0j, -2.0 + 1.0j, 2.0 - 3.0j, -3.0 - 3.0j]:
        A = oracle.m2l_operator(d, p)
        Am = oracle.m2l_operator(-d, p)
        assert np.allclose(A.T, -Am, rtol=1e-13, atol=0)
        B = np.array([[comb(n + k, k) for k in range(p)] for n in range(p)], np.float64)
        n = np.arange(p)
        left = ((-1.0) ** n) * d ** (-(n + 1))
        right = d ** (-n.astype(np.float64))
        assert np.allclose(A, left[:, None] * B * right[None, :], rtol=1e-12, atol=0)


@pytest.mark.parametrize("p", [8, 12, 20])
def test_symmetric_offset_identities(p):
    """The negative of an offset shares the scalings of the offset itself:
    A(-d) = D1(d) B' D2(d) with B'_nk = -(-1)^(n+k) C(n+k, k), and the log row
    r(-d)_k = (-1)^k r(d)_k for k >= 1, r(-d)_0 = r(d)_0 +- i pi."""
    from math import comb, pi
    for d in [2.0 + 0j, -2.0 + 1.0j, 1.0 - 2.0j, -2.0 - 2.0j, 0.0 + 2.0j]:
        Am = oracle.m2l_operator(-d, p)
        n = np.arange(p)
        Bp = np.array([[-((-1) ** (a + k)) * comb(a + k, k) for k in range(p)] for a in range(p)], np.float64)
        left = ((-1.0) ** n) * d ** (-(n + 1))
        right = d ** (-n.astype(np.float64))
        assert np.allclose(Am, left[:, None] * Bp * right[None, :], rtol=1e-12, atol=0)
        r, rm = oracle.log_row(d, p), oracle.log_row(-d, p)
        assert np.allclose(rm[1:], ((-1.0) ** n[1:]) * r[1:], rtol=1e-13, atol=0)
        assert np.isclose(abs(rm[0] - r[0]), pi, rtol=1e-14) and abs((rm[0] - r[0]).real) < 1e-14


def test_single_pair_p2m_m2l_l2p_vs_direct():
    """One source box, one well-separated target box: P2M -> M2L -> L2P
    reproduces the direct Cauchy and log sums to the truncation error."""
    g = sy.rng(5)
    cs, ct = 0.3 + 0.3j, 0.3 + 0.3j + 3 * 0.125
    h = 0.125
    zs = cs + h * (g.random(20) - 0.5 + 1j * (g.random(20) - 0.5))
    q = 2 * g.random(20) - 1
    zt = ct + h * (g.random(10) - 0.5 + 1j * (g.random(10) - 0.5))
    p = 20
    M = np.array([np.sum(q * (zs - cs) ** k) for k in range(p)])
    A = oracle.m2l_operator(ct - cs, p)
    L = A @ M
    b = np.sum(oracle.log_row(ct - cs, p) * M)
    w = zt - ct
    f = np.array([np.sum(L * wi ** np.arange(p)) for wi in w])
    phi = np.array([b + np.sum(L * wi ** (np.arange(p) + 1) / (np.arange(p) + 1)) for wi in w])
    f_ex = np.array([np.sum(q / (z - zs)) for z in zt])
    phi_ex = np.array([np.sum(q * np.log(np.abs(z - zs))) for z in zt])
    assert _rel(f, f_ex) < 1e-9
    assert _rel(phi.real, phi_ex) < 1e-10


# --------------------------------------------------------------- counts ---

def test_interaction_list_counts_closed_form():
    """Brute-force list sizes versus IL(l) = 4(3*2^l - 4)^2 - (3*2^l - 2)^2, the
    count of same-level box pairs whose parents touch minus pairs that touch."""
    for l in range(2, 7):
        ns = 1 << l
        tot = sum(oracle.interaction_list(l, ix, iy).size for ix in range(ns) for iy in range(ns))
        assert tot == 4 * (3 * 2 ** l - 4) ** 2 - (3 * 2 ** l - 2) ** 2
        mx = max(oracle.interaction_list(l, ix, iy).size for ix in range(ns) for iy in range(ns))
        assert mx == (12 if l == 2 else 27)  # Sec. 4.1: 27 per interior node in 2D


def test_padded_counts_match_paper_tables():
    """The paper's translation counts are 27 list entries for every box of
    levels 2..L (Table tab:m2ltesla; example 4^5 x 27 in Sec. 4.1)."""
    rows = np.loadtxt(os.path.join(HERE, "golden", "paper_m2l_translation_counts.txt"),
                      dtype=np.int64)
    for depth, count in rows:
        boxes = sum(4 ** l for l in range(2, depth + 1))
        assert 27 * boxes == count
        # every interior box of the deepest level of the brute-force list has 27
        ns = 1 << min(depth, 5)
        sizes = [oracle.interaction_list(min(depth, 5), ix, iy).size
                 for ix in range(3, ns - 3) for iy in range(3, ns - 3)]
        assert all(s == 27 for s in sizes)
    assert 4 ** 5 * 27 == 27648


def test_interaction_list_is_symmetric_and_well_separated():
    l = 4
    ns = 1 << l
    pairs = set()
    for ix in range(ns):
        for iy in range(ns):
            t = oracle.morton(ix, iy, l)
            for s in oracle.interaction_list(l, ix, iy):
                pairs.add((t, int(s)))
    for t, s in pairs:
        assert (s, t) in pairs


# ----------------------------------------------------------------- tree ---

def test_build_tree_sorts_stably_and_clamps():
    xy = np.array([[0.9, 0.1], [1.0, 1.0], [0.1, 0.1], [0.0, 0.0], [0.99, 0.1], [0.5, 0.5]],
                  np.float32).astype(np.float64)
    perm, ls = oracle.build_tree(xy, 1)
    assert list(perm) == [2, 3, 0, 4, 1, 5]
    assert list(ls) == [0, 2, 4, 4, 6]
    with pytest.raises(ValueError):
        oracle.build_tree(np.array([[0.5, 1.5]]), 2)


# --------------------------------------------------------- exact stages ---

def test_m2m_equals_p2m_at_parent():
    """A truncated binomial shift is exact: M2M of the leaves' expansions must
    equal P2M computed directly about the parent centres."""
    depth, p = 4, 12
    xy = sy.uniform(3000, 11).astype(np.float64)
    q = sy.charges(3000, 12).astype(np.float64)
    perm, ls = oracle.build_tree(xy, depth)
    M = oracle.m2m(oracle.p2m(xy[perm], q[perm], ls, depth, p), depth, p)
    for lev in range(1, depth):
        perm2, ls2 = oracle.build_tree(xy, lev)
        Mp = oracle.p2m(xy[perm2], q[perm2], ls2, lev, p)
        o0, o1 = oracle.level_offset(lev), oracle.level_offset(lev + 1)
        assert np.allclose(M[o0:o1], Mp[o0:o1], rtol=1e-11, atol=1e-12)


def test_l2l_reexpansion_is_exact():
    """Re-expanding a degree p-1 local polynomial about a child centre changes
    nothing: evaluating the parent's expansion and the child's gives the same
    f and phi at every point of the child."""
    depth, p = 3, 10
    g = sy.rng(21)
    nb = oracle.num_boxes(depth)
    Lm = np.zeros((nb, p), complex)
    bm = np.zeros(nb, complex)
    o = oracle.level_offset(depth - 1)
    cnt = 4 ** (depth - 1)
    Lm[o:o + cnt] = g.standard_normal((cnt, p)) + 1j * g.standard_normal((cnt, p))
    bm[o:o + cnt] = g.standard_normal(cnt) + 1j * g.standard_normal(cnt)
    L, b = oracle.l2l(Lm, bm, depth, p)
    t = sy.uniform(500, 22).astype(np.float64)
    tp, tls = oracle.build_tree(t, depth)
    phi1, f1 = oracle.l2p(t[tp], tls, L, b, depth, p)
    tp2, tls2 = oracle.build_tree(t, depth - 1)
    nb2 = oracle.num_boxes(depth - 1)
    phi2, f2 = oracle.l2p(t[tp2], tls2, Lm[:nb2], bm[:nb2], depth - 1, p)
    a1 = np.empty_like(phi1); a1[tp] = phi1
    a2 = np.empty_like(phi2); a2[tp2] = phi2
    c1 = np.empty_like(f1); c1[tp] = f1
    c2 = np.empty_like(f2); c2[tp2] = f2
    assert np.allclose(a1, a2, rtol=1e-12, atol=1e-12)
    assert np.allclose(c1, c2, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------- the whole FMM ---

def _c1(seed=1, n=4096):
    xy = sy.uniform(n, seed).astype(np.float64)
    q = sy.charges(n, seed + 1).astype(np.float64)
    return xy, q


def test_fmm_vs_direct_c1():
    """N=4096 uniform, depth 4, p=8: FP64 FMM vs the O(N^2) sum.  Thresholds
    calibrated once on this seed (measured 7.1e-6 / 3.6e-5) and frozen."""
    xy, q = _c1()
    phi_d, f_d = oracle.direct(xy, q, xy)
    phi, f = oracle.fmm(xy, q, xy, 4, 8)
    assert _rel(phi.real, phi_d.real) < 2e-5
    assert _rel(f, f_d) < 1e-4


def test_fmm_convergence_in_p():
    xy, q = _c1(seed=3, n=2048)
    phi_d, f_d = oracle.direct(xy, q, xy)
    errs = []
    for p in (4, 8, 12, 16, 20):
        phi, f = oracle.fmm(xy, q, xy, 4, p)
        errs.append(_rel(f, f_d))
    for a, b in zip(errs, errs[1:]):
        assert b < 0.5 * a or b < 1e-12
    assert errs[-1] < 1e-8


def test_fmm_ngon_closed_form():
    """The FMM with a 64-gon of equal charges matches the closed form."""
    nside, r, c = 64, 0.3, 0.5 + 0.5j
    src = c + r * np.exp(2j * np.pi * np.arange(nside) / nside)
    xy = np.stack([src.real, src.imag], 1)
    q = np.ones(nside)
    t = sy.uniform(200, 9).astype(np.float64)
    phi, f = oracle.fmm(xy, q, t, 4, 20)
    w = (t[:, 0] + 1j * t[:, 1]) - c
    assert _rel(phi.real, np.log(np.abs(w ** nside - r ** nside))) < 1e-9
    assert _rel(f, nside * w ** (nside - 1) / (w ** nside - r ** nside)) < 1e-8


def test_m2l_linearity():
    depth, p = 4, 8
    g = sy.rng(7)
    nb = oracle.num_boxes(depth)
    M1 = g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))
    M2 = g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))
    a, bb = 0.3 - 1.2j, -2.0 + 0.5j
    L1, b1 = oracle.m2l(M1, depth, p)
    L2, b2 = oracle.m2l(M2, depth, p)
    L3, b3 = oracle.m2l(a * M1 + bb * M2, depth, p)
    assert np.allclose(L3, a * L1 + bb * L2, rtol=1e-12, atol=1e-9)
    assert np.allclose(b3, a * b1 + bb * b2, rtol=1e-12, atol=1e-9)


def test_m2l_adjoint_dot_product_and_skew_symmetry():
    """<M2L(M), G> = <M, M2L^T(G)> (bilinear, no conjugation), with the
    transpose written as an independent scatter; and without the log row the
    whole per-level M2L is skew: M2L^T = -M2L."""
    depth, p = 4, 8
    g = sy.rng(8)
    nb = oracle.num_boxes(depth)
    M = g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))
    G = g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))
    gb = g.standard_normal(nb) + 1j * g.standard_normal(nb)
    L, b = oracle.m2l(M, depth, p)
    gM = oracle.m2l_transpose(G, gb, depth, p)
    lhs = np.sum(L[oracle.level_offset(2):] * G[oracle.level_offset(2):]) + \
        np.sum(b[oracle.level_offset(2):] * gb[oracle.level_offset(2):])
    rhs = np.sum(M * gM)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    gM0 = oracle.m2l_transpose(G, None, depth, p)
    LG, _ = oracle.m2l(G, depth, p, with_b=False)
    assert np.allclose(gM0, -LG, rtol=1e-12, atol=1e-9)


def test_scaled_basis_roundtrip_is_exact():
    depth, p = 5, 12
    g = sy.rng(4)
    nb = oracle.num_boxes(depth)
    M = g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))
    assert np.array_equal(oracle.unscale_multipoles(oracle.scale_multipoles(M, depth), depth), M)
    assert np.array_equal(oracle.unscale_locals(oracle.scale_locals(M, depth), depth), M)


def test_scale_multipoles_closed_form():
    """One source q at z: the multipole expansion of the level-l box holding it
    is M_k = q (z - c_l)^k, so the scaled one must be q ((z - c_l) / h_l)^k with
    h_l = 2^-l.  The closed form is formed here from the box centre; only
    P2M, M2M and scale_multipoles come from the oracle.  A wrong exponent sign
    or power in the helper fails at every level but the root."""
    depth, p = 6, 12
    z = 0.3712890625 + 0.6259765625j  # exact in FP32 and FP64
    q = -0.75
    xy = np.array([[z.real, z.imag]])
    perm, ls = oracle.build_tree(xy, depth)
    M = oracle.m2m(oracle.p2m(xy[perm], np.array([q]), ls, depth, p), depth, p)
    Ms = oracle.scale_multipoles(M, depth)
    k = np.arange(p)
    for l in range(depth + 1):
        h = 2.0 ** -l
        ix, iy = int(z.real / h), int(z.imag / h)
        c = (ix + 0.5) * h + 1j * (iy + 0.5) * h
        row = Ms[oracle.level_offset(l) + oracle.morton(ix, iy, l)]
        expect = q * ((z - c) / h) ** k
        assert np.allclose(row, expect, rtol=1e-12, atol=1e-14), l
        # every other box of the level is empty
        lev = Ms[oracle.level_offset(l):oracle.level_offset(l + 1)]
        assert np.count_nonzero(np.abs(lev).sum(axis=1)) == 1


def test_scale_locals_closed_form():
    """A unit charge at the centre of box s gives, in a box t of its
    interaction list, L_n = (-1)^n q d^-(n+1) with d = c_t - c_s (the k = 0
    column of Eq. (eq:M2Lmat)).  Scaled by h^(n+1), that is
    (-1)^n q delta^-(n+1) with delta = d / h the integer box offset: the same
    numbers at every level.  The closed form uses only the integer offset."""
    p, q = 12, 1.5
    n = np.arange(p)
    for l in (2, 3, 5):
        side = 1 << l
        sx, sy = 1, side - 2
        for tx, ty in ((sx + 2, sy), (sx + 3, sy - 2), (sx - 1, sy + 1), (sx + 2, sy + 1)):
            if not (0 <= tx < side and 0 <= ty < side):
                continue
            t_m = oracle.morton(tx, ty, l)
            if oracle.morton(sx, sy, l) not in oracle.interaction_list(l, tx, ty):
                continue
            depth = l
            M = np.zeros((oracle.num_boxes(depth), p), np.complex128)
            M[oracle.level_offset(l) + oracle.morton(sx, sy, l), 0] = q
            L, _ = oracle.m2l(M, depth, p, l, l)
            Ls = oracle.scale_locals(L, depth)
            delta = complex(tx - sx, ty - sy)
            expect = (-1.0) ** n * q * delta ** -(n + 1.0)
            assert np.allclose(Ls[oracle.level_offset(l) + t_m], expect, rtol=1e-13, atol=0), (l, tx, ty)
            # and unscaled it carries the level's powers of h
            h = 2.0 ** -l
            assert np.allclose(L[oracle.level_offset(l) + t_m], expect * h ** -(n + 1.0), rtol=1e-13, atol=0)


def test_transpose_gather_equals_scatter():
    """The sampled transpose (a gather over each source's own list) equals the
    literal scatter, which the dot-product test pins, at every box of every
    level, with and without the log row's cotangent."""
    depth, p = 4, 8
    g = sy.rng(12)
    nb = oracle.num_boxes(depth)
    G = g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))
    gb = g.standard_normal(nb) + 1j * g.standard_normal(nb)
    for gbv in (gb, None):
        ref = oracle.m2l_transpose(G, gbv, depth, p)
        for l in range(2, depth + 1):
            lo, hi = oracle.level_offset(l), oracle.level_offset(l + 1)
            boxes = np.arange(hi - lo)
            got = oracle.m2l_transpose_boxes(G[lo:hi], None if gbv is None else gbv[lo:hi], l, p, boxes)
            assert np.allclose(got, ref[lo:hi], rtol=1e-12, atol=1e-12), l


def test_scaled_operator_is_level_independent():
    """In the scaled basis L~_n = L_n h^(n+1), M~_k = M_k / h^k the M2L matrix
    depends only on the offset in box widths."""
    p = 12
    for lev in (2, 5, 9):
        h = 2.0 ** -lev
        d_box = 2.0 - 3.0j
        A = oracle.m2l_operator(d_box * h, p)
        n = np.arange(p)
        As = (h ** (n + 1))[:, None] * A * (h ** n)[None, :]
        assert np.allclose(As, oracle.m2l_operator(d_box, p), rtol=1e-13, atol=0)


# ----------------------------------------------------------- gradients ---

def _loss_setup(n=4096, nt=256, depth=4, p=12):
    xy = sy.uniform(n, 31).astype(np.float64)
    q = sy.charges(n, 32).astype(np.float64)
    t = sy.uniform(nt, 33).astype(np.float64)
    return xy, q, t, depth, p


def test_gradient_matches_exact_direct_gradient():
    xy, q, t, depth, p = _loss_setup()
    phi, _ = oracle.fmm(xy, q, t, depth, p)
    gq, gxy = oracle.fmm_grad(xy, q, t, depth, p, (2 * phi.real).astype(complex))
    phid, _ = oracle.direct(xy, q, t)
    gqd, gxyd = oracle.direct_grad(xy, q, t, (2 * phid.real).astype(complex))
    assert _rel(gq, gqd) < 1e-6
    assert _rel(gxy, gxyd) < 1e-5


def test_gradient_matches_central_differences():
    """Central differences (h = 1e-3) of l = sum (Re phi)^2 through the FP64
    FMM at a frozen tree, for sources away from targets and leaf edges."""
    xy, q, t, depth, p = _loss_setup()
    phi, _ = oracle.fmm(xy, q, t, depth, p)
    gq, gxy = oracle.fmm_grad(xy, q, t, depth, p, (2 * phi.real).astype(complex))
    hstep = 1e-3
    side = 2.0 ** depth
    tz = t[:, 0] + 1j * t[:, 1]
    cand = []
    for s in sy.rng(34).permutation(xy.shape[0]):
        z = xy[s, 0] + 1j * xy[s, 1]
        frac = np.concatenate([xy[s] * side - np.floor(xy[s] * side)])
        if np.min(np.abs(tz - z)) > 1e-2 and np.all(frac > 2 * hstep * side) and \
                np.all(frac < 1 - 2 * hstep * side):
            cand.append(s)
        if len(cand) == 12:
            break

    def loss(xy_, q_):
        ph, _ = oracle.fmm(xy_, q_, t, depth, p)
        return np.sum(ph.real ** 2)

    fd_x, an_x, fd_q, an_q = [], [], [], []
    for s in cand:
        for dim in range(2):
            a = xy.copy(); a[s, dim] += hstep
            b = xy.copy(); b[s, dim] -= hstep
            fd_x.append((loss(a, q) - loss(b, q)) / (2 * hstep))
            an_x.append(gxy[s, dim])
        a = q.copy(); a[s] += hstep
        b = q.copy(); b[s] -= hstep
        fd_q.append((loss(xy, a) - loss(xy, b)) / (2 * hstep))
        an_q.append(gq[s])
    assert _rel(np.array(an_q), np.array(fd_q)) < 1e-9  # l is quadratic in q
    assert _rel(np.array(an_x), np.array(fd_x)) < 2e-3


def test_target_position_gradient_is_the_field():
    """d(Re phi)/dx_t = Re f and d(Re phi)/dy_t = -Im f at a target (phi is
    holomorphic in z_t with phi' = f), through the FP64 FMM: central
    differences of l = sum (Re phi)^2 over target positions against
    2 Re phi (Re f, -Im f), for targets away from leaf edges."""
    xy, q, t, depth, p = _loss_setup(nt=64)
    phi, f = oracle.fmm(xy, q, t, depth, p)
    hstep, side = 1e-6, 2.0 ** depth
    fd, an = [], []
    for i in range(t.shape[0]):
        frac = t[i] * side - np.floor(t[i] * side)
        if np.any(frac < 1e-3) or np.any(frac > 1 - 1e-3):
            continue
        for dim in range(2):
            a = t.copy(); a[i, dim] += hstep
            b = t.copy(); b[i, dim] -= hstep
            la = np.sum(oracle.fmm(xy, q, a, depth, p)[0].real ** 2)
            lb = np.sum(oracle.fmm(xy, q, b, depth, p)[0].real ** 2)
            fd.append((la - lb) / (2 * hstep))
            g = 2 * phi[i].real * f[i]
            an.append(g.real if dim == 0 else -g.imag)
        if len(fd) >= 16:
            break
    assert len(fd) >= 16
    assert _rel(np.array(an), np.array(fd)) < 1e-6
