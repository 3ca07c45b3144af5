"""GPU parity of the fast Gauss transform's Hermite stage (include/fgt2d.h)
against the FP64 oracle (Sec. 2.2, Sec. 4.2).

Tolerances.  Coefficients are summed in FP64 on both sides and rounded once
to FP32 on the GPU, so each one agrees to 2^-24 relative (2.5e-7 allowed).
The evaluation runs in FP32: per target it sums p^2 (2K+1)^2 terms
A_ab h_a h_b whose magnitudes stay within a small factor of |G| (|A_ab| decays
as (r/2)^(a+b)/(a! b!) while |h_n| grows at most as 2^(n/2) sqrt(n!)), and the
Hermite recurrences add about n ulp to h_n.  Measured against max |G| the
error is a few 1e-7; the tests allow 1e-5 (2e-5 for p = 16)."""
import math

import numpy as np
import pytest

import oracle
import synthetic as sy
from oracle import fgt as ofgt
from tests._inputs import rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1009_3457_amd as P
    return P


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _sigma32(depth):
    """sigma = sqrt(2) 2^-depth (box width r sqrt(2) sigma with r = 1/2), as
    the FP32 value the library receives."""
    return float(np.float32(math.sqrt(2.0) * 2.0 ** -depth))


def _sources(n, depth, seed, kind="uniform"):
    xy = sy.uniform(n, seed) if kind == "uniform" else sy.mixed(n, seed)
    q = sy.charges(n, seed + 1)
    perm, ls = oracle.build_tree(xy.astype(np.float64), depth)
    return xy, q, perm, ls


def _gpu_coeffs(P, xy, q, depth, p, sigma):
    perm, ls = P.build_tree(_t(xy), depth)
    return P.fgt_hermite_coeffs(P.gather(_t(xy), perm), P.gather(_t(q), perm), ls, depth, p, sigma)


def _max_rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("p", [1, 5, 9, 12, 16])
def test_coefficients_match_oracle(P, p):
    depth, sigma = 4, _sigma32(4)
    xy, q, perm, ls = _sources(30000, depth, 3, "mixed")
    A = _gpu_coeffs(P, xy, q, depth, p, sigma).cpu().numpy().astype(np.float64)
    Ar = ofgt.hermite_coeffs(xy[perm].astype(np.float64), q[perm].astype(np.float64), ls, depth, p, sigma)
    assert np.all(np.abs(A - Ar) <= 2.5e-7 * np.abs(Ar) + 1e-37)
    empty = np.diff(ls) == 0
    assert not A[empty].any()


@pytest.mark.parametrize("depth,p,K,nt,order", [
    (4, 5, 8, 25600, "sorted"),
    (4, 9, 8, 25600, "sorted"),
    (4, 12, 8, 25600, "sorted"),
    (5, 12, 8, 102400 + 37, "sorted"),   # ragged tail
    (5, 16, 3, 5000, "random"),          # unsorted: one sweep per distinct box
    (3, 12, 0, 3001, "sorted"),          # own box only
    (3, 7, 7, 2000, "random"),           # K spans the whole grid
    (1, 4, 1, 500, "random"),
    (0, 6, 0, 300, "sorted"),            # a single box
    (4, 14, 5, 7777, "random"),          # p not a multiple of 4
    (2, 13, 3, 999, "sorted"),
])
def test_eval_matches_oracle(P, depth, p, K, nt, order):
    """Evaluation alone: the GPU kernel and the oracle on the same FP32
    coefficients (the oracle's, rounded once)."""
    print(f"fgt eval depth={depth} p={p} K={K} nt={nt} {order}", flush=True)
    sigma = _sigma32(depth)
    xy, q, perm, ls = _sources(100 * 4 ** depth, depth, 7)
    A32 = ofgt.hermite_coeffs(xy[perm].astype(np.float64), q[perm].astype(np.float64), ls, depth, p,
                              sigma).astype(np.float32)
    t = sy.uniform(nt, 8)
    if order == "sorted":
        tp, _ = oracle.build_tree(t.astype(np.float64), depth)
        t = t[tp]
    t[:3] = [[0.0, 0.0], [1.0, 1.0], [1.0, 0.0]]  # the closed edges of the domain
    G = P.fgt_hermite_eval(_t(t), depth, p, sigma, K, _t(A32)).cpu().numpy()
    Gr = ofgt.hermite_eval(t.astype(np.float64), depth, p, sigma, K, A32.astype(np.float64))
    tol = 2e-5 if p >= 16 else 1e-5
    assert _max_rel(G, Gr) < tol, _max_rel(G, Gr)


@pytest.mark.parametrize("depth,p", [(4, 12), (5, 9)])
def test_gauss_transform_matches_direct_sum(P, depth, p):
    """End to end: tree, coefficients and evaluation on the GPU against the
    exact transform of Eq. (eqn:dgt); at K = 8 and r = 1/2 the cutoff leaves
    exp(-16) per source and the oracle's own Hermite result is within 4e-8."""
    import torch
    sigma = _sigma32(depth)
    n = 100 * 4 ** depth
    xy = sy.mixed(n, 21)
    q = sy.charges(n, 22)
    t = sy.uniform(4000, 23)
    G = P.gauss_transform(_t(xy), _t(q), _t(t), depth, p, sigma, 8).cpu().numpy()
    Gd = ofgt.direct(xy.astype(np.float64), q.astype(np.float64), t.astype(np.float64), sigma)
    assert _max_rel(G, Gd) < 1e-5
    assert rel(G, Gd) < 1e-5
    del torch


def test_empty_and_sparse_inputs(P):
    """No targets: nothing to do.  Sources in one corner: most boxes empty,
    their coefficients zero, far targets get exactly zero."""
    import torch
    depth, p, sigma = 4, 9, _sigma32(4)
    A = torch.zeros(256, p, p, dtype=torch.float32, device="cuda")
    assert P.fgt_hermite_eval(torch.zeros(0, 2, device="cuda"), depth, p, sigma, 2, A).numel() == 0
    xy = (sy.uniform(500, 31) * 0.1).astype(np.float32)  # inside box (0, 0) .. (1, 1)
    q = sy.charges(500, 32)
    A = _gpu_coeffs(P, xy, q, depth, p, sigma)
    t = np.array([[0.95, 0.95], [0.03, 0.02], [0.5, 0.05]], np.float32)
    G = P.fgt_hermite_eval(_t(t), depth, p, sigma, 2, A).cpu().numpy()
    assert G[0] == 0.0 and G[2] == 0.0 and G[1] != 0.0
    perm, ls = oracle.build_tree(xy.astype(np.float64), depth)
    Gr = ofgt.hermite_eval(t.astype(np.float64), depth, p, sigma, 2,
                           ofgt.hermite_coeffs(xy[perm].astype(np.float64), q[perm].astype(np.float64),
                                               ls, depth, p, sigma))
    assert abs(G[1] - Gr[1]) < 1e-5 * abs(Gr[1])


def test_full_size_sampled():
    """The benchmark's workload, 6,553,600 targets on a 256 x 256 grid, p = 12,
    K = 8, in the launch configuration the benchmark times: every target
    evaluated on the GPU, 3000 of them checked against the oracle."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1009_3457_amd as P
    depth, p, K = 8, 12, 8
    sigma = _sigma32(depth)
    n = 100 * 4 ** depth
    print(f"fgt full size n={n}", flush=True)
    xy = sy.uniform(n, 41)
    q = sy.charges(n, 42)
    t = sy.uniform(n, 43)
    perm, ls = P.build_tree(_t(xy), depth)
    A = P.fgt_hermite_coeffs(P.gather(_t(xy), perm), P.gather(_t(q), perm), ls, depth, p, sigma)
    tperm, _ = P.build_tree(_t(t), depth)
    ts = P.gather(_t(t), tperm)
    G = P.fgt_hermite_eval(ts, depth, p, sigma, K, A).cpu().numpy()
    ts = ts.cpu().numpy()
    pr, lr = oracle.build_tree(xy.astype(np.float64), depth)
    Ar = ofgt.hermite_coeffs(xy[pr].astype(np.float64), q[pr].astype(np.float64), lr, depth, p, sigma)
    idx = np.random.Generator(np.random.PCG64(44)).choice(n, 3000, replace=False)
    Gr = ofgt.hermite_eval(ts[idx].astype(np.float64), depth, p, sigma, K, Ar)
    assert _max_rel(G[idx], Gr) < 1e-5
