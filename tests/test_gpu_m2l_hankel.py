"""GPU parity of the Hankel-form M2L (precision FMM2D_F64_HANKEL: every
translation of Eq. (eq:M2Lmat) as a Hankel product between two diagonal
scalings, the interaction-list sum taken over spectra of length 2p in FP64)
and of its adjoint, against the FP64 oracle, through the C ABI.

Tolerances (relative Frobenius error per level): L~ and gM~ 1e-6 (FP64
arithmetic; what remains is the rounding of the FP32 inputs and outputs),
b 1e-5 (the log row is summed in FP32, as in the other forms).  A worst-box
check bounds the error of any single box against the level's RMS box norm.
"""
import functools

import numpy as np
import pytest

import oracle
from tests._inputs import full_size_multipoles, level_slices, multipoles, rel

pytestmark = pytest.mark.gpu

TOL_L = 1e-6
TOL_B = 1e-5


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1009_3457_amd as P
    return P


def _run(P, Ms32, depth, p, lmin=2, lmax=None, sentinel=None, with_b=True):
    import torch
    M = torch.from_numpy(Ms32).cuda()
    nb = Ms32.shape[0]
    L = torch.full((nb, p), complex(sentinel or 0.0), dtype=torch.complex64, device="cuda")
    b = torch.full((nb,), complex(sentinel or 0.0), dtype=torch.complex64, device="cuda") if with_b else None
    P.m2l_raw(M, depth, p, lmin, lmax, P.F64_HANKEL, L=L, b=b, with_b=with_b)
    torch.cuda.synchronize()
    return L.cpu().numpy(), None if b is None else b.cpu().numpy()


def _run_adj(P, gL32, gb32, depth, p, lmin=2, lmax=None):
    import torch
    gL = torch.from_numpy(gL32).cuda()
    gb = None if gb32 is None else torch.from_numpy(gb32).cuda()
    gM = P.m2l_backward(gL, gb, depth, p, lmin, lmax, P.F64_HANKEL)
    torch.cuda.synchronize()
    return gM.cpu().numpy()


def _worst_box(A, R):
    rms = np.sqrt(np.mean(np.sum(np.abs(R) ** 2, axis=1)))
    return np.max(np.linalg.norm(A - R, axis=1)) / rms


@pytest.mark.parametrize("p", [8, 12, 16, 20])
@pytest.mark.parametrize("depth", [2, 3, 5])
def test_hankel_matches_oracle_every_level(P, p, depth):
    print(f"m2l hankel p={p} depth={depth}", flush=True)
    Ms32, M_exact = multipoles(depth, p, 4 ** depth * 12, seed=p + depth)
    L, b = _run(P, Ms32, depth, p)
    Lr, br = oracle.m2l(M_exact, depth, p)
    Lr = oracle.scale_locals(Lr, depth)
    for l, sl in level_slices(depth):
        assert rel(L[sl], Lr[sl]) < TOL_L, (l, rel(L[sl], Lr[sl]))
        assert rel(b[sl], br[sl]) < TOL_B, (l, rel(b[sl], br[sl]))
        assert _worst_box(L[sl], Lr[sl]) < 10 * TOL_L


@pytest.mark.parametrize("p", [8, 20])
def test_hankel_every_coefficient(P, p):
    """Each coefficient n of L~ separately (the scalings (-1)^n rho^n / n!
    span many decades; a lost small term would show in the high orders)."""
    depth = 5
    Ms32, M_exact = multipoles(depth, p, 4 ** depth * 12, seed=90 + p, kind="mixed")
    L, _ = _run(P, Ms32, depth, p)
    Lr = oracle.scale_locals(oracle.m2l(M_exact, depth, p)[0], depth)
    lo = oracle.level_offset(2)
    for n in range(p):
        assert rel(L[lo:, n], Lr[lo:, n]) < 10 * TOL_L, (n, rel(L[lo:, n], Lr[lo:, n]))


def test_hankel_level_range_leaves_other_levels_untouched(P):
    depth, p = 5, 20
    Ms32, M_exact = multipoles(depth, p, 4 ** depth * 10, seed=3)
    L, b = _run(P, Ms32, depth, p, lmin=3, lmax=4, sentinel=7.0)
    Lr, br = oracle.m2l(M_exact, depth, p, 3, 4)
    Lr = oracle.scale_locals(Lr, depth)
    for l, sl in level_slices(depth, lmin=0):
        if 3 <= l <= 4:
            assert rel(L[sl], Lr[sl]) < TOL_L
            assert rel(b[sl], br[sl]) < TOL_B
        else:
            assert np.all(L[sl] == 7.0) and np.all(b[sl] == 7.0)


def test_hankel_without_b_leaves_l_unchanged(P):
    depth, p = 4, 12
    Ms32, _ = multipoles(depth, p, 4 ** depth * 10, seed=8)
    L1, _ = _run(P, Ms32, depth, p)
    L2, _ = _run(P, Ms32, depth, p, with_b=False)
    assert np.array_equal(L1.view(np.uint32), L2.view(np.uint32))


@functools.lru_cache(maxsize=1)
def _d7_p20():
    Ms32, M_exact = multipoles(7, 20, 1 << 18, seed=43, kind="mixed")
    Lr, br = oracle.m2l(M_exact, 7, 20)
    return Ms32, oracle.scale_locals(Lr, 7), br


def test_hankel_multitile_every_box(P):
    """Depth 7 (256 tiles at level 7: every workgroup takes several tiles in
    turn), p = 20, every box of every level."""
    print("m2l hankel depth=7 p=20 every box", flush=True)
    Ms32, Lr, br = _d7_p20()
    L, b = _run(P, Ms32, 7, 20)
    for l, sl in level_slices(7):
        assert rel(L[sl], Lr[sl]) < TOL_L, (l, rel(L[sl], Lr[sl]))
        assert rel(b[sl], br[sl]) < TOL_B, (l, rel(b[sl], br[sl]))
        assert _worst_box(L[sl], Lr[sl]) < 10 * TOL_L


def _sample_boxes(level, seed, extra=40):
    ns = 1 << level
    g = np.random.Generator(np.random.PCG64(seed + level))
    cand = [(0, 0), (ns - 1, ns - 1), (0, ns - 1), (ns - 1, 0), (1, ns // 2), (ns // 2, ns - 2),
            (2, 1), (ns - 3, ns - 2)]
    cand += [tuple(v) for v in g.integers(0, ns, size=(extra, 2))]
    return np.array(sorted({oracle.morton(int(x) % ns, int(y) % ns, level) for x, y in cand}), np.int64)


@pytest.mark.parametrize("depth,p,n", [(8, 12, 1 << 20), (10, 20, 1 << 24)])
def test_hankel_full_size_sampled(P, depth, p, n):
    """The benchmark workloads in the launch configuration the benchmark
    times, sampled target boxes of every level (corners and edges included)."""
    print(f"m2l hankel full size depth={depth} p={p}", flush=True)
    if depth == 8:
        Ms32, M_exact = multipoles(depth, p, n, seed=2, kind="uniform")
    else:
        Ms32, M_exact = full_size_multipoles(depth, p, n, "mixed")
    L, b = _run(P, Ms32, depth, p)
    for l, sl in level_slices(depth):
        boxes = _sample_boxes(l, 81)
        Lr, br = oracle.m2l_boxes(M_exact[sl], l, p, boxes)
        Lr_s = Lr * (2.0 ** -l) ** (np.arange(p) + 1.0)[None, :]
        assert rel(L[sl][boxes], Lr_s) < TOL_L, (l, rel(L[sl][boxes], Lr_s))
        assert rel(b[sl][boxes], br) < TOL_B


def test_hankel_is_deterministic(P):
    depth, p = 6, 20
    Ms32, _ = multipoles(depth, p, 4 ** depth * 16, seed=5)
    L1, b1 = _run(P, Ms32, depth, p)
    L2, b2 = _run(P, Ms32, depth, p)
    assert np.array_equal(L1.view(np.uint32), L2.view(np.uint32))
    assert np.array_equal(b1.view(np.uint32), b2.view(np.uint32))


# ------------------------------------------------------------ adjoint ---

def _cotangents(depth, p, seed, with_b):
    g = np.random.Generator(np.random.PCG64(seed))
    nb = oracle.num_boxes(depth)
    decay = 0.6 ** np.arange(p)
    gL32 = ((g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))) * decay).astype(np.complex64)
    gb32 = (g.standard_normal(nb) + 1j * g.standard_normal(nb)).astype(np.complex64) if with_b else None
    return gL32, gb32


@pytest.mark.parametrize("p", [8, 12, 16, 20])
@pytest.mark.parametrize("with_b", [True, False])
def test_hankel_backward_matches_oracle_transpose(P, p, with_b):
    print(f"m2l hankel backward p={p} with_b={with_b}", flush=True)
    depth = 5
    gL32, gb32 = _cotangents(depth, p, 200 + p, with_b)
    gM = _run_adj(P, gL32, gb32, depth, p)
    gL_un = oracle.scale_locals(gL32.astype(np.complex128), depth)
    gM_un = oracle.m2l_transpose(gL_un, None if gb32 is None else gb32.astype(np.complex128), depth, p)
    gM_ref = oracle.unscale_multipoles(gM_un, depth)
    for l, sl in level_slices(depth):
        assert rel(gM[sl], gM_ref[sl]) < (TOL_B if with_b else TOL_L), (l, rel(gM[sl], gM_ref[sl]))


@pytest.mark.parametrize("depth,p", [(8, 12), (9, 16), (10, 20)])
def test_hankel_adjoint_multitile_sampled(P, depth, p):
    """gM~ element by element on sampled source boxes of every level of a
    tree deep enough that every workgroup takes several tiles."""
    print(f"m2l hankel adjoint depth={depth} p={p}", flush=True)
    gL32, gb32 = _cotangents(depth, p, 300 + depth + p, True)
    gM = _run_adj(P, gL32, gb32, depth, p)
    k = np.arange(p)
    for l, sl in level_slices(depth):
        h = 2.0 ** -l
        boxes = _sample_boxes(l, 17)
        gL_un = gL32[sl].astype(np.complex128) * h ** (k + 1.0)
        ref = oracle.m2l_transpose_boxes(gL_un, gb32[sl].astype(np.complex128), l, p, boxes) * h ** k
        assert rel(gM[sl][boxes], ref) < TOL_B, (l, rel(gM[sl][boxes], ref))


def test_hankel_backward_level_range(P):
    """Sources outside lmin..lmax get gM~ = 0."""
    depth, p = 5, 12
    gL32, gb32 = _cotangents(depth, p, 77, True)
    gM = _run_adj(P, gL32, gb32, depth, p, lmin=3, lmax=4)
    for l, sl in level_slices(depth, lmin=0):
        if not 3 <= l <= 4:
            assert np.all(gM[sl] == 0), l


@pytest.mark.parametrize("depth,p", [(8, 12), (10, 20)])
def test_hankel_adjoint_dot_product_full_size(P, depth, p):
    """<M2L(M), G> = <M, M2L^T(G)> (bilinear) at benchmark sizes."""
    Ms32, _ = multipoles(depth, p, 4 ** depth * 16, seed=9)
    g = np.random.Generator(np.random.PCG64(9))
    nb = Ms32.shape[0]
    G32 = ((g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))) *
           0.5 ** np.arange(p)).astype(np.complex64)
    Gb32 = (g.standard_normal(nb) + 1j * g.standard_normal(nb)).astype(np.complex64)
    L, b = _run(P, Ms32, depth, p)
    gM = _run_adj(P, G32, Gb32, depth, p)
    lo = oracle.level_offset(2)
    lhs = np.sum(L[lo:].astype(np.complex128) * G32[lo:]) + np.sum(b[lo:].astype(np.complex128) * Gb32[lo:])
    rhs = np.sum(Ms32[lo:].astype(np.complex128) * gM[lo:])
    assert abs(lhs - rhs) < 1e-5 * (abs(lhs) + 1e-30)


# ------------------------------------------------- through the whole FMM ---

def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("n,depth,p", [(30000, 5, 20), (4096, 4, 12)])
def test_fmm_potential_hankel_matches_oracle(P, n, depth, p):
    import synthetic as sy
    print(f"fmm hankel n={n} depth={depth} p={p}", flush=True)
    xy = sy.mixed(n, 61)
    q = sy.charges(n, 62)
    t = sy.uniform(2048, 63)
    phi, f = P.potential(_t(xy), _t(q), _t(t), depth=depth, p=p, precision="f64_hankel")
    phir, fr = oracle.fmm(xy.astype(np.float64), q.astype(np.float64), t.astype(np.float64), depth, p)
    assert rel(phi.cpu().numpy().real, phir.real) < 1e-5
    assert rel(f.cpu().numpy(), fr) < 1e-5


def test_gradient_hankel_matches_oracle(P):
    import synthetic as sy
    n, depth, p = 4096, 4, 20
    xy = sy.uniform(n, 71)
    q = sy.charges(n, 72)
    t = sy.uniform(4096, 73)
    xg = _t(xy).requires_grad_(True)
    qg = _t(q).requires_grad_(True)
    phi, _ = P.potential(xg, qg, _t(t), depth=depth, p=p, precision="f64_hankel")
    (phi.real ** 2).sum().backward()
    phir, _ = oracle.fmm(xy.astype(np.float64), q.astype(np.float64), t.astype(np.float64), depth, p)
    gq_r, gxy_r = oracle.fmm_grad(xy.astype(np.float64), q.astype(np.float64), t.astype(np.float64), depth, p,
                                  (2 * phir.real).astype(np.complex128))
    assert rel(qg.grad.cpu().numpy(), gq_r) < 1e-5
    assert rel(xg.grad.cpu().numpy(), gxy_r) < 1e-5
