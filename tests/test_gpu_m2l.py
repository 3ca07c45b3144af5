"""GPU parity of the M2L contraction and its adjoint against the FP64 oracle,
through the C ABI (via the thin torch binding).  Inputs are the oracle's
multipole expansions of seeded point sets, rounded to FP32; the oracle then
translates exactly those rounded values with Eq. (eq:M2Lmat).

Tolerance (FP32): relative Frobenius error per level <= 1e-5 on L~ and b.
"""
import numpy as np
import pytest

import oracle
from tests._inputs import full_size_multipoles, level_slices, multipoles, rel

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1009_3457_amd as P
    return P


def _run_m2l(P, Ms32, depth, p, lmin=2, lmax=None, sentinel=None):
    import torch
    M = torch.from_numpy(Ms32).cuda()
    nb = Ms32.shape[0]
    L = torch.full((nb, p), complex(sentinel or 0.0), dtype=torch.complex64, device="cuda")
    b = torch.full((nb,), complex(sentinel or 0.0), dtype=torch.complex64, device="cuda")
    P.m2l_raw(M, depth, p, lmin, lmax, P.F32, L=L, b=b)
    torch.cuda.synchronize()
    return L.cpu().numpy(), b.cpu().numpy()


def _ref(M_exact, depth, p, lmin=2, lmax=None):
    L, b = oracle.m2l(M_exact, depth, p, lmin, lmax)
    return oracle.scale_locals(L, depth), b


@pytest.mark.parametrize("p", [8, 12, 16, 20])
@pytest.mark.parametrize("depth", [2, 3, 5])
def test_m2l_f32_matches_oracle_every_level(P, p, depth):
    print(f"m2l f32 depth={depth} p={p}", flush=True)
    Ms32, M_exact = multipoles(depth, p, 4 ** depth * 16, seed=10 + depth)
    L, b = _run_m2l(P, Ms32, depth, p)
    Lr, br = _ref(M_exact, depth, p)
    for l, sl in level_slices(depth):
        assert rel(L[sl], Lr[sl]) < TOL_F32, (l, rel(L[sl], Lr[sl]))
        assert rel(b[sl], br[sl]) < TOL_F32, (l, rel(b[sl], br[sl]))


def test_m2l_level_range_leaves_other_levels_untouched(P):
    depth, p = 5, 12
    Ms32, M_exact = multipoles(depth, p, 4 ** depth * 8, seed=3)
    L, b = _run_m2l(P, Ms32, depth, p, lmin=3, lmax=4, sentinel=7.0)
    Lr, br = _ref(M_exact, depth, p, 3, 4)
    for l, sl in level_slices(depth):
        if 3 <= l <= 4:
            assert rel(L[sl], Lr[sl]) < TOL_F32
            assert rel(b[sl], br[sl]) < TOL_F32
        else:
            assert np.all(L[sl] == 7.0) and np.all(b[sl] == 7.0)
    lo = oracle.level_offset(2)
    assert np.all(L[:lo] == 7.0)


def test_m2l_single_source_closed_form(P):
    """One unit multipole M~_0 = 1 in one box: every box of its list receives
    column 0 of Eq. (eq:M2Lmat), L~_n = (-1)^n d^-(n+1) (d in box widths)."""
    import torch
    depth, p = 4, 12
    nb = oracle.num_boxes(depth)
    M = np.zeros((nb, p), np.complex64)
    l, sx, sy = 4, 6, 9
    s = oracle.level_offset(l) + oracle.morton(sx, sy, l)
    M[s, 0] = 1.0
    L, b = _run_m2l(P, M, depth, p)
    hits = 0
    for tx in range(16):
        for ty in range(16):
            t = oracle.level_offset(l) + oracle.morton(tx, ty, l)
            lst = oracle.interaction_list(l, tx, ty)
            if oracle.morton(sx, sy, l) in lst:
                d = complex(tx - sx, ty - sy)
                n = np.arange(p)
                expect = ((-1.0) ** n) * d ** (-(n + 1.0))
                assert np.allclose(L[t], expect, rtol=2e-6, atol=1e-9)
                assert np.isclose(b[t], np.log(d) + np.log(2.0 ** -l), rtol=2e-6)
                hits += 1
            else:
                assert np.all(L[t] == 0)
    assert hits == 27


@pytest.mark.parametrize("kind", ["uniform", "mixed"])
def test_m2l_f32_full_size_c2_sampled(P, kind):
    """N = 2^20, depth 8, p = 12 (the benchmark workload) in the same launch
    configuration as the benchmark; checked on sampled target boxes of every
    level, boundary boxes included."""
    print(f"m2l f32 C2 sampled kind={kind}", flush=True)
    depth, p = 8, 12
    Ms32, M_exact = multipoles(depth, p, 1 << 20, seed=2, kind=kind)
    L, b = _run_m2l(P, Ms32, depth, p)
    g = np.random.Generator(np.random.PCG64(77))
    for l, sl in level_slices(depth):
        ns = 1 << l
        cand = [(0, 0), (ns - 1, ns - 1), (0, ns - 1), (ns - 1, 0), (1, ns // 2), (ns // 2, ns - 2)]
        cand += [tuple(v) for v in g.integers(0, ns, size=(60, 2))]
        boxes = np.array(sorted({oracle.morton(int(x), int(y), l) for x, y in cand}), np.int64)
        Lr, br = oracle.m2l_boxes(M_exact[sl], l, p, boxes)
        h = 2.0 ** -l
        Lr_s = Lr * h ** (np.arange(p) + 1.0)[None, :]
        got = L[sl][boxes]
        assert rel(got, Lr_s) < TOL_F32, (l, rel(got, Lr_s))
        assert rel(b[sl][boxes], br) < TOL_F32


@pytest.mark.parametrize("depth,p,n", [(9, 16, 1 << 22), (10, 20, 1 << 24)])
def test_m2l_f32_full_size_sampled_large(P, depth, p, n):
    """The 2^22-point depth-9 p = 16 and 2^24-point depth-10 p = 20 workloads
    (half clustered, half uniform) in FP32, sampled boxes of every level."""
    print(f"m2l f32 full size depth={depth} p={p}", flush=True)
    Ms32, M_exact = full_size_multipoles(depth, p, n, "mixed")
    L, b = _run_m2l(P, Ms32, depth, p)
    g = np.random.Generator(np.random.PCG64(79))
    for l, sl in level_slices(depth):
        ns = 1 << l
        cand = [(0, 0), (ns - 1, ns - 1), (0, ns - 1), (ns - 1, 0), (2, ns // 2), (ns // 2, ns - 3)]
        cand += [tuple(v) for v in g.integers(0, ns, size=(40, 2))]
        boxes = np.array(sorted({oracle.morton(int(x), int(y), l) for x, y in cand}), np.int64)
        Lr, br = oracle.m2l_boxes(M_exact[sl], l, p, boxes)
        Lr_s = Lr * (2.0 ** -l) ** (np.arange(p) + 1.0)[None, :]
        assert rel(L[sl][boxes], Lr_s) < TOL_F32, (l, rel(L[sl][boxes], Lr_s))
        assert rel(b[sl][boxes], br) < TOL_F32


def test_m2l_is_deterministic(P):
    depth, p = 6, 12
    Ms32, _ = multipoles(depth, p, 4 ** depth * 16, seed=5)
    L1, b1 = _run_m2l(P, Ms32, depth, p)
    L2, b2 = _run_m2l(P, Ms32, depth, p)
    assert np.array_equal(L1.view(np.uint32), L2.view(np.uint32))
    assert np.array_equal(b1.view(np.uint32), b2.view(np.uint32))


# --------------------------------------------------------------- adjoint ---

def _run_adj(P, gL32, gb32, depth, p, lmin=2, lmax=None):
    import torch
    gL = torch.from_numpy(gL32).cuda()
    gb = None if gb32 is None else torch.from_numpy(gb32).cuda()
    gM = P.m2l_backward(gL, gb, depth, p, lmin, lmax, P.F32)
    torch.cuda.synchronize()
    return gM.cpu().numpy()


@pytest.mark.parametrize("p", [8, 12, 16, 20])
@pytest.mark.parametrize("with_b", [True, False])
def test_m2l_backward_matches_oracle_transpose(P, p, with_b):
    print(f"m2l_backward p={p} with_b={with_b}", flush=True)
    depth = 5
    g = np.random.Generator(np.random.PCG64(100 + p))
    nb = oracle.num_boxes(depth)
    decay = 0.6 ** np.arange(p)
    gL32 = ((g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))) * decay).astype(np.complex64)
    gb32 = (g.standard_normal(nb) + 1j * g.standard_normal(nb)).astype(np.complex64) if with_b else None
    gM = _run_adj(P, gL32, gb32, depth, p)
    # the transpose in the scaled basis is the unscaled transpose conjugated by
    # the (exact, diagonal) scalings: gM~ = S_M^-1 A^T S_L^-1 ... written out:
    gL_un = oracle.scale_locals(gL32.astype(np.complex128), depth)  # gL~ h^(n+1)
    gM_un = oracle.m2l_transpose(gL_un, None if gb32 is None else gb32.astype(np.complex128), depth, p)
    gM_ref = oracle.unscale_multipoles(gM_un, depth)  # h^k gM
    for l, sl in level_slices(depth):
        assert rel(gM[sl], gM_ref[sl]) < TOL_F32, (l, rel(gM[sl], gM_ref[sl]))


def test_m2l_adjoint_dot_product_full_size(P):
    """<M2L(M), G> = <M, M2L^T(G)> (bilinear) at the benchmark size."""
    import torch
    depth, p = 8, 12
    Ms32, _ = multipoles(depth, p, 1 << 20, seed=9)
    g = np.random.Generator(np.random.PCG64(9))
    nb = Ms32.shape[0]
    G32 = ((g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))) *
           0.5 ** np.arange(p)).astype(np.complex64)
    Gb32 = (g.standard_normal(nb) + 1j * g.standard_normal(nb)).astype(np.complex64)
    L, b = _run_m2l(P, Ms32, depth, p)
    gM = _run_adj(P, G32, Gb32, depth, p)
    lo = oracle.level_offset(2)
    lhs = np.sum(L[lo:].astype(np.complex128) * G32[lo:]) + np.sum(b[lo:].astype(np.complex128) * Gb32[lo:])
    rhs = np.sum(Ms32[lo:].astype(np.complex128) * gM[lo:])
    assert abs(lhs - rhs) < 1e-5 * (abs(lhs) + 1e-30)
