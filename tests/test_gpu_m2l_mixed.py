"""GPU parity of the split-precision M2L (BF16x3 and FP16x3 on MFMA, FP32
accumulation) and its adjoint against the FP64 oracle, through the C ABI.

The oracle translates exactly the FP32 inputs the GPU receives, with
Eq. (eq:M2Lmat) in FP64.  Tolerance after split-precision recovery: relative
Frobenius error per level <= 1e-4 on L~ and b (and on the adjoint's gM~).
"""
import numpy as np
import pytest

import oracle
from tests._inputs import full_size_multipoles, level_slices, multipoles, rel

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-4
PRECS = ["bf16x3", "f16x3"]


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1009_3457_amd as P
    return P


def _run(P, Ms32, depth, p, prec, lmin=2, lmax=None, sentinel=None):
    import torch
    M = torch.from_numpy(Ms32).cuda()
    nb = Ms32.shape[0]
    L = torch.full((nb, p), complex(sentinel or 0.0), dtype=torch.complex64, device="cuda")
    b = torch.full((nb,), complex(sentinel or 0.0), dtype=torch.complex64, device="cuda")
    P.m2l_raw(M, depth, p, lmin, lmax, P.PRECISIONS[prec], L=L, b=b)
    torch.cuda.synchronize()
    return L.cpu().numpy(), b.cpu().numpy()


def _run_adj(P, gL32, gb32, depth, p, prec):
    import torch
    gL = torch.from_numpy(gL32).cuda()
    gb = None if gb32 is None else torch.from_numpy(gb32).cuda()
    gM = P.m2l_backward(gL, gb, depth, p, 2, None, P.PRECISIONS[prec])
    torch.cuda.synchronize()
    return gM.cpu().numpy()


def _ref(M_exact, depth, p, lmin=2, lmax=None):
    L, b = oracle.m2l(M_exact, depth, p, lmin, lmax)
    return oracle.scale_locals(L, depth), b


def _ref_adj(gL32, gb32, depth, p):
    gL_un = oracle.scale_locals(gL32.astype(np.complex128), depth)
    gM_un = oracle.m2l_transpose(gL_un, None if gb32 is None else gb32.astype(np.complex128), depth, p)
    return oracle.unscale_multipoles(gM_un, depth)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("p", [8, 12, 16, 20])
@pytest.mark.parametrize("depth", [2, 3, 5])
def test_m2l_mixed_matches_oracle_every_level(P, prec, p, depth):
    """Levels 2 and 3 are smaller than one 16x16 tile; level 5 spans 4 tiles."""
    print(f"m2l {prec} depth={depth} p={p}", flush=True)
    Ms32, M_exact = multipoles(depth, p, 4 ** depth * 16, seed=20 + depth, kind="mixed")
    L, b = _run(P, Ms32, depth, p, prec)
    Lr, br = _ref(M_exact, depth, p)
    for l, sl in level_slices(depth):
        assert rel(L[sl], Lr[sl]) < TOL_MIXED, (l, rel(L[sl], Lr[sl]))
        assert rel(b[sl], br[sl]) < TOL_MIXED, (l, rel(b[sl], br[sl]))


@pytest.mark.parametrize("prec", PRECS)
def test_m2l_mixed_level_range_leaves_other_levels_untouched(P, prec):
    depth, p = 6, 16
    Ms32, M_exact = multipoles(depth, p, 4 ** depth * 8, seed=4)
    L, b = _run(P, Ms32, depth, p, prec, lmin=3, lmax=5, sentinel=7.0)
    Lr, br = _ref(M_exact, depth, p, 3, 5)
    for l, sl in level_slices(depth):
        if 3 <= l <= 5:
            assert rel(L[sl], Lr[sl]) < TOL_MIXED
            assert rel(b[sl], br[sl]) < TOL_MIXED
        else:
            assert np.all(L[sl] == 7.0) and np.all(b[sl] == 7.0)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("scale", [2.0 ** 60, 2.0 ** -60, 3.0e4])
def test_m2l_mixed_is_scale_equivariant(P, prec, scale):
    """M2L is linear: inputs far outside FP16's range (and large enough to
    overflow it) still give the scaled result, via the per-tile exponent."""
    depth, p = 5, 16
    Ms32, M_exact = multipoles(depth, p, 4 ** depth * 16, seed=31)
    Ms = (Ms32.astype(np.complex128) * scale).astype(np.complex64)
    L, b = _run(P, Ms, depth, p, prec)
    Lr, br = _ref(oracle.unscale_multipoles(Ms.astype(np.complex128), depth), depth, p)
    for l, sl in level_slices(depth):
        assert rel(L[sl], Lr[sl]) < TOL_MIXED, (l, rel(L[sl], Lr[sl]))
        assert rel(b[sl], br[sl]) < TOL_MIXED


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("depth,p,n", [(9, 16, 1 << 22), (10, 20, 1 << 24), (9, 12, 1 << 22)])
def test_m2l_mixed_full_size_sampled(P, prec, depth, p, n):
    """The 2^22-point depth-9 p = 16 and 2^24-point depth-10 p = 20 workloads
    (half clustered, half uniform) in the benchmark's launch configuration,
    checked on sampled target boxes of every level, boundary boxes included.
    These sizes give every workgroup several tiles (operator prefetch carried
    from tile to tile)."""
    print(f"m2l {prec} full size depth={depth} p={p}", flush=True)
    Ms32, M_exact = full_size_multipoles(depth, p, n, "mixed")
    L, b = _run(P, Ms32, depth, p, prec)
    g = np.random.Generator(np.random.PCG64(78))
    for l, sl in level_slices(depth):
        ns = 1 << l
        cand = [(0, 0), (ns - 1, ns - 1), (0, ns - 1), (ns - 1, 0), (1, ns // 2), (ns // 2, ns - 2)]
        cand += [tuple(v) for v in g.integers(0, ns, size=(60, 2))]
        boxes = np.array(sorted({oracle.morton(int(x), int(y), l) for x, y in cand}), np.int64)
        Lr, br = oracle.m2l_boxes(M_exact[sl], l, p, boxes)
        Lr_s = Lr * (2.0 ** -l) ** (np.arange(p) + 1.0)[None, :]
        assert rel(L[sl][boxes], Lr_s) < TOL_MIXED, (l, rel(L[sl][boxes], Lr_s))
        assert rel(b[sl][boxes], br) < TOL_MIXED


@pytest.mark.parametrize("prec", PRECS)
def test_m2l_mixed_is_deterministic(P, prec):
    depth, p = 6, 16
    Ms32, _ = multipoles(depth, p, 4 ** depth * 16, seed=6)
    L1, b1 = _run(P, Ms32, depth, p, prec)
    L2, b2 = _run(P, Ms32, depth, p, prec)
    assert np.array_equal(L1.view(np.uint32), L2.view(np.uint32))
    assert np.array_equal(b1.view(np.uint32), b2.view(np.uint32))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("p", [8, 12, 16, 20])
@pytest.mark.parametrize("with_b", [True, False])
def test_m2l_mixed_backward_matches_oracle_transpose(P, prec, p, with_b):
    print(f"m2l_backward {prec} p={p} with_b={with_b}", flush=True)
    depth = 5
    g = np.random.Generator(np.random.PCG64(200 + p))
    nb = oracle.num_boxes(depth)
    decay = 0.6 ** np.arange(p)
    gL32 = ((g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))) * decay).astype(np.complex64)
    gb32 = (g.standard_normal(nb) + 1j * g.standard_normal(nb)).astype(np.complex64) if with_b else None
    gM = _run_adj(P, gL32, gb32, depth, p, prec)
    gM_ref = _ref_adj(gL32, gb32, depth, p)
    for l, sl in level_slices(depth):
        assert rel(gM[sl], gM_ref[sl]) < TOL_MIXED, (l, rel(gM[sl], gM_ref[sl]))


@pytest.mark.parametrize("prec", PRECS)
def test_m2l_mixed_adjoint_dot_product_full_size(P, prec):
    """<M2L(M), G> = <M, M2L^T(G)> (bilinear) at the 2^22-point depth-9
    p = 16 size, each side computed in split precision."""
    depth, p = 9, 16
    Ms32, _ = multipoles(depth, p, 1 << 22, seed=9, kind="mixed")
    g = np.random.Generator(np.random.PCG64(9))
    nb = Ms32.shape[0]
    G32 = ((g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))) *
           0.5 ** np.arange(p)).astype(np.complex64)
    Gb32 = (g.standard_normal(nb) + 1j * g.standard_normal(nb)).astype(np.complex64)
    L, b = _run(P, Ms32, depth, p, prec)
    gM = _run_adj(P, G32, Gb32, depth, p, prec)
    lo = oracle.level_offset(2)
    lhs = np.sum(L[lo:].astype(np.complex128) * G32[lo:]) + np.sum(b[lo:].astype(np.complex128) * Gb32[lo:])
    rhs = np.sum(Ms32[lo:].astype(np.complex128) * gM[lo:])
    assert abs(lhs - rhs) < 1e-4 * (abs(lhs) + 1e-30)
