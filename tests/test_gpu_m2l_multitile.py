"""GPU parity of every M2L form where each workgroup of the persistent kernels
takes several tiles in turn, so the fetch of the next tile's source block
(and, in the adjoint, of its cotangents) is exercised, against the FP64
oracle through the C ABI:

  * the adjoint (plain transpose of Eq. (eq:M2Lmat) plus the log row), element
    by element on sampled source boxes of every level, at depths 8-10;
  * the forward map at p = 8 on a depth-9 tree, every box of every level;
  * the 2^20-point, depth-8, p = 12 workload (the benchmark's), every box of
    every level, in all four precisions.

The split-precision kernel runs self-staging workgroups (two per compute
unit) for the adjoint at every size and for the forward map below two tiles
per compute unit: the depth-8 forward case takes one tile per workgroup, the
depth-9 and 10 adjoint cases several tiles per self-staging workgroup, and the
depth-9 forward case the loader-backed workgroups.

Tolerances (relative Frobenius error per level): FP32 forms 1e-5, split
precision 1e-4.
"""
import functools

import numpy as np
import pytest

import oracle
from tests._inputs import level_slices, multipoles, rel

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f32_pascal": 1e-5, "bf16x3": 1e-4, "f16x3": 1e-4}


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1009_3457_amd as P
    return P


def _fwd(P, Ms32, depth, p, prec):
    import torch
    M = torch.from_numpy(Ms32).cuda()
    L, b = P.m2l_raw(M, depth, p, 2, depth, P.PRECISIONS[prec])
    torch.cuda.synchronize()
    return L.cpu().numpy(), b.cpu().numpy()


def _adj(P, gL32, gb32, depth, p, prec):
    import torch
    gL = torch.from_numpy(gL32).cuda()
    gb = None if gb32 is None else torch.from_numpy(gb32).cuda()
    gM = P.m2l_backward(gL, gb, depth, p, 2, None, P.PRECISIONS[prec])
    torch.cuda.synchronize()
    return gM.cpu().numpy()


def _sample_boxes(level, seed, extra=40):
    """Corners, edge boxes and seeded random boxes of one level (Morton)."""
    ns = 1 << level
    g = np.random.Generator(np.random.PCG64(seed + level))
    cand = [(0, 0), (ns - 1, ns - 1), (0, ns - 1), (ns - 1, 0), (1, ns // 2), (ns // 2, ns - 2),
            (2, 1), (ns - 3, ns - 2)]
    cand += [tuple(v) for v in g.integers(0, ns, size=(extra, 2))]
    return np.array(sorted({oracle.morton(int(x) % ns, int(y) % ns, level) for x, y in cand}), np.int64)


@functools.lru_cache(maxsize=2)
def _cotangents(depth, p, seed):
    """Seeded cotangents of L~ (decaying in the order, as the L2L transpose
    gives them) and of b."""
    g = np.random.Generator(np.random.PCG64(seed))
    nb = oracle.num_boxes(depth)
    decay = 0.6 ** np.arange(p)
    gL = ((g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))) * decay).astype(np.complex64)
    gb = (g.standard_normal(nb) + 1j * g.standard_normal(nb)).astype(np.complex64)
    return gL, gb


# ---------------------------------------------------- adjoint, multi-tile ---

ADJ_CASES = [
    ("f32_pascal", 8, 12, True), ("f32_pascal", 8, 12, False), ("f32_pascal", 9, 16, True),
    ("f32_pascal", 10, 20, True), ("f32_pascal", 9, 8, True),
    ("bf16x3", 9, 12, True), ("bf16x3", 9, 16, True), ("bf16x3", 10, 20, True), ("bf16x3", 9, 8, True),
    ("f16x3", 9, 12, True), ("f16x3", 9, 16, True), ("f16x3", 10, 20, True), ("f16x3", 9, 8, True),
    ("f32", 9, 16, True), ("f32", 10, 20, True), ("f32", 9, 8, True), ("f32", 8, 12, True),
]


@pytest.mark.parametrize("prec,depth,p,with_b", ADJ_CASES)
def test_adjoint_multitile_matches_oracle(P, prec, depth, p, with_b):
    """gM~ = A~^T gL~ (+ the log row's transpose times gb) on sampled source
    boxes of every level; the oracle gathers over each source's own list in
    the unscaled basis (gL = gL~ h^(n+1) in, gM~ = gM h^k out)."""
    print(f"adjoint multitile {prec} depth={depth} p={p} with_b={with_b}", flush=True)
    gL32, gb32 = _cotangents(depth, p, 300 + depth + p)
    gb32 = gb32 if with_b else None
    gM = _adj(P, gL32, gb32, depth, p, prec)
    k = np.arange(p)
    for l, sl in level_slices(depth):
        h = 2.0 ** -l
        boxes = _sample_boxes(l, 17)
        gL_un = gL32[sl].astype(np.complex128) * h ** (k + 1.0)
        ref = oracle.m2l_transpose_boxes(gL_un, None if gb32 is None else gb32[sl].astype(np.complex128),
                                         l, p, boxes) * h ** k
        err = rel(gM[sl][boxes], ref)
        assert err < TOL[prec], (l, err)


# ----------------------------------------------- forward, p = 8 multi-tile ---

@functools.lru_cache(maxsize=1)
def _d9_p8():
    Ms32, M_exact = multipoles(9, 8, 1 << 20, seed=41, kind="mixed")
    Lr, br = oracle.m2l(M_exact, 9, 8)
    return Ms32, oracle.scale_locals(Lr, 9), br


@pytest.mark.parametrize("prec", ["f32", "f32_pascal", "bf16x3", "f16x3"])
def test_forward_p8_multitile_every_box(P, prec):
    print(f"forward p=8 depth=9 {prec}", flush=True)
    Ms32, Lr, br = _d9_p8()
    L, b = _fwd(P, Ms32, 9, 8, prec)
    for l, sl in level_slices(9):
        assert rel(L[sl], Lr[sl]) < TOL[prec], (l, rel(L[sl], Lr[sl]))
        assert rel(b[sl], br[sl]) < TOL[prec], (l, rel(b[sl], br[sl]))


# ------------------------------------- the benchmark workload, every box ---

@functools.lru_cache(maxsize=1)
def _c2():
    Ms32, M_exact = multipoles(8, 12, 1 << 20, seed=2, kind="uniform")
    Lr, br = oracle.m2l(M_exact, 8, 12)
    return Ms32, oracle.scale_locals(Lr, 8), br


@pytest.mark.parametrize("prec", ["f32_pascal", "f32", "bf16x3", "f16x3"])
def test_c2_every_box_every_level(P, prec):
    """2^20 uniform points, depth 8, p = 12, L~ and b: all 87,376 boxes of
    levels 2..8 against the oracle's full M2L (2,316,900 translations)."""
    print(f"c2 every box {prec}", flush=True)
    Ms32, Lr, br = _c2()
    L, b = _fwd(P, Ms32, 8, 12, prec)
    for l, sl in level_slices(8):
        assert rel(L[sl], Lr[sl]) < TOL[prec], (l, rel(L[sl], Lr[sl]))
        assert rel(b[sl], br[sl]) < TOL[prec], (l, rel(b[sl], br[sl]))
        # no single box is far off: its error against the level's RMS box norm
        rms = np.sqrt(np.mean(np.sum(np.abs(Lr[sl]) ** 2, axis=1)))
        worst = np.max(np.linalg.norm(L[sl] - Lr[sl], axis=1))
        assert worst < 10 * TOL[prec] * rms, (l, worst / rms)
