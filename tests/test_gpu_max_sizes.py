"""The library's largest tree (depth 12: 22,369,621 boxes, 262,144 tiles at
the deepest level) through the C ABI: the M2L forward and adjoint in the
FP32 Pascal form and in BF16x3 against the FP64 oracle on sampled boxes of
shallow and deep levels, and the tree build bit for bit.  Expansions are
seeded random values decaying in the order, as M2M and L2L produce them.

Tolerances (relative Frobenius error over the sampled boxes of a level):
FP32 1e-5, split precision 1e-4."""
import functools

import numpy as np
import pytest

import oracle
import synthetic as sy
from tests._inputs import rel

pytestmark = pytest.mark.gpu

DEPTH, P_ORDER = 12, 8
LEVELS = [2, 3, 7, 11, 12]
TOL = {"f32_pascal": 1e-5, "bf16x3": 1e-4}


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1009_3457_amd as P
    return P


@functools.lru_cache(maxsize=1)
def _random_expansions(seed):
    """Scaled expansions (complex64) of every box of the depth-12 tree, the
    coefficient of order k scaled by 0.6^k, and one complex value per box."""
    g = np.random.Generator(np.random.PCG64(seed))
    nb = oracle.num_boxes(DEPTH)
    decay = (0.6 ** np.arange(P_ORDER)).astype(np.float32)
    X = np.empty((nb, P_ORDER), np.complex64)
    X.real = g.standard_normal((nb, P_ORDER), dtype=np.float32) * decay
    X.imag = g.standard_normal((nb, P_ORDER), dtype=np.float32) * decay
    y = np.empty(nb, np.complex64)
    y.real = g.standard_normal(nb, dtype=np.float32)
    y.imag = g.standard_normal(nb, dtype=np.float32)
    return X, y


def _sample_boxes(level, seed, extra=32):
    ns = 1 << level
    g = np.random.Generator(np.random.PCG64(seed + level))
    cand = [(0, 0), (ns - 1, ns - 1), (0, ns - 1), (ns - 1, 0), (1, ns // 2), (ns // 2, ns - 2), (2, 1)]
    cand += [tuple(v) for v in g.integers(0, ns, size=(extra, 2))]
    return np.array(sorted({oracle.morton(int(x) % ns, int(y) % ns, level) for x, y in cand}), np.int64)


def _level(l):
    return slice(oracle.level_offset(l), oracle.level_offset(l + 1))


@pytest.mark.parametrize("prec", ["f32_pascal", "bf16x3"])
def test_m2l_forward_at_depth_12(P, prec):
    import torch
    print(f"m2l depth 12 p=8 forward {prec}", flush=True)
    Ms32, _ = _random_expansions(121)
    M = torch.from_numpy(Ms32).cuda()
    L, b = P.m2l_raw(M, DEPTH, P_ORDER, 2, DEPTH, P.PRECISIONS[prec])
    torch.cuda.synchronize()
    del M
    k = np.arange(P_ORDER)
    for l in LEVELS:
        sl = _level(l)
        h = 2.0 ** -l
        boxes = _sample_boxes(l, 7)
        M_un = Ms32[sl].astype(np.complex128) * h ** k  # unscaled: M_k = M~_k h^k
        Lr, br = oracle.m2l_boxes(M_un, l, P_ORDER, boxes)
        Lr_s = Lr * h ** (k + 1.0)
        got = L[sl][torch.from_numpy(boxes).cuda()].cpu().numpy()
        gotb = b[sl][torch.from_numpy(boxes).cuda()].cpu().numpy()
        assert rel(got, Lr_s) < TOL[prec], (l, rel(got, Lr_s))
        assert rel(gotb, br) < TOL[prec], (l, rel(gotb, br))


@pytest.mark.parametrize("prec", ["f32_pascal", "bf16x3"])
def test_m2l_adjoint_at_depth_12(P, prec):
    import torch
    print(f"m2l depth 12 p=8 adjoint {prec}", flush=True)
    gL32, gb32 = _random_expansions(122)
    gM = P.m2l_backward(torch.from_numpy(gL32).cuda(), torch.from_numpy(gb32).cuda(), DEPTH, P_ORDER, 2, None,
                        P.PRECISIONS[prec])
    torch.cuda.synchronize()
    k = np.arange(P_ORDER)
    for l in LEVELS:
        sl = _level(l)
        h = 2.0 ** -l
        boxes = _sample_boxes(l, 9)
        gL_un = gL32[sl].astype(np.complex128) * h ** (k + 1.0)
        ref = oracle.m2l_transpose_boxes(gL_un, gb32[sl].astype(np.complex128), l, P_ORDER, boxes) * h ** k
        got = gM[sl][torch.from_numpy(boxes).cuda()].cpu().numpy()
        assert rel(got, ref) < TOL[prec], (l, rel(got, ref))


def test_build_tree_at_depth_12_bit_exact(P):
    import torch
    print("build_tree n=2^22 depth=12", flush=True)
    xy = sy.mixed(1 << 22, 13)
    perm, ls = P.build_tree(torch.from_numpy(xy).cuda(), DEPTH)
    perm_r, ls_r = oracle.build_tree(xy.astype(np.float64), DEPTH)
    assert np.array_equal(perm.cpu().numpy(), perm_r)
    assert np.array_equal(ls.cpu().numpy(), ls_r)
