"""GPU parity of the Pascal-form FP32 M2L (precision FMM2D_F32_PASCAL:
A~(d) = diag((-1)^n d^-(n+1)) B diag(d^-k), B[n][k] = C(n+k, k)) and of its
adjoint against the FP64 oracle, through the C ABI.  Same inputs and the same
tolerance as the Gauss-form FP32 kernel: relative Frobenius error per level
<= 1e-5 on L~ and b (the factorisation is exact; each factor is rounded once
to FP32 and the products accumulate in FP32)."""
import numpy as np
import pytest

import oracle
from tests._inputs import full_size_multipoles, level_slices, multipoles, rel

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1009_3457_amd as P
    return P


def _run(P, Ms32, depth, p, lmin=2, lmax=None, sentinel=None, prec=None):
    import torch
    M = torch.from_numpy(Ms32).cuda()
    nb = Ms32.shape[0]
    L = torch.full((nb, p), complex(sentinel or 0.0), dtype=torch.complex64, device="cuda")
    b = torch.full((nb,), complex(sentinel or 0.0), dtype=torch.complex64, device="cuda")
    P.m2l_raw(M, depth, p, lmin, lmax, P.F32_PASCAL if prec is None else prec, L=L, b=b)
    torch.cuda.synchronize()
    return L.cpu().numpy(), b.cpu().numpy()


def _run_adj(P, gL32, gb32, depth, p):
    import torch
    gL = torch.from_numpy(gL32).cuda()
    gb = None if gb32 is None else torch.from_numpy(gb32).cuda()
    gM = P.m2l_backward(gL, gb, depth, p, 2, None, P.F32_PASCAL)
    torch.cuda.synchronize()
    return gM.cpu().numpy()


@pytest.mark.parametrize("p", [8, 12, 16, 20])
@pytest.mark.parametrize("depth", [2, 3, 5])
def test_pascal_matches_oracle_every_level(P, p, depth):
    print(f"m2l pascal p={p} depth={depth}", flush=True)
    Ms32, M_exact = multipoles(depth, p, 4 ** depth * 12, seed=p + depth)
    L, b = _run(P, Ms32, depth, p)
    Lr, br = oracle.m2l(M_exact, depth, p)
    Lr = oracle.scale_locals(Lr, depth)
    for l, sl in level_slices(depth):
        assert rel(L[sl], Lr[sl]) < TOL, (l, rel(L[sl], Lr[sl]))
        assert rel(b[sl], br[sl]) < TOL, (l, rel(b[sl], br[sl]))


@pytest.mark.parametrize("p", [12, 16])  # b in spare MFMA rows; b formed in the loop
def test_pascal_level_range_leaves_other_levels_untouched(P, p):
    depth = 5
    Ms32, M_exact = multipoles(depth, p, 4 ** depth * 10, seed=3)
    L, b = _run(P, Ms32, depth, p, lmin=3, lmax=4, sentinel=7.0)
    Lr, br = oracle.m2l(M_exact, depth, p, 3, 4)
    Lr = oracle.scale_locals(Lr, depth)
    for l, sl in level_slices(depth, lmin=0):
        if 3 <= l <= 4:
            assert rel(L[sl], Lr[sl]) < TOL
            assert rel(b[sl], br[sl]) < TOL
        else:
            assert np.all(L[sl] == 7.0) and np.all(b[sl] == 7.0)


@pytest.mark.parametrize("depth,p,n", [(8, 12, 1 << 20), (9, 16, 1 << 22), (10, 20, 1 << 24)])
def test_pascal_full_size_sampled(P, depth, p, n):
    """The benchmark workloads in the launch configuration the benchmark
    times, sampled target boxes of every level (corners and edges included)."""
    print(f"m2l pascal full size depth={depth} p={p}", flush=True)
    if depth == 8:
        Ms32, M_exact = multipoles(depth, p, n, seed=2, kind="uniform")
    else:
        Ms32, M_exact = full_size_multipoles(depth, p, n, "mixed")
    L, b = _run(P, Ms32, depth, p)
    g = np.random.Generator(np.random.PCG64(81))
    for l, sl in level_slices(depth):
        ns = 1 << l
        cand = [(0, 0), (ns - 1, ns - 1), (0, ns - 1), (ns - 1, 0), (1, ns // 2), (ns // 2, ns - 2)]
        cand += [tuple(v) for v in g.integers(0, ns, size=(40, 2))]
        boxes = np.array(sorted({oracle.morton(int(x), int(y), l) for x, y in cand}), np.int64)
        Lr, br = oracle.m2l_boxes(M_exact[sl], l, p, boxes)
        Lr_s = Lr * (2.0 ** -l) ** (np.arange(p) + 1.0)[None, :]
        assert rel(L[sl][boxes], Lr_s) < TOL, (l, rel(L[sl][boxes], Lr_s))
        assert rel(b[sl][boxes], br) < TOL


def test_pascal_agrees_with_gauss_form(P):
    """Both FP32 forms of the same translation, on the same inputs."""
    depth, p = 6, 12
    Ms32, _ = multipoles(depth, p, 4 ** depth * 16, seed=11)
    L1, b1 = _run(P, Ms32, depth, p)
    L2, b2 = _run(P, Ms32, depth, p, prec=P.F32)
    lo = oracle.level_offset(2)
    assert rel(L1[lo:], L2[lo:]) < 2 * TOL
    assert rel(b1[lo:], b2[lo:]) < 2 * TOL


def test_pascal_is_deterministic(P):
    depth, p = 6, 20
    Ms32, _ = multipoles(depth, p, 4 ** depth * 16, seed=5)
    L1, b1 = _run(P, Ms32, depth, p)
    L2, b2 = _run(P, Ms32, depth, p)
    assert np.array_equal(L1.view(np.uint32), L2.view(np.uint32))
    assert np.array_equal(b1.view(np.uint32), b2.view(np.uint32))


@pytest.mark.parametrize("p", [8, 12, 16, 20])
@pytest.mark.parametrize("with_b", [True, False])
def test_pascal_backward_matches_oracle_transpose(P, p, with_b):
    print(f"m2l pascal backward p={p} with_b={with_b}", flush=True)
    depth = 5
    g = np.random.Generator(np.random.PCG64(200 + p))
    nb = oracle.num_boxes(depth)
    decay = 0.6 ** np.arange(p)
    gL32 = ((g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))) * decay).astype(np.complex64)
    gb32 = (g.standard_normal(nb) + 1j * g.standard_normal(nb)).astype(np.complex64) if with_b else None
    gM = _run_adj(P, gL32, gb32, depth, p)
    gL_un = oracle.scale_locals(gL32.astype(np.complex128), depth)
    gM_un = oracle.m2l_transpose(gL_un, None if gb32 is None else gb32.astype(np.complex128), depth, p)
    gM_ref = oracle.unscale_multipoles(gM_un, depth)
    for l, sl in level_slices(depth):
        assert rel(gM[sl], gM_ref[sl]) < TOL, (l, rel(gM[sl], gM_ref[sl]))


@pytest.mark.parametrize("depth,p", [(8, 12), (9, 16)])
def test_pascal_adjoint_dot_product_full_size(P, depth, p):
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


@pytest.mark.parametrize("n,depth,p", [(60000, 6, 16), (30000, 5, 20), (4096, 4, 12), (4096, 4, 8)])
def test_fmm_potential_pascal_matches_oracle(P, n, depth, p):
    import synthetic as sy
    print(f"fmm pascal n={n} depth={depth} p={p}", flush=True)
    xy = sy.mixed(n, 61)
    q = sy.charges(n, 62)
    t = sy.uniform(2048, 63)
    phi, f = P.potential(_t(xy), _t(q), _t(t), depth=depth, p=p, precision="f32_pascal")
    phir, fr = oracle.fmm(xy.astype(np.float64), q.astype(np.float64), t.astype(np.float64), depth, p)
    assert rel(phi.cpu().numpy().real, phir.real) < TOL
    assert rel(f.cpu().numpy(), fr) < TOL


@pytest.mark.parametrize("n,depth,p", [(4096, 4, 12), (60000, 6, 16)])
def test_gradient_pascal_matches_oracle(P, n, depth, p):
    """Loss sum over 4096 targets of (Re phi)^2; the backward pass runs the
    Pascal-form adjoint M2L."""
    import synthetic as sy
    print(f"gradient pascal n={n} depth={depth} p={p}", flush=True)
    xy = sy.uniform(n, 71)
    q = sy.charges(n, 72)
    t = sy.uniform(4096, 73)
    xg = _t(xy).requires_grad_(True)
    qg = _t(q).requires_grad_(True)
    phi, _ = P.potential(xg, qg, _t(t), depth=depth, p=p, precision="f32_pascal")
    (phi.real ** 2).sum().backward()
    phir, _ = oracle.fmm(xy.astype(np.float64), q.astype(np.float64), t.astype(np.float64), depth, p)
    gq_r, gxy_r = oracle.fmm_grad(xy.astype(np.float64), q.astype(np.float64), t.astype(np.float64), depth, p,
                                  (2 * phir.real).astype(np.complex128))
    assert rel(qg.grad.cpu().numpy(), gq_r) < TOL
    assert rel(xg.grad.cpu().numpy(), gxy_r) < TOL
