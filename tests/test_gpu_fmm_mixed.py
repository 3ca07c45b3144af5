"""The whole FMM and its gradients with the M2L in split precision (BF16x3,
FP16x3), against the FP64 oracle on the same tree and order p.  Every other
stage is the same as in FP32; the tolerance is the split-precision M2L's,
1e-4 relative (L2 norm), on Re phi, the field and the gradients."""
import numpy as np
import pytest

import oracle
import synthetic as sy
from tests._inputs import rel

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-4


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


@pytest.mark.parametrize("prec", ["bf16x3", "f16x3"])
@pytest.mark.parametrize("n,depth,p", [(60000, 6, 16), (30000, 5, 20), (4096, 4, 12), (4096, 4, 8)])
def test_fmm_potential_split_precision_matches_oracle(P, prec, n, depth, p):
    print(f"fmm {prec} n={n} depth={depth} p={p}", flush=True)
    xy = sy.mixed(n, 41)
    q = sy.charges(n, 42)
    t = sy.uniform(2048, 43)
    phi, f = P.potential(_t(xy), _t(q), _t(t), depth=depth, p=p, precision=prec)
    phir, fr = oracle.fmm(xy.astype(np.float64), q.astype(np.float64), t.astype(np.float64), depth, p)
    assert rel(phi.cpu().numpy().real, phir.real) < TOL_MIXED
    assert rel(f.cpu().numpy(), fr) < TOL_MIXED


@pytest.mark.parametrize("prec", ["bf16x3", "f16x3"])
@pytest.mark.parametrize("n,depth,p", [(4096, 4, 12), (60000, 6, 16)])
def test_gradient_split_precision_matches_oracle(P, prec, n, depth, p):
    """Loss sum over 4096 targets of (Re phi)^2; the backward pass runs the
    split-precision adjoint M2L."""
    print(f"gradient {prec} n={n} depth={depth} p={p}", flush=True)
    xy = sy.uniform(n, 51)
    q = sy.charges(n, 52)
    t = sy.uniform(4096, 53)
    xg = _t(xy).requires_grad_(True)
    qg = _t(q).requires_grad_(True)
    phi, _ = P.potential(xg, qg, _t(t), depth=depth, p=p, precision=prec)
    (phi.real ** 2).sum().backward()
    phir, _ = oracle.fmm(xy.astype(np.float64), q.astype(np.float64), t.astype(np.float64), depth, p)
    gq_r, gxy_r = oracle.fmm_grad(xy.astype(np.float64), q.astype(np.float64), t.astype(np.float64), depth, p,
                                  (2 * phir.real).astype(np.complex128))
    assert rel(qg.grad.cpu().numpy(), gq_r) < TOL_MIXED
    assert rel(xg.grad.cpu().numpy(), gxy_r) < TOL_MIXED


@pytest.mark.parametrize("prec", ["bf16x3", "f16x3"])
@pytest.mark.parametrize("p", [16, 20])
def test_m2l_autograd_split_precision_matches_adjoint(P, prec, p):
    """torch.autograd through the M2L Function in split precision: the
    gradient of Re<W, L> + Re<w, b> equals the conjugated transpose."""
    depth = 5
    g = np.random.Generator(np.random.PCG64(7 + p))
    nb = oracle.num_boxes(depth)
    M = ((g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))) * 0.5 ** np.arange(p)).astype(np.complex64)
    W = (g.standard_normal((nb, p)) + 1j * g.standard_normal((nb, p))).astype(np.complex64)
    w = (g.standard_normal(nb) + 1j * g.standard_normal(nb)).astype(np.complex64)
    Mt = _t(M).requires_grad_(True)
    L, b = P.m2l(Mt, depth, p, precision=prec)
    ((L * _t(W)).real.sum() + (b * _t(w)).real.sum()).backward()
    W_un = oracle.scale_locals(W.astype(np.complex128), depth)
    ref = np.conj(oracle.unscale_multipoles(oracle.m2l_transpose(W_un, w.astype(np.complex128), depth, p), depth))
    lo = oracle.level_offset(2)
    assert rel(Mt.grad.cpu().numpy()[lo:], ref[lo:]) < TOL_MIXED
