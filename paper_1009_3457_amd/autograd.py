"""Differentiable wrappers: the M2L as a torch.autograd.Function whose backward
is the hand-written adjoint M2L, and the whole FMM potential/field evaluation
whose backward chains the plain transposes of every stage.

Complex gradients follow PyTorch's convention: for a real loss l and a
holomorphic linear map y = A x, grad_x = A^H grad_y = conj(A^T conj(grad_y)).
The library computes plain transposes A^T, so the wrappers conjugate around
them.
"""
from __future__ import annotations

import torch

from . import _binding as B


class M2LFunction(torch.autograd.Function):
    """(L~, b) = M2L(M~) on levels lmin..lmax (other levels of L~, b are zero)."""

    @staticmethod
    def forward(ctx, M, depth, p, lmin, lmax, precision):
        M = M.contiguous()
        L, b = B.m2l(M, depth, p, lmin, lmax, precision)
        ctx.cfg = (depth, p, lmin, lmax, precision)
        return L, b

    @staticmethod
    def backward(ctx, gL, gb):
        depth, p, lmin, lmax, precision = ctx.cfg
        dev = gL.device if gL is not None else gb.device
        nb = B.num_boxes(depth)
        cL = torch.zeros(nb, p, dtype=torch.complex64, device=dev) if gL is None \
            else gL.conj().resolve_conj().contiguous()
        cb = None if gb is None else gb.conj().resolve_conj().contiguous()
        gM = B.m2l_backward(cL, cb, depth, p, lmin, lmax, precision)
        return gM.conj().resolve_conj(), None, None, None, None, None


def m2l(M, depth: int, p: int, lmin: int = 2, lmax: int | None = None, precision="f32"):
    prec = B.PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    lmax = depth if lmax is None else lmax
    return M2LFunction.apply(M, depth, p, lmin, lmax, prec)


class _Plan:
    """Sorted sources/targets of one evaluation (a frozen tree)."""

    def __init__(self, xy, q, txy, depth):
        self.depth = depth
        self.perm, self.ls = B.build_tree(xy, depth)
        self.tperm, self.tls = B.build_tree(txy, depth)
        self.xs = B.gather(xy, self.perm)
        self.qs = B.gather(q, self.perm)
        self.ts = B.gather(txy, self.tperm)


def fmm_forward(plan: _Plan, p: int, precision: int):
    depth = plan.depth
    M = B.p2m(plan.xs, plan.qs, plan.ls, depth, p)
    B.m2m(M, depth, p)
    Lm, bm = B.m2l(M, depth, p, 2, depth, precision)
    L, b = B.l2l(Lm, bm, depth, p)
    phi, field = B.l2p(plan.ts, plan.tls, L, b, depth, p)
    B.p2p(plan.xs, plan.qs, plan.ls, plan.ts, plan.tls, depth, phi, field)
    return B.scatter(phi, plan.tperm), B.scatter(field, plan.tperm)


def fmm_backward(plan: _Plan, p: int, precision: int, gphi, gfield):
    """Returns (grad_q [n], grad_xy [n, 2]) in the original source order."""
    depth = plan.depth
    dev = plan.xs.device
    nt = plan.ts.shape[0]

    def _cot(g):
        if g is None:
            return None
        return B.gather(g.conj().resolve_conj().contiguous(), plan.tperm)

    cphi, cfield = _cot(gphi), _cot(gfield)
    gL, gb = B.l2p_backward(plan.ts, plan.tls, cphi, cfield, depth, p)
    gLm, gbm = B.l2l_backward(gL, gb, depth, p)
    gM = B.m2l_backward(gLm, gbm, depth, p, 2, depth, precision)
    B.m2m_backward(gM, depth, p)
    gq, G = B.p2m_backward(plan.xs, plan.qs, plan.ls, depth, p, gM)
    B.p2p_backward(plan.xs, plan.qs, plan.ls, plan.ts, plan.tls, depth, cphi, cfield, gq, G)
    gq = B.scatter(gq, plan.perm)
    G = B.scatter(G, plan.perm)
    gxy = torch.stack([G.real, -G.imag], dim=1).contiguous()
    del nt, dev
    return gq, gxy


class FMMPotential(torch.autograd.Function):
    """(phi, field) at the targets for sources (xy, q); differentiable in xy and q
    at a frozen tree.  Targets are treated as constants."""

    @staticmethod
    def forward(ctx, xy, q, txy, depth, p, precision):
        xy = xy.detach().contiguous()
        q = q.detach().contiguous()
        txy = txy.detach().contiguous()
        plan = _Plan(xy, q, txy, depth)
        phi, field = fmm_forward(plan, p, precision)
        ctx.plan = plan
        ctx.cfg = (p, precision)
        return phi, field

    @staticmethod
    def backward(ctx, gphi, gfield):
        p, precision = ctx.cfg
        gq, gxy = fmm_backward(ctx.plan, p, precision, gphi, gfield)
        return gxy, gq, None, None, None, None


def potential(xy, q, targets=None, depth: int = 8, p: int = 12, precision="f32"):
    """phi(z) = sum_s q_s log(z - z_s) and field f(z) = sum_s q_s/(z - z_s) at the
    targets (default: the sources, with self-interaction excluded), by the FMM.

    xy [n, 2] and q [n] float32 on the GPU; returns complex64 (phi, field)."""
    prec = B.PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    t = xy.detach() if targets is None else targets
    return FMMPotential.apply(xy, q, t, depth, p, prec)
