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
    """Differentiable M2L of the scaled multipoles M (levels lmin..lmax);
    precision as in potential()."""
    prec = B.PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    lmax = depth if lmax is None else lmax
    return M2LFunction.apply(M, depth, p, lmin, lmax, prec)


class _Plan:
    """Sorted sources/targets of one evaluation (a frozen tree).  The domain
    flags of both tree builds stay on the device; `check()` reads them."""

    def __init__(self, xy, q, txy, depth):
        self.depth = depth
        self.perm, self.ls, f1 = B.build_tree(xy, depth, check=False)
        self.tperm, self.tls, f2 = B.build_tree(txy, depth, check=False)
        self.flags = (f1, f2)
        self.xs = B.gather(xy, self.perm)
        self.qs = B.gather(q, self.perm)
        self.ts = B.gather(txy, self.tperm)

    def check(self):
        B.check_domain(*self.flags)


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
    return gq, gxy


class FMMPotential(torch.autograd.Function):
    """(phi, field) at the targets for sources (xy, q) at a frozen tree.

    Differentiable in xy and q, and in the target positions txy for a
    cotangent of phi: phi is holomorphic in the evaluation point z_t with
    dphi/dz_t = field(z_t), the field this evaluation returns (its far part
    is the derivative of the L2P series, its near part that of the P2P sum).
    A cotangent of the field with targets that require a gradient would need
    dfield/dz_t, which is not computed: that case raises NotImplementedError.
    """

    @staticmethod
    def forward(ctx, xy, q, txy, depth, p, precision):
        ctx.set_materialize_grads(False)
        xy = xy.detach().contiguous()
        q = q.detach().contiguous()
        txy = txy.detach().contiguous()
        plan = _Plan(xy, q, txy, depth)
        phi, field = fmm_forward(plan, p, precision)
        plan.check()  # waits once, after every stage has been enqueued
        ctx.plan = plan
        ctx.cfg = (p, precision)
        ctx.save_for_backward(field)
        return phi, field

    @staticmethod
    def backward(ctx, gphi, gfield):
        p, precision = ctx.cfg
        need_xy, need_q, need_t = ctx.needs_input_grad[:3]
        gxy = gq = gt = None
        if (need_xy or need_q) and (gphi is not None or gfield is not None):
            gq, gxy = fmm_backward(ctx.plan, p, precision, gphi, gfield)
        if need_t:
            if gfield is not None:
                raise NotImplementedError(
                    "the gradient with respect to target positions is available for a cotangent of phi "
                    "only; a cotangent of the field would need its derivative")
            if gphi is not None:
                (field,) = ctx.saved_tensors
                w = gphi.conj() * field  # dl/dx = Re(conj(g) f), dl/dy = Re(conj(g) i f) = -Im(conj(g) f)
                gt = torch.stack([w.real, -w.imag], dim=1).contiguous()
        return gxy, gq, gt, None, None, None


def potential(xy, q, targets=None, depth: int = 8, p: int = 12, precision="f32"):
    """phi(z) = sum_s q_s log(z - z_s) and field f(z) = sum_s q_s/(z - z_s) at the
    targets (default: the sources, with self-interaction excluded), by the FMM.

    xy [n, 2] and q [n] float32 on the GPU; returns complex64 (phi, field).
    precision selects the M2L form: "f32" (Gauss), "f32_pascal", "bf16x3",
    "f16x3" or "f64_hankel" (the keys of PRECISIONS), or its integer code.
    Gradients (at a frozen tree) flow to q and xy, and to the targets' positions
    for a loss on phi.  With targets=None the sources are also the evaluation
    points, so xy's gradient holds both the source-side and the target-side
    terms; a loss on the field then raises NotImplementedError in backward
    when xy requires a gradient."""
    prec = B.PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    t = xy if targets is None else targets
    return FMMPotential.apply(xy, q, t, depth, p, prec)
