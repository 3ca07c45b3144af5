"""Fast Gauss transform through its Hermite stage (arXiv:1009.3457, Sec. 2.2
and Sec. 4.2) on the library's kernels (include/fgt2d.h).

    G(y) = sum_i q_i exp(-|x_i - y|^2 / (2 sigma^2))

Sources are grouped into the 4^depth boxes of the uniform grid over [0,1]^2;
each box's Hermite series (p x p terms) is evaluated at the targets whose box
lies within K boxes of it in both directions.
"""
from __future__ import annotations

import torch

from . import _binding as B


def gauss_transform(xy: torch.Tensor, q: torch.Tensor, targets: torch.Tensor, depth: int, p: int,
                    sigma: float, K: int) -> torch.Tensor:
    """G at the targets (float32 [nt], original order).  xy [n, 2], q [n] and
    targets [nt, 2] float32 on the GPU, points in [0,1]^2."""
    perm, ls = B.build_tree(xy.contiguous(), depth)
    A = B.fgt_hermite_coeffs(B.gather(xy.contiguous(), perm), B.gather(q.contiguous(), perm), ls, depth, p,
                             sigma)
    tperm, _ = B.build_tree(targets.contiguous(), depth)  # box order keeps each wave within a few boxes
    G = B.fgt_hermite_eval(B.gather(targets.contiguous(), tperm), depth, p, sigma, K, A)
    return B.scatter(G, tperm)
