"""FP64 oracle of the fast Gauss transform's Hermite-series evaluation
(arXiv:1009.3457, Sec. 2.2 and Sec. 4.2).  Test infrastructure only, like the
rest of ``oracle``: thin ctypes wrappers around ``fgt2d_oracle.c``.

Two dimensions; boxes are the 4^depth leaves of the uniform grid over [0,1)^2
(Morton order, as the FMM tree); coefficients are float64 ``[4^depth, p, p]``
indexed ``[box, a, b]`` for the multi-index alpha = (a, b).
"""
from __future__ import annotations

import numpy as np

from . import _d, _f64, _i32, _load, build_tree  # noqa: F401


def hermite_functions(t: float, p: int) -> np.ndarray:
    """h_n(t) = exp(-t^2) H_n(t), n < p (physicists' Hermite polynomials)."""
    h = np.zeros(p, np.float64)
    _load().ora_hermite_functions(float(t), p, _d(h))
    return h


def direct(xy, q, txy, sigma: float) -> np.ndarray:
    """Eq. (eqn:dgt): G(y) = sum_i q_i exp(-|x_i - y|^2 / (2 sigma^2))."""
    xy, q, txy = _f64(xy), _f64(q), _f64(txy)
    G = np.zeros(txy.shape[0], np.float64)
    _load().ora_fgt_direct(_d(xy), _d(q), xy.shape[0], _d(txy), txy.shape[0], float(sigma), _d(G))
    return G


def direct_boxes(xy_sorted, q_sorted, leaf_start, depth: int, txy, sigma: float, K: int) -> np.ndarray:
    """Eq. (eqn:dgt) over the sources of the (2K+1)^2 boxes around each target's box."""
    xs, qs, txy = _f64(xy_sorted), _f64(q_sorted), _f64(txy)
    G = np.zeros(txy.shape[0], np.float64)
    _load().ora_fgt_direct_boxes(_d(xs), _d(qs), _i32(leaf_start), depth, _d(txy), txy.shape[0],
                                 float(sigma), int(K), _d(G))
    return G


def hermite_coeffs(xy_sorted, q_sorted, leaf_start, depth: int, p: int, sigma: float) -> np.ndarray:
    """Eq. (eqn:A_alpha) for every box: A[box, a, b]."""
    xs, qs = _f64(xy_sorted), _f64(q_sorted)
    A = np.zeros((1 << (2 * depth), p, p), np.float64)
    _load().ora_fgt_hermite_coeffs(_d(xs), _d(qs), _i32(leaf_start), depth, p, float(sigma), _d(A))
    return A


def hermite_eval(txy, depth: int, p: int, sigma: float, K: int, A) -> np.ndarray:
    """Eq. (eqn:hermite) at each target over the (2K+1)^2 boxes around its box."""
    txy = _f64(txy)
    A = np.ascontiguousarray(A, np.float64)
    G = np.zeros(txy.shape[0], np.float64)
    _load().ora_fgt_hermite_eval(_d(txy), txy.shape[0], depth, p, float(sigma), int(K), _d(A), _d(G))
    return G


def gauss_transform(xy, q, txy, depth: int, p: int, sigma: float, K: int):
    """Hermite coefficients from the sources, evaluated at the targets; also
    returns the coefficients."""
    xy = _f64(xy)
    perm, ls = build_tree(xy, depth)
    A = hermite_coeffs(xy[perm], _f64(q)[perm], ls, depth, p, sigma)
    return hermite_eval(txy, depth, p, sigma, K, A), A
