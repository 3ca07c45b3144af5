#!/usr/bin/env python3
"""Coefficients of the atan polynomial in p2p.hip (atan2_p2p).

atan(a) on [0, 1] is approximated by the odd polynomial a P(a^2), P of degree
7 (eight coefficients), with the smallest largest absolute error: the minimax
polynomial, found by the Remez exchange algorithm on the basis a^(2j+1).
Each step solves for the coefficients and the levelled error E on a
reference of nine points (sum_j c_j x_i^(2j+1) + (-1)^i E = atan(x_i)), then
moves the reference to the extrema of the new error curve, until the
extrema are level.  The coefficients are then rounded to FP32, and the
largest error of the rounded polynomial, evaluated in FP32 by Horner's rule
with fused multiply-adds as the kernel does, is reported.

Run: python fit_atan.py   (prints the coefficients as C literals, highest
order first, in the order the kernel's Horner steps use them)
"""
from __future__ import annotations

import numpy as np

NTERMS = 8  # a, a^3, ..., a^15


def _basis(x):
    return np.stack([x ** (2 * j + 1) for j in range(NTERMS)], axis=1)


def _solve(ref):
    n = NTERMS
    A = np.zeros((n + 1, n + 1))
    A[:, :n] = _basis(ref)
    A[:, n] = (-1.0) ** np.arange(n + 1)
    sol = np.linalg.solve(A, np.arctan(ref))
    return sol[:n], sol[n]


def _extrema(c, grid):
    err = _basis(grid) @ c - np.arctan(grid)
    # points where the error changes direction, plus the interval ends
    idx = [0]
    for i in range(1, grid.size - 1):
        if (err[i] - err[i - 1]) * (err[i + 1] - err[i]) <= 0:
            idx.append(i)
    idx.append(grid.size - 1)
    idx = np.array(sorted(set(idx)))
    # keep one extremum per sign run, the largest in magnitude
    keep = []
    for i in idx:
        if keep and np.sign(err[i]) == np.sign(err[keep[-1]]):
            if abs(err[i]) > abs(err[keep[-1]]):
                keep[-1] = i
        else:
            keep.append(i)
    return grid[np.array(keep)], err


def remez(iters=30):
    n = NTERMS
    ref = 0.5 - 0.5 * np.cos(np.pi * np.arange(n + 1) / n)  # Chebyshev points on [0, 1]
    grid = np.linspace(0.0, 1.0, 200001)
    c, E = _solve(ref)
    for _ in range(iters):
        ext, err = _extrema(c, grid)
        if ext.size < n + 1:
            break
        # the n + 1 consecutive extrema with the largest smallest magnitude
        errs = np.abs(_basis(ext) @ c - np.arctan(ext))
        best, start = -1.0, 0
        for s in range(ext.size - n):
            m = errs[s:s + n + 1].min()
            if m > best:
                best, start = m, s
        ref = ext[start:start + n + 1]
        c, E = _solve(ref)
        if np.max(np.abs(err)) - abs(E) < 1e-3 * abs(E):
            break
    return c, E


def horner_f32(c32, a):
    """a P(a^2) in FP32 with a fused multiply-add per step (as the kernel)."""
    a = a.astype(np.float32)
    t = (a * a).astype(np.float32)
    r = np.full_like(a, c32[-1])
    for cj in c32[-2::-1]:
        r = (r.astype(np.float64) * t.astype(np.float64) + np.float64(cj)).astype(np.float32)
    return (r * a).astype(np.float32)


def main():
    c, E = remez()
    c32 = c.astype(np.float32)
    a = np.linspace(0.0, 1.0, 2000001)
    err64 = np.max(np.abs(_basis(a) @ c - np.arctan(a)))
    err32 = np.max(np.abs(horner_f32(c32, a).astype(np.float64) - np.arctan(a)))
    print(f"levelled error E = {abs(E):.3e}; largest error: FP64 {err64:.3e}, FP32 Horner {err32:.3e}")
    print("coefficients, highest order first:")
    for cj in c32[::-1]:
        print(f"  {float(cj)!r}f")


if __name__ == "__main__":
    main()
