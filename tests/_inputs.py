"""Shared construction of oracle-side reference inputs for the tests.

Only the seeded generators (synthetic) and the oracle are used here; nothing
comes from the GPU library."""
import functools

import numpy as np

import oracle
import synthetic as sy


def multipoles(depth: int, p: int, n: int, seed: int, kind: str = "uniform"):
    """Scaled multipole expansions of a seeded point set, as the GPU receives
    them (complex64), and the exactly equivalent unscaled FP64 array."""
    if kind == "uniform":
        xy = sy.uniform(n, seed)
    elif kind == "mixed":
        xy = sy.mixed(n, seed)
    else:
        xy = sy.clustered(n, seed)
    q = sy.charges(n, seed + 1000)
    xy64, q64 = xy.astype(np.float64), q.astype(np.float64)
    perm, ls = oracle.build_tree(xy64, depth)
    M = oracle.m2m(oracle.p2m(xy64[perm], q64[perm], ls, depth, p), depth, p)
    Ms32 = oracle.scale_multipoles(M, depth).astype(np.complex64)
    M_exact = oracle.unscale_multipoles(Ms32.astype(np.complex128), depth)
    return Ms32, M_exact


def level_slices(depth: int, lmin: int = 2):
    return [(l, slice(oracle.level_offset(l), oracle.level_offset(l + 1)))
            for l in range(lmin, depth + 1)]


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


@functools.lru_cache(maxsize=3)
def full_size_multipoles(depth: int, p: int, n: int, kind: str):
    """multipoles() of the large workloads, computed once per test session."""
    return multipoles(depth, p, n, seed=3, kind=kind)
