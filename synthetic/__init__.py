"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module draws random numbers and nothing else: it holds none of the fast
multipole method's arithmetic.  Every generator draws in FP64 from
``numpy.random.Generator(PCG64(seed))`` and rounds once to FP32, so the GPU
library and the FP64 oracle receive bit-identical inputs (the oracle promotes
the FP32 values exactly to FP64).

Workloads (the paper measures on synthetic data only; these stand in for the
shapes its FMM benchmarks imply):
  * ``uniform``      points uniform in [0,1)^2;
  * ``clustered``    a Gaussian mixture of ``n_centres`` isotropic clusters with
                     centres uniform in [0.2,0.8]^2 and standard deviation
                     ``sigma``, each sample redrawn until it lies in [0,1)^2;
  * ``mixed``        a fraction of clustered points over a uniform background;
  * ``charges``      source strengths uniform in [-1,1];
  * ``expansions``   random complex coefficients with a per-order decay, used
                     only where an M2L is exercised on its own.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _to_unit_f32(a: np.ndarray) -> np.ndarray:
    """Round FP64 samples in [0,1) to FP32, keeping them strictly below 1."""
    a32 = a.astype(np.float32)
    below = np.nextafter(np.float32(1.0), np.float32(0.0))
    return np.minimum(a32, below)


def uniform(n: int, seed: int) -> np.ndarray:
    """``n`` points uniform in [0,1)^2 as float32 [n, 2]."""
    return _to_unit_f32(rng(seed).random((n, 2)))


def clustered(n: int, seed: int, n_centres: int = 8, sigma: float = 0.05) -> np.ndarray:
    """Gaussian-mixture points (float32 [n, 2]) confined to [0,1)^2 by resampling."""
    g = rng(seed)
    centres = 0.2 + 0.6 * g.random((n_centres, 2))
    which = g.integers(0, n_centres, size=n)
    out = np.empty((n, 2), np.float64)
    todo = np.arange(n)
    while todo.size:
        pts = centres[which[todo]] + sigma * g.standard_normal((todo.size, 2))
        ok = np.all((pts >= 0.0) & (pts < 1.0), axis=1)
        out[todo[ok]] = pts[ok]
        todo = todo[~ok]
    return _to_unit_f32(out)


def mixed(n: int, seed: int, clustered_fraction: float = 0.5, n_centres: int = 8,
          sigma: float = 0.05) -> np.ndarray:
    """``clustered_fraction`` of the points clustered, the rest uniform; shuffled."""
    nc = int(round(n * clustered_fraction))
    a = clustered(nc, seed * 2 + 1, n_centres, sigma)
    b = uniform(n - nc, seed * 2 + 2)
    pts = np.concatenate([a, b], axis=0)
    perm = rng(seed).permutation(n)
    return np.ascontiguousarray(pts[perm])


def charges(n: int, seed: int) -> np.ndarray:
    """Source strengths uniform in [-1, 1], float32 [n]."""
    return (2.0 * rng(seed).random(n) - 1.0).astype(np.float32)


def expansions(nbox: int, p: int, seed: int, decay: float = 0.5) -> np.ndarray:
    """Random complex64 coefficients [nbox, p] with |c_k| ~ decay^k."""
    g = rng(seed)
    scale = decay ** np.arange(p)
    re = g.standard_normal((nbox, p)) * scale
    im = g.standard_normal((nbox, p)) * scale
    return (re + 1j * im).astype(np.complex64)
