"""Host-side logic of the benchmark (no GPU): the near-field pair count and
the per-translation flop counts the roofline uses."""
import numpy as np
import pytest

import bench


def _brute_pairs(counts, depth):
    def dec(m):
        x = y = 0
        for b in range(depth):
            x |= ((m >> (2 * b)) & 1) << b
            y |= ((m >> (2 * b + 1)) & 1) << b
        return x, y
    pos = [dec(m) for m in range(4 ** depth)]
    tot = 0
    for a in range(4 ** depth):
        for b in range(4 ** depth):
            if abs(pos[a][0] - pos[b][0]) <= 1 and abs(pos[a][1] - pos[b][1]) <= 1:
                tot += counts[a] * counts[b] - (counts[a] if a == b else 0)
    return tot


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_near_field_pairs_brute_force(depth):
    c = np.random.default_rng(depth).integers(0, 6, 4 ** depth)
    ls = np.concatenate([[0], np.cumsum(c)])
    assert bench.near_field_pairs(ls, depth) == _brute_pairs(c, depth)


def test_near_field_pairs_uniform_grid():
    # k points in every leaf of a 2^d x 2^d grid: interior leaves see 9 k - 1
    # partners per point; the count of neighbour pairs follows in closed form
    d, k = 4, 3
    side = 1 << d
    ls = np.arange(0, k * side * side + 1, k)
    nb = sum((side - abs(dx)) * (side - abs(dy)) for dx in (-1, 0, 1) for dy in (-1, 0, 1))
    assert bench.near_field_pairs(ls, d) == k * k * nb - k * side * side


@pytest.mark.parametrize("prec", ["f32", "f32_pascal", "bf16x3", "f64_hankel"])
def test_own_flops_below_dense_only_where_the_form_saves(prec):
    for p in (8, 12, 16, 20):
        own = bench.own_flops_per_translation(p, prec, "L")
        dense = bench.dense_flops_per_translation(p, "L")
        assert own > 0
        if prec in ("f32_pascal", "f64_hankel"):
            assert own < dense
