"""The allocation-free tree build (fmm2d_build_tree_noalloc) against the
ordinary one (fmm2d_build_tree) through the C ABI: identical perm,
leaf_start and domain flag (bit for bit), on two calls in a row with the
second input smaller, and on a point outside the domain; both also equal the
oracle's stable leaf sort."""
import numpy as np
import pytest

import oracle
import synthetic as sy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1009_3457_amd import _binding as B
    return B


def _both(B, xy, depth):
    import torch
    t = torch.from_numpy(xy).cuda()
    p1, l1, f1 = B.build_tree(t, depth, check=False)
    p2, l2, f2 = B.build_tree_noalloc(t, depth)
    torch.cuda.synchronize()
    return (p1.cpu().numpy(), l1.cpu().numpy(), int(f1.item())), (p2.cpu().numpy(), l2.cpu().numpy(), int(f2.item()))


def test_noalloc_matches_build_tree_twice_second_smaller(B):
    cases = [(B.NOALLOC_MAX_POINTS, 9, "mixed"), (100003, 6, "uniform")]
    for n, depth, kind in cases:
        print(f"build_tree_noalloc n={n} depth={depth} {kind}", flush=True)
        xy = sy.mixed(n, 5) if kind == "mixed" else sy.uniform(n, 5)
        xy[0] = (1.0, 1.0)
        xy[2] = xy[3]
        (p1, l1, f1), (p2, l2, f2) = _both(B, xy, depth)
        assert f1 == 0 and f2 == 0
        assert np.array_equal(p1, p2) and np.array_equal(l1, l2)
        pr, lr = oracle.build_tree(xy.astype(np.float64), depth)
        assert np.array_equal(p2, pr) and np.array_equal(l2, lr)


def test_noalloc_flags_points_outside(B):
    xy = sy.uniform(5000, 6)
    xy[123] = (0.5, 1.5)
    (_, _, f1), (_, _, f2) = _both(B, xy, 5)
    assert f1 != 0 and f2 != 0
    xy = sy.uniform(7000, 7)
    (p1, l1, f1), (p2, l2, f2) = _both(B, xy, 5)  # the next call starts from a clear flag
    assert f1 == 0 and f2 == 0 and np.array_equal(p1, p2) and np.array_equal(l1, l2)


def test_noalloc_empty_input(B):
    (p1, l1, f1), (p2, l2, f2) = _both(B, np.zeros((0, 2), np.float32), 3)
    assert p2.size == 0 and np.array_equal(l1, l2) and not l2.any() and f2 == 0


def test_noalloc_rejects_more_points_than_its_array(B):
    import torch
    xy = torch.zeros(B.NOALLOC_MAX_POINTS + 1, 2, dtype=torch.float32, device="cuda")
    with pytest.raises(B.FMMError, match="exceeds|outside"):
        B.build_tree_noalloc(xy, 8)
