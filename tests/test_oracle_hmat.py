"""Pins of the oracle's hierarchical block partition (oracle/hmat.py) against
what the definition of an interaction-list partition fixes, independent of
the code under test: every pair of non-empty leaves lies in exactly one block
(far blocks expanded to their leaves, plus near blocks), far blocks are
separated by at least one cell, an interior cell of a full tree has the
textbook 6^d - 3^d cells in its interaction list, and summing the dense
blocks of the partition reproduces K x."""
import itertools

import numpy as np
import pytest

from oracle import dense, hmat


def _points(d, N, seed):
    return np.random.default_rng(seed).uniform(0, 1, (N, d))


@pytest.mark.parametrize("d,N,L", [(1, 300, 5), (2, 800, 4), (3, 600, 3)])
def test_blocks_cover_every_leaf_pair_once(d, N, L):
    X = _points(d, N, d)
    box = [[0.0, 1.0]] * d
    far, near = hmat.partition(X, box, L)
    leaves = {tuple(int(v) for v in c) for c in hmat.leaf_cells(X, box, L)}
    count = {}
    for (k, c, c2) in far:
        sh = L - k
        # leaves under c and c2 that hold points
        for a in leaves:
            if tuple(v >> sh for v in a) != c:
                continue
            for b in leaves:
                if tuple(v >> sh for v in b) == c2:
                    count[(a, b)] = count.get((a, b), 0) + 1
    for (a, b) in near:
        count[(a, b)] = count.get((a, b), 0) + 1
    assert len(count) == len(leaves) ** 2
    assert set(count.values()) == {1}


@pytest.mark.parametrize("d", [1, 2, 3])
def test_far_blocks_are_separated(d):
    X = _points(d, 500, 7)
    far, near = hmat.partition(X, [[0.0, 1.0]] * d, 3)
    assert far
    for (k, c, c2) in far:
        assert max(abs(a - b) for a, b in zip(c, c2)) >= 2
        assert max(abs((a >> 1) - (b >> 1)) for a, b in zip(c, c2)) <= 1
    for (c, c2) in near:
        assert max(abs(a - b) for a, b in zip(c, c2)) <= 1


@pytest.mark.parametrize("d,L", [(2, 3), (3, 3)])
def test_interior_interaction_list_size(d, L):
    # one point at the centre of every leaf: a full tree
    side = 2 ** L
    cells = np.array(list(itertools.product(range(side), repeat=d)), float)
    X = (cells + 0.5) / side
    far, _ = hmat.partition(X, [[0.0, 1.0]] * d, L)
    c = tuple([side // 2] * d)   # an interior cell at the leaf level
    lst = [f for f in far if f[0] == L and f[1] == c]
    assert len(lst) == 6 ** d - 3 ** d


def test_dense_blocks_of_the_partition_sum_to_K():
    d, L = 2, 3
    X = _points(d, 400, 3)
    box = [[0.0, 1.0]] * d
    far, near = hmat.partition(X, box, L)
    leaves = hmat.leaf_cells(X, box, L)
    K = dense.dense_K("se", X, X, np.array([0.7]))
    x = np.random.default_rng(4).standard_normal(X.shape[0])
    y = np.zeros(X.shape[0])
    for (k, c, c2) in far:
        rows = np.all((leaves >> (L - k)) == np.array(c), axis=1)
        cols = np.all((leaves >> (L - k)) == np.array(c2), axis=1)
        y[rows] += K[np.ix_(rows, cols)] @ x[cols]
    for (c, c2) in near:
        rows = np.all(leaves == np.array(c), axis=1)
        cols = np.all(leaves == np.array(c2), axis=1)
        y[rows] += K[np.ix_(rows, cols)] @ x[cols]
    assert np.abs(y - K @ x).max() <= 1e-12 * np.abs(K @ x).max()


def test_morton_order_keeps_cells_contiguous():
    d, L = 3, 3
    X = _points(d, 700, 9)
    leaves = hmat.leaf_cells(X, [[0.0, 1.0]] * d, L)
    order = np.argsort(hmat.morton(leaves, L), kind="stable")
    for k in range(L + 1):
        cells = [tuple(c) for c in (leaves[order] >> (L - k))]
        # each cell's points form one run in Morton order
        seen, prev = set(), None
        for c in cells:
            if c != prev:
                assert c not in seen
                seen.add(c)
                prev = c
