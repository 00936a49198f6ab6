"""Block partition of a hierarchical matrix over a uniform tree (test
infrastructure only): the leaf level, the cell of every point, the far
blocks of every level (interaction lists) and the near blocks between
neighbouring leaves, written from their definitions with plain loops over
cell pairs.

The tree is the uniform refinement of the root box: level k has 2^k cells
per dimension; the far blocks at level k >= 2 are the pairs of non-empty
cells (c, c') whose parents are equal or neighbours (max_j |p_j - p'_j| <= 1)
while the cells themselves are not (max_j |c_j - c'_j| >= 2); the near blocks
are the pairs of non-empty leaves with max_j |c_j - c'_j| <= 1.  This is the
interaction-list partition of fast multipole and hierarchical-matrix codes
(Section 1 names their admissible blocks as the method's use); every pair of
points falls in exactly one block.
"""
import numpy as np


def leaf_level(N, d, leaf_points):
    """Smallest L with N / 2^(L d) <= leaf_points (and L d <= 30)."""
    L = 0
    while N / 2.0 ** (L * d) > leaf_points and (L + 1) * d <= 30:
        L += 1
    return L


def leaf_cells(X, box, L):
    """Integer cell coordinates (N, d) of every point at level L:
    floor((x - lo) / (hi - lo) * 2^L), clamped to [0, 2^L - 1]."""
    b = np.asarray(box, float)
    side = 2 ** L
    u = (np.asarray(X, float) - b[:, 0]) / (b[:, 1] - b[:, 0]) * float(side)
    return np.clip(np.floor(u).astype(np.int64), 0, side - 1)


def morton(cells, L):
    """Morton codes (bit b of coordinate j at b d + j) of integer cells (N, d)."""
    cells = np.asarray(cells, np.int64)
    d = cells.shape[1]
    m = np.zeros(cells.shape[0], np.int64)
    for b in range(L):
        for j in range(d):
            m |= ((cells[:, j] >> b) & 1) << (b * d + j)
    return m


def partition(X, box, L):
    """(far, near): far = set of (k, cell tuple, cell tuple) for k = 2..L,
    near = set of (leaf tuple, leaf tuple); cells hold points of X."""
    leaves = leaf_cells(X, box, L)
    far, near = set(), set()
    for k in range(2, L + 1):
        cells = sorted({tuple(int(v) for v in c) for c in (leaves >> (L - k))})
        for c in cells:
            for c2 in cells:
                parents_near = max(abs((a >> 1) - (b >> 1)) for a, b in zip(c, c2)) <= 1
                cells_apart = max(abs(a - b) for a, b in zip(c, c2)) >= 2
                if parents_near and cells_apart:
                    far.add((k, c, c2))
    lv = sorted({tuple(int(v) for v in c) for c in leaves})
    for c in lv:
        for c2 in lv:
            if max(abs(a - b) for a, b in zip(c, c2)) <= 1:
                near.add((c, c2))
    return far, near
