"""Pins of the interaction-list oracle (oracle/pairs.py).

- The class reading (one TT per canonical pair geometry) rests on the grid
  tensor being invariant under translation, axis reflection and axis
  permutation for kernels of r = ||x - y||: checked entry by entry against
  the pair's own grid, with reflected axes reading the nodes backwards.
- The batched apply / backward are checked against the block-sparse matrix
  written out densely (a separate formulation), the adjoint identity and
  central differences in theta.
- A class TT applied to a pair matches dense K at the level of its tolerance.
"""
import numpy as np
import pytest

from oracle import dense, kernels, pairs


def _pair(c, o, h, ns, nt, d=3):
    c = np.asarray(c)
    t = c + np.asarray(o)
    return {"box_s": [[c[i] * h, (c[i] + 1) * h] for i in range(d)],
            "box_t": [[t[i] * h, (t[i] + 1) * h] for i in range(d)], "n_src": ns, "n_tgt": nt}


def test_frame_reproduces_pair_grid_entries():
    """Entries of the pair's own grid = canonical grid at permuted / reversed indices."""
    h = 0.25
    p = _pair([1, 0, 2], [-2, 3, 0], h, 1, 1)
    fr = pairs.frame(p["box_s"], p["box_t"])
    n = 6
    own = kernels.Problem("matern", 3, p["box_s"], p["box_t"], [[0.5, 2.0], [0.5, 2.5]], n, 5)
    can = kernels.Problem("matern", 3, fr["box_s"], fr["box_t"], [[0.5, 2.0], [0.5, 2.5]], n, 5)
    rng = np.random.default_rng(0)
    idx = np.stack([rng.integers(0, own.n[j], 300) for j in range(own.D)], axis=1)
    cidx = np.empty_like(idx)
    for j, i in enumerate(fr["perm"]):
        for side in (0, 5):                     # x axis j, y axis j (D = 8: x 0..2, theta 3..4, y 5..7)
            src = idx[:, side + i]
            cidx[:, side + j] = src if fr["sign"][j] > 0 else n - 1 - src
    cidx[:, 3:5] = idx[:, 3:5]
    a = own.entries(idx)
    b = can.entries(cidx)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
    # offsets in the canonical frame are non-negative and sorted with the sides
    assert fr["sign"][0] * (-2) != 0 and sorted(fr["key"]) == list(fr["key"])


def test_classes_dedupe_only_equal_geometry():
    h = 0.125
    ps = [_pair([0, 0, 0], [2, 0, 0], h, 5, 5), _pair([3, 3, 3], [0, -2, 0], h, 5, 5),
          _pair([1, 1, 1], [0, 0, 3], h, 5, 5), _pair([1, 1, 1], [2, 1, 0], h, 5, 5),
          _pair([4, 4, 4], [1, 0, -2], h, 5, 5)]
    cls, frames = pairs.classes(ps, "matern32")
    assert cls[0] == cls[1]                     # same |offset| pattern, other axis and sign
    assert cls[2] != cls[0]                     # distance 3 instead of 2
    assert cls[3] == cls[4]                     # (2, 1, 0) ~ (1, 0, -2) after permutation / reflection
    assert len(frames) == 3
    cls_p, frames_p = pairs.classes(ps, "poly")   # no invariance assumed for the test kernels
    assert len(frames_p) == len(ps)


def _small_batch(seed=0):
    rng = np.random.default_rng(seed)
    h = 0.25
    geo = [([0, 0], [2, 0]), ([3, 1], [-2, 0]), ([1, 1], [0, 2]), ([0, 3], [2, -1]), ([2, 2], [-1, -2])]
    ps, xs, ys = [], [], []
    so = to = 0
    for c, o in geo:
        ns, nt = int(rng.integers(3, 9)), int(rng.integers(3, 9))
        p = _pair(c, o, h, ns, nt, d=2)
        p.update(src_off=so, tgt_off=to)
        bs, bt = np.array(p["box_s"]), np.array(p["box_t"])
        xs.append(rng.uniform(bs[:, 0], bs[:, 1], (ns, 2)))
        ys.append(rng.uniform(bt[:, 0], bt[:, 1], (nt, 2)))
        so += ns
        to += nt
        ps.append(p)
    return ps, np.vstack(xs), np.vstack(ys)


def test_batched_apply_and_backward_against_dense_assembly():
    ps, X, Y = _small_batch()
    ob = pairs.offline("matern32", 2, [[0.5, 2.0]], 8, 8, ps, X, Y, 1e-7)
    assert len(ob["frames"]) < len(ps)          # some pairs share a class
    rng = np.random.default_rng(3)
    th = rng.uniform(0.5, 2.0, (3, 1))
    Hs, dHs = pairs.online(ob, th)
    xv = rng.standard_normal((Y.shape[0], 3))
    gv = rng.standard_normal((X.shape[0], 3))
    yv = pairs.apply(ob, ps, Hs, xv, X.shape[0])
    for b in range(3):
        K = pairs.assemble(ob, ps, [H[b] for H in Hs], X.shape[0], Y.shape[0])
        assert np.abs(K @ xv[:, b] - yv[:, b]).max() <= 1e-13 * np.abs(yv[:, b]).max()
    dX, dth = pairs.backward(ob, ps, Hs, dHs, xv, gv, Y.shape[0])
    # adjoint identity <dX_b, x_b> = <g_b, y_b>
    for b in range(3):
        assert abs(dX[:, b] @ xv[:, b] - gv[:, b] @ yv[:, b]) <= 1e-12 * abs(gv[:, b] @ yv[:, b]) + 1e-14
    # central differences in theta
    eps = 1e-5 * 1.5
    for b in range(3):
        f = lambda t: gv[:, b] @ pairs.apply(ob, ps, pairs.online(ob, [t])[0], xv[:, b:b + 1], X.shape[0])[:, 0]
        fd = (f(th[b] + eps) - f(th[b] - eps)) / (2 * eps)
        assert abs(fd - dth[b, 0]) <= 1e-7 * max(1.0, abs(dth[b, 0]))


def test_class_tt_matches_dense_kernel_per_pair():
    ps, X, Y = _small_batch(seed=1)
    ob = pairs.offline("matern32", 2, [[0.5, 2.0]], 10, 10, ps, X, Y, 1e-8)
    th = np.array([[0.8]])
    Hs, _ = pairs.online(ob, th)
    for i, p in enumerate(ps):
        K = dense.dense_K("matern32", X[p["src_off"]:p["src_off"] + p["n_src"]],
                          Y[p["tgt_off"]:p["tgt_off"] + p["n_tgt"]], th[0])
        Kh = ob["S"][i] @ Hs[ob["class"][i]][0] @ ob["T"][i].T
        # interpolation-limited level with n = 10 for boxes of side 1/4 whose centres are >= 2 sides
        # apart (about 1e-5 here, the same for every pair of a class)
        assert dense.rel_error(K, Kh) < 2e-5
