"""GPU parity of the parametric hierarchical matrix (tt_kernel_hmat_*):
the block partition against the oracle's (oracle/hmat.py, bit-exact: index
work), the sort of the points (a permutation in Morton order of the oracle's
leaf cells), and H(theta) x against dense K(X, X; theta) x from the oracle.

The far blocks are PTTK low-rank blocks (the pair batch, whose per-pair
parity with oracle/pairs.py is tested in test_gpu_batch.py); the near blocks
are exact, so ||H x - K x|| / ||K x|| is set by the far blocks'
approximation: the Chebyshev interpolation at n nodes (in space and in the
parameters) and the TT truncation at tol.  The parameter boxes are chosen
where n nodes resolve the kernel (the Gaussian at l = 0.5 with 12 nodes
leaves about 1e-5 of interpolation error, as the oracle's own error for
that kernel shows); asserted within 1e-5 (float32 bulk) or 1e-7 (float64)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import dense as odense
from oracle import hmat as ohmat


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


CASES = [
    # kind, d, box_theta, n, tol, N, leaf_points, dtype, bar
    ("se", 2, [[1.0, 2.0]], 12, 1e-9, 3000, 40, "f64", 1e-7),
    ("matern32", 3, [[0.5, 2.0]], 12, 1e-7, 4000, 64, "f32", 1e-5),
    ("matern", 2, [[0.5, 2.0], [1.5, 2.5]], 14, 1e-8, 2500, 24, "f32", 1e-5),
]


@pytest.mark.parametrize("kind,d,bth,n,tol,N,leaf,dtype,bar", CASES)
def test_hmatrix_partition_and_apply_match_oracle(kind, d, bth, n, tol, N, leaf, dtype, bar):
    torch = _torch()
    import paper_2406_06344_amd as pkg
    say(f"[hmat] {kind} d={d} N={N} leaf={leaf} {dtype}")
    rng = np.random.default_rng(N)
    X = rng.uniform(0, 1, (N, d))
    if dtype == "f32":
        X = X.astype(np.float32).astype(np.float64)
    box = [[0.0, 1.0]] * d
    tdt = torch.float64 if dtype == "f64" else torch.float32
    H = pkg.HMatrix.build(torch.tensor(X), kind, d, box, bth, leaf_points=leaf, n_spatial=n, n_param=n, tol=tol,
                          dtype=tdt)
    inf = H.info()
    L = ohmat.leaf_level(N, d, leaf)
    say(f"  levels {inf['levels']} (oracle {L}), far {inf['far_pairs']}, near {inf['near_pairs']}, "
        f"classes {inf['num_classes']}")
    assert inf["levels"] == L
    far, near, perm = H.lists()
    far_o, near_o = ohmat.partition(X, box, L)
    far_g = {(int(r[0]), tuple(int(v) for v in r[1:1 + d]), tuple(int(v) for v in r[4:4 + d])) for r in far}
    near_g = {(tuple(int(v) for v in r[:d]), tuple(int(v) for v in r[3:3 + d])) for r in near}
    assert len(far_g) == len(far) and len(near_g) == len(near)
    assert far_g == far_o and near_g == near_o
    # the sort: a permutation, in Morton order of the oracle's leaf cells
    assert np.array_equal(np.sort(perm), np.arange(N))
    codes = ohmat.morton(ohmat.leaf_cells(X, box, L), L)[perm]
    assert np.all(np.diff(codes) >= 0)
    # H(theta) x against dense K x
    bt = np.asarray(bth, float)
    ths = np.stack([bt[:, 0], bt.mean(axis=1), bt[:, 1]])
    xs = rng.standard_normal((3, N))
    Y = H.apply(torch.tensor(ths, dtype=tdt), torch.tensor(xs, dtype=tdt)).double().cpu().numpy()
    errs = []
    for b in range(3):
        K = odense.dense_K(kind, X, X, ths[b])
        ref = K @ xs[b]
        errs.append(float(np.linalg.norm(Y[b] - ref) / np.linalg.norm(ref)))
        say(f"  theta {ths[b]}: |Hx - Kx| / |Kx| = {errs[-1]:.2e}")
    assert max(errs) <= bar


def test_hmatrix_argument_errors():
    torch = _torch()
    import paper_2406_06344_amd as pkg
    from paper_2406_06344_amd._lib import TTKError
    X = torch.rand(100, 2, dtype=torch.float64)
    with pytest.raises(ValueError):
        pkg.HMatrix.build(X, "se", 2, [[0, 1], [0, 1]], [[0.5, 2.0]], leaf_points=0, n_spatial=8, tol=1e-6,
                          dtype=torch.float64)
    with pytest.raises(TTKError, match="ERR_ARG"):
        pkg.HMatrix.build(X, "se", 2, [[0, 1], [1, 1]], [[0.5, 2.0]], leaf_points=8, n_spatial=8, tol=1e-6,
                          dtype=torch.float64)
    H = pkg.HMatrix.build(X, "se", 2, [[0, 1], [0, 1]], [[0.5, 2.0]], leaf_points=200, n_spatial=8, tol=1e-6,
                          dtype=torch.float64)
    assert H.info()["levels"] == 0 and H.info()["far_pairs"] == 0   # one leaf: all near
    th = torch.tensor([[1.0]], dtype=torch.float64)
    x = torch.randn(1, 100, dtype=torch.float64)
    Xn = X.numpy()
    ref = odense.dense_K("se", Xn, Xn, np.array([1.0])) @ x.numpy()[0]
    y = H.apply(th, x).cpu().numpy()[0]
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    with pytest.raises(ValueError):
        H.apply(th, torch.randn(1, 99, dtype=torch.float64))
