"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  Holds no arithmetic of the method: only workload descriptions,
point clouds, parameter samples and right-hand sides.

Points are drawn uniformly in float64 with numpy's PCG64 generator and, for
workloads whose bulk runs in float32, rounded to float32 so both sides see
the same coordinates.  The workloads mirror the paper's synthetic setups:
uniform points in unit boxes, separated boxes, Gaussian (SE) and Matern
kernels with length-scale and smoothness parameters.
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    kind: str                   # kernel name (oracle/kernels.py naming)
    d: int
    box_s: list
    box_t: list
    box_theta: list
    n_spatial: int
    n_param: int
    n_src: int
    n_tgt: int
    tol: float
    n_theta: int
    fp64: bool
    const: float = 0.0
    symmetric: bool = False
    extra: dict = field(default_factory=dict)

    @property
    def d_theta(self):
        return len(self.box_theta)


UNIT3 = [[0.0, 1.0]] * 3

WORKLOADS = {
    # Gaussian kernel, d = 2, float64 throughout.
    "se_d2_fp64": Workload("se_d2_fp64", "se", 2, [[0, 1], [0, 1]], [[2, 3], [0, 1]], [[0.5, 2.0]],
                           12, 12, 2000, 2000, 1e-8, 5, True),
    # Matern nu = 3/2 in the length scale, d = 3, separated unit cubes.  The
    # tolerance is set so that U M V^T is within 1e-5 (relative Frobenius) of
    # dense K; the error measured against dense K is about 9 x tol.
    "matern32_d3": Workload("matern32_d3", "matern32", 3, UNIT3, [[2, 3], [0, 1], [0, 1]], [[0.5, 2.0]],
                            16, 16, 100_000, 100_000, 7e-7, 16, False),
    # Symmetric PSD variant, X = Y in the unit cube, Matern (l, nu).
    "matern_global": Workload("matern_global", "matern", 3, UNIT3, UNIT3, [[0.5, 2.0], [0.5, 2.5]],
                              16, 12, 200_000, 200_000, 1e-5, 16, False, symmetric=True),
    # Batched + differentiated apply, Matern (l, nu), 1M points per side,
    # 16 nodes in every dimension (as the Matern 3/2 workload).  With 12
    # parameter nodes the interpolation in l alone leaves 1.5e-5..5.5e-5 near
    # l = 0.5; with 16, below 1e-6.  tol 7e-7 keeps U M V^T within 1e-5 of
    # dense K at every sampled theta; the cross needs about 250 sweeps.
    "matern_batched": Workload("matern_batched", "matern", 3, UNIT3, [[2, 3], [0, 1], [0, 1]],
                               [[0.5, 2.0], [0.5, 2.5]], 16, 16, 1_000_000, 1_000_000, 7e-7, 4096, False,
                               extra={"max_sweeps": 400}),
    # The non-parametric experiment of Section 4.1 (TTK, d_theta = 0): every
    # kernel of Table 1 with l = 1 (and Matern at nu = 3/2, 5/2), separated unit
    # cubes, 27 nodes per dimension, 10^4 points per side, tol 1e-9, float64.
    "ttk_e1": Workload("ttk_e1", "exp", 3, UNIT3, [[2, 3], [2, 3], [2, 3]], [], 27, 27, 10_000, 10_000, 1e-9,
                       1, True, extra={"kernels": [("exp", [1.0]), ("thinplate", None), ("biharmonic", None),
                                                   ("mq", [1.0]), ("tps", [1.0]), ("laplace2d", None),
                                                   ("laplace3d", None), ("matern32", [1.0]),
                                                   ("matern52", [1.0]), ("se", [1.0])]}),
}


def small(w: Workload, n_src, n_tgt, n_theta=None, **over):
    """A copy of workload w at smaller sizes (for parity tests)."""
    kw = dict(w.__dict__)
    kw.update(n_src=n_src, n_tgt=n_tgt, n_theta=w.n_theta if n_theta is None else n_theta)
    kw.update(over)
    return Workload(**kw)


def points(w: Workload, seed=0):
    """Source and target point clouds (N, d), uniform i.i.d. in their boxes."""
    rng = np.random.default_rng(seed)
    bs = np.asarray(w.box_s, float)
    bt = np.asarray(w.box_t, float)
    X = rng.uniform(bs[:, 0], bs[:, 1], (w.n_src, w.d))
    if w.symmetric:
        Y = X.copy()
    else:
        Y = rng.uniform(bt[:, 0], bt[:, 1], (w.n_tgt, w.d))
    if not w.fp64:
        X = X.astype(np.float32).astype(np.float64)
        Y = Y.astype(np.float32).astype(np.float64)
        # rounding may step a coordinate just past the box edge; clamp it back
        X = np.clip(X, bs[:, 0], bs[:, 1])
        Y = np.clip(Y, (bs if w.symmetric else bt)[:, 0], (bs if w.symmetric else bt)[:, 1])
    return X, Y


def thetas(w: Workload, count=None, seed=1):
    """Parameter samples uniform over the parameter box."""
    rng = np.random.default_rng(seed)
    bt = np.asarray(w.box_theta, float)
    c = w.n_theta if count is None else count
    th = rng.uniform(bt[:, 0], bt[:, 1], (c, w.d_theta))
    if not w.fp64:
        th = np.clip(th.astype(np.float32).astype(np.float64), bt[:, 0], bt[:, 1])
    return th


def rhs(n, count, seed=2, fp64=False):
    """Right-hand sides / cotangents: N(0, 1), column-major (n, count)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, count))
    if not fp64:
        v = v.astype(np.float32).astype(np.float64)
    return v


def uneven_pairs(num_pairs=512, seed=5, lo=1000, hi=64000):
    """FMM-like interaction list in [0,1]^3: level k in {2..5}, source cell c,
    offset o in {-3..3}^3 with max|o_i| >= 2 (well separated), rejecting target
    cells outside the cube; point counts log-uniform in [lo, hi] per box."""
    rng = np.random.default_rng(seed)
    pairs = []
    while len(pairs) < num_pairs:
        k = int(rng.integers(2, 6))
        m = 2 ** k
        c = rng.integers(0, m, 3)
        o = rng.integers(-3, 4, 3)
        if np.max(np.abs(o)) < 2:
            continue
        t = c + o
        if np.any(t < 0) or np.any(t >= m):
            continue
        h = 1.0 / m
        ns = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        nt = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        pairs.append({"level": k, "offset": tuple(int(v) for v in o),
                      "box_s": [[c[i] * h, (c[i] + 1) * h] for i in range(3)],
                      "box_t": [[t[i] * h, (t[i] + 1) * h] for i in range(3)],
                      "n_src": ns, "n_tgt": nt})
    return pairs
