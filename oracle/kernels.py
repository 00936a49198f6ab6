"""Kernel functions (Table 1) and the grid entry function f_kappa.

All kernels are isotropic functions of r = ||x - y||_2 (Table 1).  Readings:

* Matern: the table prints Gamma(l) and B_nu; the standard Matern form is used,
  2^(1-nu) / Gamma(nu) * z^nu * K_nu(z) with z = sqrt(2 nu) r / l and K_nu the
  modified Bessel function of the second kind; kappa(r = 0) = 1 (its limit).
  theta = (l, nu) in that order when both are parameters.
* Closed forms for nu = 1/2 (Exponential), 3/2 and 5/2 are the textbook
  reductions of the general formula (half-integer K_nu).
* Thin-plate spline at r = 0 takes its limit 0.

Two test kernels that are not in the paper serve as pins:
* "poly":  (1 + theta (x . y))^3, degree 3 in every variable, so Chebyshev
  interpolation with n >= 4 nodes reproduces it exactly (Proposition 2,
  exact case p = n).
* "sep":   exp(sum_j x_j) * theta * exp(-sum_j y_j), a product of
  one-variable functions, so every TT rank of its grid tensor is 1.

The entry function of Section 1 ("Our approach") orders the variables as
xi = (x_1..x_d, theta_1..theta_dtheta, y_1..y_d); its value at a grid
multi-index is f_kappa at the Chebyshev nodes of each dimension
(Section 2.4, the entries m_{i_1..i_D} of the grid tensor).
"""
import math

import numpy as np
from scipy import special

from . import basis

PARAM_DIMS = {
    "se": 1, "exp": 1, "matern32": 1, "matern52": 1, "matern_nu": 1,
    "matern": 2, "mq": 1, "tps": 1,
    "laplace3d": 0, "laplace2d": 0, "biharmonic": 0, "thinplate": 0,
    "poly": 1, "sep": 1,
}


def matern_general(r, ell, nu):
    """2^(1-nu)/Gamma(nu) z^nu K_nu(z), z = sqrt(2 nu) r / ell; 1 at r = 0."""
    r, ell, nu = np.broadcast_arrays(np.asarray(r, float), np.asarray(ell, float),
                                     np.asarray(nu, float))
    z = np.sqrt(2.0 * nu) * r / ell
    out = np.ones_like(z)
    pos = z > 0
    zp = z[pos]
    nup = nu[pos]
    out[pos] = np.exp((1.0 - nup) * math.log(2.0) - special.gammaln(nup)) * zp ** nup * special.kv(nup, zp)
    return out


def kappa_r(kind, r, theta, const=None):
    """Kernel value as a function of distance r and parameter array theta (P, dtheta)."""
    r = np.asarray(r, dtype=np.float64)
    th = np.asarray(theta, dtype=np.float64)
    if kind == "se":
        ell = th[..., 0]
        return np.exp(-(r / ell) ** 2)
    if kind == "exp":
        return np.exp(-r / th[..., 0])
    if kind == "matern32":
        a = math.sqrt(3.0) * r / th[..., 0]
        return (1.0 + a) * np.exp(-a)
    if kind == "matern52":
        a = math.sqrt(5.0) * r / th[..., 0]
        return (1.0 + a + a * a / 3.0) * np.exp(-a)
    if kind == "matern_nu":
        return matern_general(r, th[..., 0], const)
    if kind == "matern":
        return matern_general(r, th[..., 0], th[..., 1])
    if kind == "mq":
        return np.sqrt(1.0 + (r / th[..., 0]) ** 2)
    if kind == "tps":
        u = (r / th[..., 0]) ** 2
        with np.errstate(divide="ignore", invalid="ignore"):
            v = u * np.log(u)
        return np.where(u > 0, v, 0.0)
    if kind == "laplace3d":
        return 1.0 / r
    if kind == "laplace2d":
        return -np.log(r)
    if kind == "biharmonic":
        return r ** -2.0
    if kind == "thinplate":
        return r * r * np.log(r)
    raise ValueError(f"kernel {kind!r} is not a function of r alone")


def kappa(kind, x, y, theta, const=None):
    """kappa(x, y; theta) for arrays x (P, d), y (P, d), theta (P, dtheta)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    th = np.asarray(theta, dtype=np.float64)
    if kind == "poly":
        return (1.0 + th[..., 0] * np.sum(x * y, axis=-1)) ** 3
    if kind == "sep":
        return np.exp(np.sum(x, axis=-1)) * th[..., 0] * np.exp(-np.sum(y, axis=-1))
    r = np.sqrt(np.sum((x - y) ** 2, axis=-1))
    return kappa_r(kind, r, th, const)


def dkappa_dtheta(kind, x, y, theta, const=None):
    """Analytic d kappa / d theta_j (P, dtheta) for the closed-form kernels.

    SE: 2 r^2 kappa / l^3.  Matern 3/2: a^2 e^-a / l with a = sqrt(3) r / l.
    Matern (l, nu): d/dl = 2^(1-nu)/Gamma(nu) z^(nu+1) K_(nu-1)(z) / l from
    d/dz [z^nu K_nu(z)] = -z^nu K_(nu-1)(z); d/dnu by a central difference of
    mpmath's besselk at 30 digits.
    """
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    th = np.asarray(theta, float)
    r = np.sqrt(np.sum((x - y) ** 2, axis=-1))
    ell = th[..., 0]
    if kind == "se":
        return (2.0 * r * r / ell ** 3 * np.exp(-(r / ell) ** 2))[..., None]
    if kind == "exp":
        return (r / ell ** 2 * np.exp(-r / ell))[..., None]
    if kind == "matern32":
        a = math.sqrt(3.0) * r / ell
        return (a * a * np.exp(-a) / ell)[..., None]
    if kind == "matern52":
        a = math.sqrt(5.0) * r / ell
        return (a * a * (1.0 + a) * np.exp(-a) / (3.0 * ell))[..., None]
    if kind in ("matern", "matern_nu"):
        nu = th[..., 1] if kind == "matern" else np.full_like(ell, const)
        z = np.sqrt(2.0 * nu) * r / ell
        dl = np.zeros_like(z)
        pos = z > 0
        dl[pos] = (np.exp((1.0 - nu[pos]) * math.log(2.0) - special.gammaln(nu[pos]))
                   * z[pos] ** (nu[pos] + 1.0) * special.kv(nu[pos] - 1.0, z[pos]) / ell[pos])
        if kind == "matern_nu":
            return dl[..., None]
        import mpmath
        mpmath.mp.dps = 30
        dnu = np.empty_like(z)
        for i, (ri, li, ni) in enumerate(zip(r.ravel(), ell.ravel(), nu.ravel())):
            def f(v):
                zz = mpmath.sqrt(2 * v) * ri / li
                if zz == 0:
                    return mpmath.mpf(1)
                return 2 ** (1 - v) / mpmath.gamma(v) * zz ** v * mpmath.besselk(v, zz)
            dnu.ravel()[i] = float(mpmath.diff(f, mpmath.mpf(ni)))
        return np.stack([dl, dnu], axis=-1)
    raise ValueError(f"no analytic derivative for {kind!r}")


class Problem:
    """A parametric kernel on boxes B_s x B_theta x B_t with per-dimension
    node counts, in the variable order xi = (x, theta, y).

    theta_fixed: the kernel's parameters held at these values, d_theta = 0
    (the non-parametric TTK method of Section 4.1, where H = I)."""

    def __init__(self, kind, d, box_s, box_t, box_theta, n_spatial, n_param=None,
                 const=None, theta_fixed=None):
        self.kind = kind
        self.d = int(d)
        self.theta_fixed = None if theta_fixed is None else np.asarray(theta_fixed, float).reshape(-1)
        if self.theta_fixed is not None:
            assert self.theta_fixed.size == PARAM_DIMS[kind]
            box_theta = []
        self.dt = 0 if self.theta_fixed is not None else PARAM_DIMS[kind]
        self.const = const
        self.box_s = np.asarray(box_s, float).reshape(self.d, 2)
        self.box_t = np.asarray(box_t, float).reshape(self.d, 2)
        self.box_theta = np.asarray(box_theta, float).reshape(self.dt, 2)
        n_param = n_spatial if n_param is None else n_param
        self.D = 2 * self.d + self.dt
        self.n = [n_spatial] * self.d + [n_param] * self.dt + [n_spatial] * self.d
        self.boxes = np.concatenate([self.box_s, self.box_theta, self.box_t], axis=0)
        self.nodes = [basis.grid_nodes(a, b, nj) for (a, b), nj in zip(self.boxes, self.n)]

    def coords(self, idx):
        """Grid multi-indices (P, D) -> (x, theta, y) coordinate arrays."""
        idx = np.asarray(idx, dtype=np.int64).reshape(-1, self.D)
        cols = [self.nodes[j][idx[:, j]] for j in range(self.D)]
        pts = np.stack(cols, axis=1) if cols else np.zeros((idx.shape[0], 0))
        d, dt = self.d, self.dt
        return pts[:, :d], pts[:, d:d + dt], pts[:, d + dt:]

    def entries(self, idx):
        """f_kappa at the Chebyshev grid multi-indices idx (P, D)."""
        x, th, y = self.coords(idx)
        if self.theta_fixed is not None:
            th = np.broadcast_to(self.theta_fixed, (x.shape[0], self.theta_fixed.size))
        return kappa(self.kind, x, y, th, self.const)

    def full_tensor(self):
        """The grid tensor M of Section 2.4 (tiny grids only)."""
        grids = np.meshgrid(*[np.arange(nj) for nj in self.n], indexing="ij")
        idx = np.stack([g.ravel() for g in grids], axis=1)
        return self.entries(idx).reshape(self.n)
