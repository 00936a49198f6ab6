"""Pins for the oracle's kernel table (Table 1) and entry function."""
import math
import os

import mpmath
import numpy as np
import pytest
from scipy import special

from oracle import kernels

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_bessel_table_values():
    with open(os.path.join(GOLD, "bessel_k.txt")) as fh:
        rows = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    for nu, z, v in rows:
        assert abs(special.kv(float(nu), float(z)) - float(v)) < 1e-9


@pytest.mark.parametrize("nu", [0.5, 0.77, 1.5, 2.0, 2.5])
def test_matern_general_vs_mpmath(nu):
    mpmath.mp.dps = 30
    r = np.array([1e-6, 0.01, 0.3, 1.0, 2.7, 7.0])
    ell = 0.9
    got = kernels.matern_general(r, ell, nu)
    for ri, gi in zip(r, got):
        z = mpmath.sqrt(2 * mpmath.mpf(nu)) * mpmath.mpf(ri) / mpmath.mpf(ell)
        ref = 2 ** (1 - mpmath.mpf(nu)) / mpmath.gamma(nu) * z ** nu * mpmath.besselk(nu, z)
        assert abs(gi - float(ref)) <= 1e-13 * abs(float(ref)) + 1e-300


def test_matern_closed_forms_match_general():
    r = np.linspace(0.0, 5.0, 101)
    th = np.full((101, 1), 1.3)
    assert np.allclose(kernels.kappa_r("exp", r, th), kernels.matern_general(r, 1.3, 0.5), rtol=1e-13, atol=0)
    assert np.allclose(kernels.kappa_r("matern32", r, th), kernels.matern_general(r, 1.3, 1.5), rtol=1e-13, atol=0)
    assert np.allclose(kernels.kappa_r("matern52", r, th), kernels.matern_general(r, 1.3, 2.5), rtol=1e-13, atol=0)


def test_matern_limit_at_zero():
    assert kernels.matern_general(0.0, 1.0, 1.7) == 1.0
    assert abs(kernels.matern_general(1e-9, 1.0, 1.7) - 1.0) < 1e-8


@pytest.mark.parametrize("kind,theta", [("se", [0.8]), ("matern32", [1.1]), ("matern52", [0.7]),
                                        ("exp", [1.4]), ("matern", [0.9, 1.3])])
def test_dkappa_dtheta_central_difference(kind, theta):
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, (6, 3))
    y = rng.uniform(2, 3, (6, 3))
    th = np.tile(theta, (6, 1))
    g = kernels.dkappa_dtheta(kind, x, y, th)
    for j in range(len(theta)):
        h = 1e-5
        tp, tm = th.copy(), th.copy()
        tp[:, j] += h
        tm[:, j] -= h
        fd = (kernels.kappa(kind, x, y, tp) - kernels.kappa(kind, x, y, tm)) / (2 * h)
        assert np.allclose(g[:, j], fd, rtol=1e-7, atol=1e-12)


def _laplacian(f, x, h=1e-3):
    """Five-point-per-axis finite-difference Laplacian (fourth order) of f at x (P, dim)."""
    out = np.zeros(x.shape[0])
    for j in range(x.shape[1]):
        e = np.zeros(x.shape[1])
        e[j] = h
        out += (-f(x + 2 * e) + 16 * f(x + e) - 30 * f(x) + 16 * f(x - e) - f(x - 2 * e)) / (12 * h * h)
    return out


@pytest.mark.parametrize("kind,dim", [("laplace3d", 3), ("laplace2d", 2), ("biharmonic", 4)])
def test_potential_kernels_are_harmonic(kind, dim):
    """Laplace-3D (1/r) and Laplace-2D (-log r) are the free-space Green's
    functions of the Laplacian in 3 and 2 dimensions, and r^-2 is harmonic in
    4 dimensions: their Laplacian vanishes away from r = 0.  A wrong power or
    a wrong log would not be."""
    rng = np.random.default_rng(0)
    x = rng.uniform(0.6, 1.4, (20, dim)) * rng.choice([-1, 1], (20, dim))
    f = lambda z: kernels.kappa_r(kind, np.sqrt((z ** 2).sum(axis=1)), np.zeros((z.shape[0], 0)))
    lap = _laplacian(f, x)
    scale = np.abs(f(x)) / (np.sqrt((x ** 2).sum(axis=1)) ** 2)      # size of each second-derivative term
    assert np.abs(lap).max() <= 1e-6 * scale.max()
    # and not harmonic one dimension off (the check has teeth)
    if dim > 2:
        f_low = lambda z: kernels.kappa_r(kind, np.sqrt((z ** 2).sum(axis=1)), np.zeros((z.shape[0], 0)))
        assert np.abs(_laplacian(f_low, x[:, :dim - 1])).max() > 1e-2 * scale.max()


def test_thinplate_is_biharmonic_in_2d():
    """r^2 log r is the Green's function of the biharmonic operator in 2-D:
    Delta^2 vanishes away from 0 (Delta(r^2 log r) = 4 log r + 4)."""
    rng = np.random.default_rng(1)
    x = rng.uniform(0.7, 1.3, (15, 2)) * rng.choice([-1, 1], (15, 2))
    f = lambda z: kernels.kappa_r("thinplate", np.sqrt((z ** 2).sum(axis=1)), np.zeros((z.shape[0], 0)))
    lap = lambda z: _laplacian(f, z, h=2e-3)
    r = np.sqrt((x ** 2).sum(axis=1))
    assert np.allclose(lap(x), 4 * np.log(r) + 4, rtol=0, atol=1e-6)
    assert np.abs(_laplacian(lap, x, h=2e-2)).max() <= 1e-3


def test_tps_extremum_and_zeros():
    """(r/l)^2 log((r/l)^2) = u log u with u = (r/l)^2: zero at r = l and at
    r -> 0, minimum -1/e at u = 1/e."""
    ell = 1.7
    th = np.array([[ell]])
    assert abs(kernels.kappa_r("tps", np.array([ell]), th)[0]) <= 1e-15
    assert kernels.kappa_r("tps", np.array([0.0]), th)[0] == 0.0
    r = np.linspace(1e-3, 2 * ell, 20001)
    v = kernels.kappa_r("tps", r, np.full((r.size, 1), ell))
    i = np.argmin(v)
    assert abs(v[i] + 1 / math.e) <= 1e-7 and abs(r[i] - ell / math.sqrt(math.e)) <= 2 * (r[1] - r[0])


def test_multiquadric_is_a_hyperbola():
    """sqrt(1 + (r/l)^2): its square is a quadratic in r with value 1 at 0 and
    2 at r = l (third differences of the square vanish)."""
    ell = 0.8
    r = np.linspace(0.0, 3.0, 31)
    v2 = kernels.kappa_r("mq", r, np.full((31, 1), ell)) ** 2
    assert np.abs(np.diff(v2, 3)).max() <= 1e-12
    assert abs(kernels.kappa_r("mq", np.array([ell]), np.array([[ell]]))[0] - math.sqrt(2.0)) <= 1e-15
    assert kernels.kappa_r("mq", np.array([0.0]), np.array([[ell]]))[0] == 1.0


def test_se_gaussian_integral():
    """The SE kernel integrates to (pi l^2)^(3/2) over R^3 (Gaussian integral),
    by radial quadrature of the oracle's values."""
    from scipy import integrate
    ell = 0.7
    val, _ = integrate.quad(lambda r: 4 * math.pi * r * r * kernels.kappa_r("se", np.array([r]),
                                                                            np.array([[ell]]))[0], 0, 20 * ell)
    assert abs(val - (math.pi * ell * ell) ** 1.5) <= 1e-10 * val


@pytest.mark.parametrize("nu,z", [(0.5, 1e-4), (1.1, 1e-3), (2.5, 1e-3), (1.1, 0.05), (0.5, 0.02)])
def test_bessel_small_argument(nu, z):
    """K_nu at small z (where the Matern kernel of coincident or near points
    sits) against mpmath at 30 digits, and the leading term
    Gamma(nu)/2 (2/z)^nu of its expansion."""
    mpmath.mp.dps = 30
    ref = float(mpmath.besselk(nu, z))
    assert abs(special.kv(nu, z) - ref) <= 1e-13 * ref
    lead = math.gamma(nu) / 2 * (2 / z) ** nu
    assert abs(ref / lead - 1) < 0.1


def test_entry_order_is_x_theta_y():
    P = kernels.Problem("sep", 2, [[0, 1], [0, 1]], [[2, 3], [0, 1]], [[0.5, 2.0]], 5)
    idx = np.array([[1, 2, 3, 4, 0]])
    x, th, y = P.coords(idx)
    assert np.isclose(x[0, 0], P.nodes[0][1]) and np.isclose(x[0, 1], P.nodes[1][2])
    assert np.isclose(th[0, 0], P.nodes[2][3])
    assert np.isclose(y[0, 0], P.nodes[3][4]) and np.isclose(y[0, 1], P.nodes[4][0])
    assert 2.0 < y[0, 0] < 3.0 and 0.5 < th[0, 0] < 2.0
    v = P.entries(idx)[0]
    assert np.isclose(v, math.exp(x.sum()) * th[0, 0] * math.exp(-y.sum()))
