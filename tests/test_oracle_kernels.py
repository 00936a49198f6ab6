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


def test_kernel_table_closed_forms():
    r = np.array([0.5, 1.0, 2.0])
    th = np.array([[2.0]] * 3)
    assert np.allclose(kernels.kappa_r("se", r, th), np.exp(-(r / 2) ** 2))
    assert np.allclose(kernels.kappa_r("mq", r, th), np.sqrt(1 + (r / 2) ** 2))
    assert np.allclose(kernels.kappa_r("tps", r, th), (r / 2) ** 2 * np.log((r / 2) ** 2))
    assert np.allclose(kernels.kappa_r("laplace3d", r, th), 1 / r)
    assert np.allclose(kernels.kappa_r("laplace2d", r, th), -np.log(r))
    assert np.allclose(kernels.kappa_r("biharmonic", r, th), r ** -2)
    assert np.allclose(kernels.kappa_r("thinplate", r, th), r * r * np.log(r))


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
