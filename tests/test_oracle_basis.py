"""Pins for the oracle's Chebyshev basis and RNG (Section 2.4; Lemma 1)."""
import os

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import basis, rng

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", [2, 5, 12, 16, 27])
def test_interpolation_at_nodes(n):
    """phi(eta_i, eta_j) = delta_ij (proof of Lemma 1)."""
    a, b = -0.3, 2.1
    q = basis.lagrange_values(basis.grid_nodes(a, b, n), a, b, n)
    assert np.abs(q - np.eye(n)).max() < 1e-13


@pytest.mark.parametrize("n", [3, 8, 16])
def test_equals_textbook_lagrange(n):
    """The Chebyshev-sum basis equals prod_{j != i} (x - eta_j)/(eta_i - eta_j)."""
    a, b = 0.5, 2.0
    eta = basis.grid_nodes(a, b, n)
    x = np.random.default_rng(1).uniform(a, b, 50)
    q = basis.lagrange_values(x, a, b, n)
    lag = np.ones((50, n))
    for i in range(n):
        for j in range(n):
            if j != i:
                lag[:, i] *= (x - eta[j]) / (eta[i] - eta[j])
    assert np.abs(q - lag).max() < 1e-11


def test_nodes_are_roots_of_Tn():
    for n in (4, 12, 16):
        z = basis.cheb_nodes(n)
        assert np.abs(np.cos(n * np.arccos(z))).max() < 1e-13
        assert np.allclose(np.sort(z), np.sort(npcheb.chebroots([0] * n + [1])), atol=1e-13)


def test_affine_orientation():
    """The printed map sends zeta_1 (largest) to alpha: eta ascends."""
    eta = basis.grid_nodes(2.0, 3.0, 7)
    assert np.all(np.diff(eta) > 0) and 2.0 < eta[0] < eta[-1] < 3.0


@pytest.mark.parametrize("n", [4, 12, 16, 27, 32])
def test_lebesgue_bound(n):
    """Lemma 1: max_x sum_k |phi(zeta_k, x)| <= (2/pi) log n + 1."""
    x = np.linspace(-1, 1, 20001)
    lam = basis.lebesgue_function(x, n).max()
    assert 1.0 <= lam <= 2.0 / np.pi * np.log(n) + 1.0


def test_partition_of_unity():
    x = np.random.default_rng(2).uniform(-1, 1, 100)
    assert np.abs(basis.lagrange_values(x, -1, 1, 14).sum(-1) - 1).max() < 1e-13


@pytest.mark.parametrize("n", [5, 12, 16])
def test_basis_change_matches_numpy_chebinterpolate(n):
    """C f equals the coefficients NumPy's first-kind Chebyshev interpolation gives."""
    f = lambda t: np.exp(0.7 * t) * np.sin(2 * t) + 1.0 / (2.5 - t)
    z = basis.cheb_nodes(n)
    coef = basis.basis_change(n) @ f(z)
    ref = npcheb.chebinterpolate(f, n - 1)
    assert np.abs(coef - ref).max() < 1e-13


def test_dT_matches_numpy_chebder():
    n = 12
    t = np.concatenate([np.linspace(-1, 1, 41), [-1.0, 1.0]])
    dT = basis.cheb_dT_table(n, t)
    for k in range(n):
        c = np.zeros(k + 1)
        c[k] = 1.0
        ref = npcheb.chebval(t, npcheb.chebder(c)) if k > 0 else np.zeros_like(t)
        assert np.abs(dT[k] - ref).max() < 1e-9 * max(1, k * k)


def test_lagrange_derivative_matches_central_difference():
    a, b, n = 0.5, 2.0, 12
    x = np.linspace(0.6, 1.9, 9)
    h = 1e-6
    fd = (basis.lagrange_values(x + h, a, b, n) - basis.lagrange_values(x - h, a, b, n)) / (2 * h)
    assert np.abs(fd - basis.lagrange_derivs(x, a, b, n)).max() < 1e-6


def test_splitmix64_published_vectors():
    with open(os.path.join(GOLD, "splitmix64.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            seed, outs = line.split(":")
            g = rng.SplitMix64(int(seed))
            assert [g.next() for _ in range(3)] == [int(v) for v in outs.split()]


def test_floyd_distinct_sorted_and_uniformish():
    g = rng.keyed(7, 2, 0, 1)
    s = g.floyd(100, 30)
    assert len(s) == 30 and len(set(s)) == 30 and s == sorted(s) and 0 <= s[0] and s[-1] < 100
    g = rng.keyed(7, 2, 0, 1)
    assert g.floyd(5, 5) == [0, 1, 2, 3, 4]
    counts = np.zeros(10)
    for i in range(2000):
        for v in rng.keyed(1, i).floyd(10, 3):
            counts[v] += 1
    assert counts.min() > 500 and counts.max() < 700


def test_below_range():
    g = rng.keyed(3, 1)
    v = [g.below(7) for _ in range(2000)]
    assert min(v) == 0 and max(v) == 6


# -------------------------------------------------- coefficient tensor
def test_coefficient_route_equals_lagrange_route():
    """The interpolant as sum_k A[k] prod T_k (A = DCT along every mode) equals
    sum_i M[i] prod l_i at random off-grid points (Section 2.4's regrouping)."""
    rng = np.random.default_rng(0)
    n = (5, 6, 4, 7)
    boxes = [(0.0, 1.0), (2.0, 3.5), (-1.0, 0.5), (0.5, 2.0)]
    M = rng.standard_normal(n)
    A = basis.coefficient_tensor(M)
    pts = np.stack([rng.uniform(a, b, 200) for a, b in boxes], axis=1)
    v_coef = basis.interpolant_coefficient_form(A, boxes, pts)
    v_lag = basis.interpolant_lagrange_form(M, boxes, pts)
    assert np.abs(v_coef - v_lag).max() <= 1e-13 * np.abs(v_lag).max()


def test_coefficient_tensor_recovers_known_coefficients():
    """Grid values of sum_k A0[k] prod T_k, formed with numpy's Chebyshev
    Vandermonde matrices at the nodes (t(eta_i) = zeta_i), give back A0."""
    rng = np.random.default_rng(1)
    n = (4, 7, 5)
    A0 = rng.standard_normal(n)
    M = A0
    for j, nj in enumerate(n):
        V = npcheb.chebvander(basis.cheb_nodes(nj), nj - 1)        # V[i, k] = T_k(zeta_i)
        M = np.moveaxis(np.tensordot(V, M, axes=([1], [j])), 0, j)
    assert np.abs(basis.coefficient_tensor(M) - A0).max() <= 1e-13 * np.abs(A0).max()


@pytest.mark.parametrize("n", [3, 8, 16])
def test_coefficients_match_numpy_chebinterpolate(n):
    """One mode against numpy's interpolation at first-kind Chebyshev points.
    On [-1, 1] the printed map sends zeta to -zeta, so t = -x and the
    coefficients differ by (-1)^k."""
    f = lambda x: np.exp(0.7 * x) * np.cos(2.0 * x)
    eta = basis.grid_nodes(-1.0, 1.0, n)
    ours = basis.coefficient_tensor(f(eta))
    ref = npcheb.chebinterpolate(f, n - 1)
    assert np.abs(ours - ref * (-1.0) ** np.arange(n)).max() <= 1e-14 * np.abs(ref).max() * n


def test_polynomial_kernel_has_no_high_coefficients():
    """(1 + theta x.y)^3 has degree 3 in each variable: every coefficient with
    an index above 3 in any mode vanishes (Proposition 2, exact case)."""
    from oracle import kernels
    P = kernels.Problem("poly", 1, [[0, 1]], [[2, 3]], [[0.5, 2.0]], 6)
    A = basis.coefficient_tensor(P.full_tensor())
    high = np.zeros(A.shape, bool)
    for j in range(A.ndim):
        idx = [slice(None)] * A.ndim
        idx[j] = slice(4, None)
        high[tuple(idx)] = True
    assert np.abs(A[high]).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(A[3, 3, 3]) > 1e-7 * np.abs(A).max()     # degree exactly 3 in each mode
