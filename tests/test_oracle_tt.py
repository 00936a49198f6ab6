"""Pins for the oracle's TT helpers: unfoldings (Section 2.2), the
unfolding-by-cores formula and TT-Round (Section 2.3, Algorithm 1), and the
mixed-product rules of Section 2.1."""
import numpy as np
import pytest

from oracle import tt


def test_little_endian_unfolding_definition():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((2, 3, 4, 5))
    U = tt.unfold(X, 2)
    for i1 in range(2):
        for i2 in range(3):
            for i3 in range(4):
                for i4 in range(5):
                    assert U[i1 + i2 * 2, i3 + i4 * 4] == X[i1, i2, i3, i4]


def test_full_matches_entry_formula():
    rng = np.random.default_rng(1)
    cores = tt.random_tt(rng, [3, 4, 2, 3], [2, 3, 2])
    X = tt.full(cores)
    idx = np.array([[1, 2, 0, 2], [2, 3, 1, 0], [0, 0, 0, 0]])
    for row in idx:
        v = np.eye(1)
        for k, i in enumerate(row):
            v = v @ cores[k][:, i, :]
        assert np.isclose(X[tuple(row)], v[0, 0])
    assert np.allclose(tt.evaluate(cores, idx), [X[tuple(r)] for r in idx])


@pytest.mark.parametrize("j", [1, 2, 3])
def test_unfolding_in_terms_of_cores(j):
    """X^{j} = prod_{i<j} (I kron G_i^{2}) G_j^{2} G_{j+1}^{1} prod_{i>j+1} (G_i^{1} kron I)."""
    rng = np.random.default_rng(2)
    n = [2, 3, 2, 3]
    cores = tt.random_tt(rng, n, [2, 3, 2])
    X = tt.full(cores)
    N = len(n)
    left = np.eye(int(np.prod(n[:j])))
    for i in range(1, j):
        left = left @ np.kron(np.eye(int(np.prod(n[i:j]))), tt.g2(cores[i - 1]))
    left = left @ tt.g2(cores[j - 1])
    right = tt.g1(cores[j])
    for i in range(j + 2, N + 1):
        right = right @ np.kron(tt.g1(cores[i - 1]), np.eye(int(np.prod(n[j:i - 1]))))
    assert np.allclose(left @ right, tt.unfold(X, j), atol=1e-12)


def test_mixed_product_rules():
    rng = np.random.default_rng(3)
    s, m, p, k, q = 3, 4, 2, 5, 6
    G = rng.standard_normal((s, m))
    H = rng.standard_normal((p, k))
    A = rng.standard_normal((s, q))
    B = rng.standard_normal((p, q))

    def kr(P, Q):
        return np.stack([np.kron(P[:, i], Q[:, i]) for i in range(P.shape[1])], axis=1)

    lhs = np.kron(G.T, H.T) @ kr(A, B)
    assert np.allclose(lhs, kr(G.T @ A, H.T @ B))
    # (A^T face-split B^T)(G kron H) = (A^T G) face-split (B^T H), with
    # P^T face-split Q^T = (P khatri-rao Q)^T
    lhs2 = kr(A, B).T @ np.kron(G, H)
    assert np.allclose(lhs2, kr(G.T @ A, H.T @ B).T)


def test_tt_svd_recovers_exact_ranks():
    rng = np.random.default_rng(4)
    cores = tt.random_tt(rng, [4, 5, 4, 3], [2, 3, 2])
    X = tt.full(cores)
    c2 = tt.tt_svd(X, 1e-12)
    assert tt.ranks(c2) == [1, 2, 3, 2, 1]
    assert np.linalg.norm(tt.full(c2) - X) <= 1e-12 * np.linalg.norm(X)


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-8])
def test_tt_round_guarantee(eps):
    """||X - X^||_F <= eps ||X||_F (Algorithm 1's guarantee)."""
    rng = np.random.default_rng(5)
    cores = tt.random_tt(rng, [5, 6, 5, 4], [4, 6, 4])
    for c in cores:
        c *= np.exp(-np.arange(c.shape[2]))[None, None, :]
    X = tt.full(cores)
    R = tt.tt_round(cores, eps)
    err = np.linalg.norm(tt.full(R) - X)
    assert err <= eps * np.linalg.norm(X) * (1 + 1e-10)
    assert max(tt.ranks(R)) <= max(tt.ranks(cores))


def test_tt_round_doubled_tt_returns_to_rank():
    """X + X written as a rank-2r TT rounds back to rank r."""
    rng = np.random.default_rng(6)
    n = [4, 5, 4]
    cores = tt.random_tt(rng, n, [2, 3])
    dbl = []
    for k, G in enumerate(cores):
        r0, nn, r1 = G.shape
        if k == 0:
            dbl.append(np.concatenate([G, G], axis=2))
        elif k == len(cores) - 1:
            dbl.append(np.concatenate([G, G], axis=0))
        else:
            Z = np.zeros((2 * r0, nn, 2 * r1))
            Z[:r0, :, :r1] = G
            Z[r0:, :, r1:] = G
            dbl.append(Z)
    X2 = tt.full(dbl)
    assert np.allclose(X2, 2 * tt.full(cores))
    R = tt.tt_round(dbl, 1e-12)
    assert tt.ranks(R) == [1, 2, 3, 1]
    assert np.allclose(tt.full(R), X2, atol=1e-11 * np.abs(X2).max())


def test_tt_round_leaves_left_orthonormal_cores():
    rng = np.random.default_rng(7)
    cores = tt.random_tt(rng, [4, 4, 4, 4], [3, 4, 3])
    R = tt.tt_round(cores, 1e-10)
    for G in R[:-1]:
        M = tt.g2(G)
        assert np.allclose(M.T @ M, np.eye(M.shape[1]), atol=1e-12)
