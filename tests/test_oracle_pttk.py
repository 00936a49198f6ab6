"""Pins for the oracle's PTTK stages (Section 3)."""
import numpy as np
import pytest

from oracle import basis, cross, dense, driver, kernels, pttk, tt


def _tiny(kind="matern32", d=2, n=5, box_t=None):
    box_t = [[2, 3]] * d if box_t is None else box_t
    return kernels.Problem(kind, d, [[0, 1]] * d, box_t, [[0.5, 2.0]] * kernels.PARAM_DIMS[kind], n)


def test_phase3_recursion_equals_explicit_product():
    """S = F_s L and T = F_t R (Section 3.1): the recursion of Algorithm 2
    against the explicit face-splitting / Kronecker formulas."""
    rng = np.random.default_rng(0)
    d, n = 3, 4
    cs = tt.random_tt(rng, [n] * d + [n] * d, [3, 5, 4, 5, 3])
    cores_s = cs[:d]
    cores_s[-1] = cores_s[-1]
    cores_t = cs[d:]
    X = rng.uniform(0, 1, (13, d))
    Y = rng.uniform(2, 3, (11, d))
    box_s = np.array([[0, 1]] * d, float)
    box_t = np.array([[2, 3]] * d, float)
    U = pttk.factor_values(X, box_s, n)
    V = pttk.factor_values(Y, box_t, n)
    S = pttk.phase3_source(U, cores_s)
    T = pttk.phase3_target(V, cores_t)
    Se, Te = pttk.phase3_explicit(U, V, cores_s, cores_t, n)
    assert np.abs(S - Se).max() <= 1e-13 * np.abs(Se).max()
    assert np.abs(T - Te).max() <= 1e-13 * np.abs(Te).max()


def test_low_rank_form_equals_full_grid_interpolant():
    """With exact cores (TT-SVD at 1e-14) S H(theta) T^T equals the full
    interpolant F_s M_F^{d}(theta) F_t^T of Section 2.4 (both built here from
    their definitions)."""
    P = _tiny("matern32", d=2, n=5)
    M = P.full_tensor()
    cores = tt.tt_svd(M, 1e-14)
    G = pttk.round_and_gauge(cores, 1e-15, 2, 1)
    rng = np.random.default_rng(1)
    X = rng.uniform(0, 1, (9, 2))
    Y = rng.uniform(2, 3, (7, 2))
    U = pttk.factor_values(X, P.box_s, 5)
    V = pttk.factor_values(Y, P.box_t, 5)
    S = pttk.phase3_source(U, G[:2])
    T = pttk.phase3_target(V, G[3:])
    for th in (0.6, 1.7):
        H = pttk.online_H(G[2:3], [th], P.box_theta, 5)
        q = basis.lagrange_values(np.array(th), 0.5, 2.0, 5)
        MF = np.einsum("abcde,c->abde", M, q)
        Fs = pttk.face_split([U[1], U[0]])
        Ft = pttk.face_split([V[1], V[0]])
        K = Fs @ tt.unfold(MF, 2) @ Ft.T
        assert np.abs(S @ H @ T.T - K).max() <= 1e-12 * np.abs(K).max()


def test_interpolant_matches_kernel_at_grid_nodes():
    """Pin (b) on the full grid: at source/target points on the nodes and theta
    on a node, the interpolant equals kappa."""
    P = _tiny("se", d=2, n=6)
    M = P.full_tensor()
    G = pttk.round_and_gauge(tt.tt_svd(M, 1e-15), 1e-15, 2, 1)
    X = np.array([[P.nodes[0][i], P.nodes[1][j]] for i in range(6) for j in range(6)])
    Y = np.array([[P.nodes[3][i], P.nodes[4][j]] for i in range(6) for j in range(0, 6, 2)])
    S = pttk.phase3_source(pttk.factor_values(X, P.box_s, 6), G[:2])
    T = pttk.phase3_target(pttk.factor_values(Y, P.box_t, 6), G[3:])
    th = P.nodes[2][3]
    H = pttk.online_H(G[2:3], [th], P.box_theta, 6)
    K = dense.dense_K("se", X, Y, [th])
    assert np.abs(S @ H @ T.T - K).max() <= 1e-12 * np.abs(K).max()


def test_gauge_orthonormality_and_invariance():
    P = _tiny("matern", d=2, n=5)
    M = P.full_tensor()
    c = tt.tt_svd(M, 1e-10)
    G = pttk.round_and_gauge(c, 1e-12, 2, 2)
    for g in G[:3]:
        A = tt.g2(g)
        assert np.allclose(A.T @ A, np.eye(A.shape[1]), atol=1e-12)
    for g in G[4:]:
        A = tt.g1(g)
        assert np.allclose(A @ A.T, np.eye(A.shape[0]), atol=1e-12)
    assert np.linalg.norm(tt.full(G) - M) <= 2e-10 * np.linalg.norm(M)
    for g in G[:3]:
        A = tt.g2(g)
        piv = np.argmax(np.abs(A), axis=0)
        assert np.all(A[piv, np.arange(A.shape[1])] > 0)


def test_online_H_equals_contraction_of_parameter_modes():
    P = _tiny("matern", d=1, n=6)
    M = P.full_tensor()
    G = pttk.round_and_gauge(tt.tt_svd(M, 1e-14), 1e-15, 1, 2)
    th = [0.83, 1.91]
    H = pttk.online_H(G[1:3], th, P.box_theta, 6)
    q1 = basis.lagrange_values(np.array(th[0]), 0.5, 2.0, 6)
    q2 = basis.lagrange_values(np.array(th[1]), 0.5, 2.0, 6)
    MF = np.einsum("abcd,b,c->ad", M, q1, q2)
    assert np.abs(tt.g2(G[0]) @ H @ tt.g1(G[3]) - MF).max() <= 1e-12 * np.abs(MF).max()


def test_dH_central_difference_and_exact_for_polynomial():
    P = _tiny("matern", d=1, n=8)
    M = P.full_tensor()
    G = pttk.round_and_gauge(tt.tt_svd(M, 1e-13), 1e-14, 1, 2)
    th = np.array([1.1, 1.4])
    dH = pttk.online_dH(G[1:3], th, P.box_theta, 8)
    for j in range(2):
        h = 1e-5 * 1.5
        tp, tm = th.copy(), th.copy()
        tp[j] += h
        tm[j] -= h
        fd = (pttk.online_H(G[1:3], tp, P.box_theta, 8) - pttk.online_H(G[1:3], tm, P.box_theta, 8)) / (2 * h)
        assert np.abs(fd - dH[j]).max() <= 1e-7 * np.abs(dH[j]).max()
    # polynomial kernel: interpolant is exact, so dH gives d kappa / d theta exactly
    Pp = kernels.Problem("poly", 1, [[0, 1]], [[2, 3]], [[0.5, 2.0]], 5)
    Gp = pttk.round_and_gauge(tt.tt_svd(Pp.full_tensor(), 1e-14), 1e-15, 1, 1)
    X = np.array([[0.3], [0.8]])
    Y = np.array([[2.2], [2.9], [2.5]])
    S = pttk.phase3_source(pttk.factor_values(X, Pp.box_s, 5), Gp[:1])
    T = pttk.phase3_target(pttk.factor_values(Y, Pp.box_t, 5), Gp[2:])
    t0 = 1.3
    dHp = pttk.online_dH(Gp[1:2], [t0], Pp.box_theta, 5)[0]
    exact = 3 * (1 + t0 * X @ Y.T) ** 2 * (X @ Y.T)
    assert np.abs(S @ dHp @ T.T - exact).max() <= 1e-10 * np.abs(exact).max()


def test_apply_backward_adjoint_and_fd():
    P = _tiny("matern", d=2, n=5)
    G = pttk.round_and_gauge(tt.tt_svd(P.full_tensor(), 1e-10), 1e-11, 2, 2)
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 1, (20, 2))
    Y = rng.uniform(2, 3, (17, 2))
    S = pttk.phase3_source(pttk.factor_values(X, P.box_s, 5), G[:2])
    T = pttk.phase3_target(pttk.factor_values(Y, P.box_t, 5), G[4:])
    B = 4
    thetas = rng.uniform([0.5, 0.5], [2.0, 2.0], (B, 2))
    Xb = rng.standard_normal((17, B))
    Gb = rng.standard_normal((20, B))
    Hs = [pttk.online_H(G[2:4], t, P.box_theta, 5) for t in thetas]
    dHs = [pttk.online_dH(G[2:4], t, P.box_theta, 5) for t in thetas]
    Yb, W = pttk.apply_batched(S, Hs, T, Xb)
    for b in range(B):
        assert np.allclose(Yb[:, b], pttk.apply(S, Hs[b], T, Xb[:, b]), rtol=1e-13, atol=1e-14)
    dX, dth = pttk.backward_batched(S, Hs, dHs, T, Xb, Gb)
    # adjoint identity <dX_b, x_b> = <g_b, y_b>
    for b in range(B):
        assert abs(dX[:, b] @ Xb[:, b] - Gb[:, b] @ Yb[:, b]) <= 1e-12 * abs(Gb[:, b] @ Yb[:, b]) + 1e-14
    # central differences on L in theta
    for b in range(B):
        for j in range(2):
            h = 1e-5
            tp, tm = thetas[b].copy(), thetas[b].copy()
            tp[j] += h
            tm[j] -= h
            Lp = Gb[:, b] @ pttk.apply(S, pttk.online_H(G[2:4], tp, P.box_theta, 5), T, Xb[:, b])
            Lm = Gb[:, b] @ pttk.apply(S, pttk.online_H(G[2:4], tm, P.box_theta, 5), T, Xb[:, b])
            assert abs((Lp - Lm) / (2 * h) - dth[b, j]) <= 1e-7 * max(1.0, abs(dth[b, j]))


def test_ttk_special_case_identity_core():
    """dtheta = 0: H = I and the apply is S T^T x (Section 4.1)."""
    P = kernels.Problem("laplace3d", 1, [[0, 1]], [[2, 3]], [], 8)
    G = pttk.round_and_gauge(tt.tt_svd(P.full_tensor(), 1e-13), 1e-14, 1, 0)
    X = np.array([[0.1], [0.5], [0.9]])
    Y = np.array([[2.3], [2.7]])
    S = pttk.phase3_source(pttk.factor_values(X, P.box_s, 8), G[:1])
    T = pttk.phase3_target(pttk.factor_values(Y, P.box_t, 8), G[1:])
    K = 1.0 / np.abs(X - Y.T)
    assert S.shape[1] == T.shape[1]
    assert np.abs(S @ T.T - K).max() <= 1e-5 * np.abs(K).max()


def test_global_symmetric_part_identity_and_psd():
    """Symmetric-part identity of Section 3.5 and Algorithm 4's W >= 0."""
    P = kernels.Problem("se", 1, [[0, 1]], [[0, 1]], [[0.3, 1.0]], 8)
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 1, (30, 1))
    out = driver.offline(P, X, X, 1e-8, seed=0)
    S, T = out["S"], out["T"]
    Q, R = pttk.global_offline(S, T)
    th = 0.55
    H = pttk.online_H(out["param"], [th], P.box_theta, 8)
    rs = S.shape[1]
    Hh = np.zeros((rs + T.shape[1],) * 2)
    Hh[:rs, rs:] = H / 2
    Hh[rs:, :rs] = H.T / 2
    lhs = 0.5 * (S @ H @ T.T + T @ H.T @ S.T)
    ST = np.hstack([S, T])
    assert np.abs(lhs - ST @ Hh @ ST.T).max() <= 1e-13 * np.abs(lhs).max()
    W, nneg = pttk.global_online(R, H, rs)
    A = Q @ W @ Q.T
    assert np.allclose(A, A.T, atol=1e-14)
    lam = np.linalg.eigvalsh(W)
    assert lam.min() >= -1e-12 * np.abs(lam).max()
    K = dense.dense_K("se", X, X, [th])
    assert dense.rel_error(K, A) < 1e-3          # interpolation-level report, n = 8
    (Uc, Lc), _ = pttk.global_online(R, H, rs, compress=True, eps=1e-6)
    Z = Q @ Uc
    assert dense.rel_error(A, Z @ np.diag(Lc) @ Z.T) <= 1e-6 * 1.01 * np.linalg.norm(A) / np.linalg.norm(A)


def test_storage_formula_counts_the_stored_arrays():
    """Section 3.2's storage count equals the number of floats the offline
    stage actually produces (S, T and the parameter cores)."""
    P = _tiny("matern", d=2, n=5)
    rng = np.random.default_rng(8)
    X = rng.uniform(0, 1, (23, 2))
    Y = rng.uniform(2, 3, (19, 2))
    out = driver.offline(P, X, Y, 1e-6, seed=0)
    stored = out["S"].size + out["T"].size + sum(G.size for G in out["param"])
    assert pttk.storage_floats(23, 19, out["ranks"], 5, 2, 2) == stored


def test_sign_rule_on_both_sides():
    """R10: after the gauge, every column of a source/parameter core's G^{2}
    and every row of a target core's G^{1} has its largest-|.| entry positive
    (lowest index on ties); flipping signs by hand and re-applying the rule
    restores the cores, and the represented tensor never changes."""
    P = _tiny("matern", d=2, n=5)
    M = P.full_tensor()
    G = pttk.round_and_gauge(tt.tt_svd(M, 1e-10), 1e-12, 2, 2)
    for g in G[4:]:
        A = tt.g1(g)
        piv = np.argmax(np.abs(A), axis=1)
        assert np.all(A[np.arange(A.shape[0]), piv] > 0)
    rng = np.random.default_rng(9)
    s = rng.choice([-1.0, 1.0], G[5].shape[0])
    s[0] = -1.0
    flipped = G[5] * s[:, None, None]                   # flip rows of the last target core ...
    prev = G[4] * s[None, None, :]                      # ... and compensate in its left neighbour
    Gf = G[:4] + [prev, flipped]
    assert np.linalg.norm(tt.full(Gf) - tt.full(G)) <= 1e-13 * np.linalg.norm(M)
    g5, g4 = pttk.sign_fix_right(flipped, prev)
    assert np.array_equal(g5, G[5]) and np.array_equal(g4, G[4])
    # ties go to the lowest index: a row whose two largest entries are +-m
    T = np.zeros((2, 3, 1))
    T[0, :, 0] = [-2.0, 2.0, 1.0]
    T[1, :, 0] = [1.0, 3.0, -3.0]
    Pv = np.ones((1, 2, 2))
    Tf, Pf = pttk.sign_fix_right(T, Pv)
    assert Tf[0, 0, 0] == 2.0 and Tf[1, 1, 0] == 3.0 and Pf[0, 0, 0] == -1.0 and Pf[0, 0, 1] == 1.0


def test_paper_phase4_preserves_product():
    P = _tiny("matern32", d=2, n=6)
    rng = np.random.default_rng(5)
    X = rng.uniform(0, 1, (40, 2))
    Y = rng.uniform(2, 3, (40, 2))
    out = driver.offline(P, X, Y, 1e-8, seed=1)
    S2, param2, T2 = pttk.phase4_paper(out["S"], out["param"], out["T"], 1e-8)
    for th in (0.7, 1.9):
        H1 = pttk.online_H(out["param"], [th], P.box_theta, 6)
        H2 = pttk.online_H(param2, [th], P.box_theta, 6)
        A = out["S"] @ H1 @ out["T"].T
        assert dense.rel_error(A, S2 @ H2 @ T2.T) <= 1e-6
    assert S2.shape[1] <= out["S"].shape[1]


def test_dense_brute_force_small_se():
    """Pin (d) as a report: the end-to-end error against dense K at tol 1e-8 on
    a tiny d = 1 problem (the level is empirical in the paper)."""
    P = kernels.Problem("se", 1, [[0, 1]], [[2, 3]], [[0.5, 2.0]], 12)
    rng = np.random.default_rng(6)
    X = rng.uniform(0, 1, (200, 1))
    Y = rng.uniform(2, 3, (200, 1))
    out = driver.offline(P, X, Y, 1e-8, seed=0)
    for th in (1.0, 2.0):
        H = pttk.online_H(out["param"], [th], P.box_theta, 12)
        K = dense.dense_K("se", X, Y, [th])
        assert dense.rel_error(K, out["S"] @ H @ out["T"].T) < 1e-4


def test_ttk_at_fixed_theta_is_the_parametric_tensor_at_a_node():
    """Non-parametric TTK (Section 4.1) for a kernel with a parameter: the grid
    tensor at theta fixed to a parameter node is the parametric grid tensor's
    slice at that node, and S T^T interpolates K at fixed theta (H = I)."""
    Pp = kernels.Problem("exp", 2, [[0, 1]] * 2, [[2, 3], [0, 1]], [[0.5, 2.0]], 6)
    Mp = Pp.full_tensor()
    j = 4
    Pf = kernels.Problem("exp", 2, [[0, 1]] * 2, [[2, 3], [0, 1]], [], 6, theta_fixed=[Pp.nodes[2][j]])
    assert Pf.dt == 0 and Pf.D == 4
    assert np.array_equal(Pf.full_tensor(), Mp[:, :, j, :, :])
    rng = np.random.default_rng(2)
    X = rng.uniform(0, 1, (30, 2))
    Y = rng.uniform([2, 0], [3, 1], (25, 2))
    out = driver.offline(Pf, X, Y, 1e-10, seed=0)
    assert out["param"] == []
    K = dense.dense_K("exp", X, Y, [Pp.nodes[2][j]])
    assert dense.rel_error(K, out["S"] @ out["T"].T) < 1e-5       # interpolation level at n = 6
