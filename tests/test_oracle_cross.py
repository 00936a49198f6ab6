"""Pins for the oracle's TT greedy-cross (Appendices A and B)."""
import numpy as np
import pytest

from oracle import basis, cross, kernels, pttk, tt


def _ent_from_tt(cores):
    n = [c.shape[1] for c in cores]
    return cross.Entries(lambda idx: tt.evaluate(cores, idx), n)


def _nested(L, R, N):
    for k in range(2, N):
        prev = {tuple(e) for e in L[k - 1]}
        assert all(tuple(e[:-1]) in prev for e in L[k])
    for k in range(1, N - 1):
        nxt = {tuple(e) for e in R[k + 1]}
        assert all(tuple(e[1:]) in nxt for e in R[k])


def test_exact_low_rank_recovered():
    """A tensor with exact TT ranks (2,3,3,2): the cross interpolant is exact
    (skeleton exactness of Appendix A for exactly low-rank matrices)."""
    rng = np.random.default_rng(0)
    n = [5, 6, 5, 6, 5]
    cores = tt.random_tt(rng, n, [2, 3, 3, 2])
    ent = _ent_from_tt(cores)
    c, info = cross.greedy_cross(ent, 1e-12, seed=3)
    X = tt.full(cores)
    assert np.linalg.norm(tt.full(c) - X) <= 1e-10 * np.linalg.norm(X)
    assert all(r <= e for r, e in zip(info["ranks"], [1, 2, 3, 3, 2, 1]))
    assert info["converged"]
    _nested(info["L"], info["R"], len(n))


def test_interpolates_evaluated_fibres():
    """Pin (b): the cross interpolant reproduces X on every fibre it is built from."""
    P = kernels.Problem("matern32", 1, [[0, 1]], [[2, 3]], [[0.5, 2.0]], 8)
    ent = cross.Entries(P.entries, P.n)
    c, info = cross.greedy_cross(ent, 1e-6, seed=1)
    L, R = info["L"], info["R"]
    Xh = tt.full(c)
    N = len(P.n)
    for k in range(1, N + 1):
        F = cross.fibre(ent, L, R, k)
        rl = L[k - 1].shape[0]
        for row in range(F.shape[0]):
            s, ik = row % rl, row // rl
            for t in range(F.shape[1]):
                mi = tuple(L[k - 1][s]) + (ik,) + tuple(R[k][t])
                assert abs(Xh[mi] - F[row, t]) <= 1e-11 * np.abs(F).max()


def test_polynomial_kernel_reproduced_exactly():
    """Pin (a): (1 + theta x.y)^3 has degree 3 < n in every variable, so the
    whole chain (cross, rounding, Phase 3, online) reproduces it off-grid."""
    d, n = 2, 5
    P = kernels.Problem("poly", d, [[0, 1], [-1, 0.5]], [[2, 3], [0, 1]], [[0.5, 2.0]], n)
    ent = cross.Entries(P.entries, P.n)
    c, info = cross.greedy_cross(ent, 1e-13, seed=0)
    G = pttk.round_and_gauge(c, 1e-14, d, 1)
    rng = np.random.default_rng(1)
    X = rng.uniform(P.box_s[:, 0], P.box_s[:, 1], (40, d))
    Y = rng.uniform(P.box_t[:, 0], P.box_t[:, 1], (30, d))
    S = pttk.phase3_source(pttk.factor_values(X, P.box_s, n), G[:d])
    T = pttk.phase3_target(pttk.factor_values(Y, P.box_t, n), G[d + 1:])
    for th in (0.5, 0.77, 1.6, 2.0):
        H = pttk.online_H(G[d:d + 1], [th], P.box_theta, n)
        K = (1 + th * X @ Y.T) ** 3
        assert np.abs(S @ H @ T.T - K).max() <= 1e-11 * np.abs(K).max()


def test_separable_rank_one():
    """Pin (c): exp(sum x) theta exp(-sum y) has every TT rank 1."""
    P = kernels.Problem("sep", 2, [[0, 1], [0, 1]], [[2, 3], [0, 1]], [[0.5, 2.0]], 6)
    M = P.full_tensor()
    assert tt.ranks(tt.tt_svd(M, 1e-12)) == [1] * 6
    ent = cross.Entries(P.entries, P.n)
    c1, info1 = cross.greedy_cross(ent, 1e-12, seed=0, init_card=1)
    assert info1["ranks"] == [1] * 6
    assert np.linalg.norm(tt.full(c1) - M) <= 1e-12 * np.linalg.norm(M)


def test_init_half_sweeps_and_nesting():
    P = kernels.Problem("se", 2, [[0, 1], [0, 1]], [[2, 3], [0, 1]], [[0.5, 2.0]], 6)
    ent = cross.Entries(P.entries, P.n)
    L, R, info = cross.greedy_init(ent, 5, max_it=3)
    assert len(info["snapshots"]) == 6
    assert info["max_cond"] == min(info["snapshots"])
    assert np.isfinite(info["max_cond"])
    for k in range(1, 5):
        assert L[k].shape == (2, k) and R[k].shape == (2, 5 - k)
        assert not np.array_equal(L[k][0], L[k][1]) and not np.array_equal(R[k][0], R[k][1])
    _nested(L, R, 5)
    # every init probe: 4 entries per (j1, j2) per k per half-sweep
    assert ent.count == 3 * 2 * 4 * 4 * 36


def test_init_choice_is_the_argmin_condition_number():
    """Brute-force check of the first left-to-right step (k = 1) of Algorithm 7."""
    P = kernels.Problem("matern32", 1, [[0, 1]], [[2, 3]], [[0.5, 2.0]], 5)
    ent = cross.Entries(P.entries, P.n)
    L, R, info = cross.greedy_init(ent, 2, max_it=1)
    from oracle import rng as rngmod
    g = rngmod.keyed(2, rngmod.TAG_INIT)
    q1 = [g.below(5) for _ in range(3)]
    q2 = [g.below(5) for _ in range(3)]
    best, arg = np.inf, None
    for j1 in range(5):
        for j2 in range(5):
            if j1 == j2:
                continue
            M = np.array([[P.entries([[j1] + q1[1:]])[0], P.entries([[j1] + q2[1:]])[0]],
                          [P.entries([[j2] + q1[1:]])[0], P.entries([[j2] + q2[1:]])[0]]])
            c = np.linalg.cond(M, 2)
            if c < best * (1 - 1e-12):
                best, arg = c, (j1, j2)
    L_first = info["snapshot_sets"][0][0]
    assert [int(L_first[1][0, 0]), int(L_first[1][1, 0])] == list(arg)


def test_replay_of_own_log_is_consistent():
    P = kernels.Problem("matern32", 1, [[0, 1]], [[2, 3]], [[0.5, 2.0]], 8)
    c1, i1 = cross.greedy_cross(cross.Entries(P.entries, P.n), 1e-7, seed=4)
    c2, i2 = cross.greedy_cross(cross.Entries(P.entries, P.n), 1e-7, seed=4, forced=i1["log"])
    assert all(r["replay_sample_ok"] and r["replay_search_ok"] and r["replay_add_ok"] for r in i2["log"])
    for k in range(1, 3):
        assert np.array_equal(i1["L"][k], i2["L"][k]) and np.array_equal(i1["R"][k], i2["R"][k])


def test_replay_detects_a_bad_pivot():
    """A forced pivot outside the tie band is flagged by the replay check."""
    P = kernels.Problem("matern32", 1, [[0, 1]], [[2, 3]], [[0.5, 2.0]], 8)
    ent = cross.Entries(P.entries, P.n)
    L, R, _ = cross.greedy_init(ent, 4)
    good = cross.update_cross(ent, [None if x is None else x.copy() for x in L], [None if x is None else x.copy() for x in R], 1, 0, 4, 256)
    bad = dict(good)
    if good["bit"] == 1:
        bad["pivot_col"] = (good["pivot_col"] + 1) % 8
    else:
        bad["pivot_row"] = (good["pivot_row"] + 1) % 8
    rec = cross.update_cross(ent, [None if x is None else x.copy() for x in L], [None if x is None else x.copy() for x in R], 1, 0, 4, 256, forced=bad)
    assert rec["replay_sample_ok"] and not rec["replay_search_ok"]


def test_prop1_tt_error_amplification_bound():
    """Proposition 1's computable part: |K_TT - K_full|_C <= lambda^D ||M - M^||_C."""
    n, d = 6, 1
    P = kernels.Problem("exp", d, [[0, 1]], [[2, 3]], [[0.5, 2.0]], n)
    M = P.full_tensor()
    c, _ = cross.greedy_cross(cross.Entries(P.entries, P.n), 1e-3, seed=0)
    Mh = tt.full(c)
    lam = basis.lebesgue_function(np.linspace(-1, 1, 20001), n).max()
    rng = np.random.default_rng(0)
    X = rng.uniform(0, 1, (25, 1))
    Y = rng.uniform(2, 3, (25, 1))
    worst = 0.0
    for th in (0.5, 0.9, 2.0):
        q = [basis.lagrange_values(X[:, 0], 0, 1, n), basis.lagrange_values(np.array(th), 0.5, 2.0, n),
             basis.lagrange_values(Y[:, 0], 2, 3, n)]
        Kf = np.einsum("abc,pa,b,qc->pq", M, q[0], q[1], q[2])
        Kt = np.einsum("abc,pa,b,qc->pq", Mh, q[0], q[1], q[2])
        worst = max(worst, np.abs(Kf - Kt).max())
    assert worst <= lam ** 3 * np.abs(M - Mh).max() * (1 + 1e-12)


def test_replay_band_ignores_values_reported_by_the_replayed_computation():
    """The replay judges a forced choice by the oracle's own residuals and
    noise estimate: residual values carried in the forced record (however
    wrong) change nothing, and a wrong pivot stays flagged."""
    P = kernels.Problem("matern32", 1, [[0, 1]], [[2, 3]], [[0.5, 2.0]], 8)
    ent = cross.Entries(P.entries, P.n)
    L, R, _ = cross.greedy_init(ent, 4)
    cp = lambda S: [None if x is None else x.copy() for x in S]
    good = cross.update_cross(ent, cp(L), cp(R), 1, 0, 4, 256)
    choice = {k: good[k] for k in ("sample_pos", "pivot_row", "pivot_col", "added")}
    ref = cross.update_cross(ent, cp(L), cp(R), 1, 0, 4, 256, forced=choice)
    junk = dict(choice, sample_max=1e30, pivot_abs=-5.0)
    rec = cross.update_cross(ent, cp(L), cp(R), 1, 0, 4, 256, forced=junk)
    for key in ("replay_sample_ok", "replay_search_ok", "replay_add_ok", "noise", "tau"):
        assert rec[key] == ref[key], key
    assert rec["replay_sample_ok"] and rec["replay_search_ok"] and rec["replay_add_ok"]
    bad = dict(choice)
    if good["bit"] == 1:
        bad["pivot_col"] = (good["pivot_col"] + 1) % 8
    else:
        bad["pivot_row"] = (good["pivot_row"] + 1) % 8
    bad["pivot_abs"] = good["pivot_abs"]            # claiming the right value does not help
    rec = cross.update_cross(ent, cp(L), cp(R), 1, 0, 4, 256, forced=bad)
    assert not rec["replay_search_ok"]


def test_residual_noise_estimate_is_rounding_sized():
    """The three FP64 orders of the skeleton residual agree to rounding of a
    well-conditioned intersection matrix, and the disagreement grows with its
    condition number, as a forward-error bound of a linear solve does."""
    rng = np.random.default_rng(3)
    r, m = 12, 300
    AxJ = rng.standard_normal((m, r))
    AIy = rng.standard_normal((r, m))
    Axy = rng.standard_normal(m)
    Qa, _ = np.linalg.qr(rng.standard_normal((r, r)))
    Qb, _ = np.linalg.qr(rng.standard_normal((r, r)))
    spreads = []
    for cond in (1.0, 1e6, 1e12):
        P = Qa @ np.diag(np.logspace(0, -np.log10(cond), r)) @ Qb
        Rr, spread = cross._skeleton_residuals(P, AxJ, AIy, Axy)
        exact = np.einsum("mr,rm->m", AxJ, np.linalg.solve(P, AIy)) - Axy
        assert np.array_equal(Rr, exact)
        scale = np.abs(Rr).max()
        assert spread <= 1e3 * np.finfo(float).eps * cond * scale
        spreads.append(spread / scale)
    assert spreads[0] < 1e-13 and spreads[2] > spreads[0]
