"""TT greedy-cross (Appendices A and B), step by step.

Index sets.  I^{<=k} (k = 0..N-1) and I^{>k} (k = 1..N) are stored as integer
arrays L[k] of shape (r_k, k) and R[k] of shape (r_k, N-k), one multi-index
per row, 0-based, in insertion order.  L[0] and R[N] hold the single empty
multi-index.  Nestedness (Appendix A, "Nested index sets") holds because sets
only grow and every new element extends an element of the neighbouring set.

Super-core unfolding.  For k = 1..N-1 the matrix [X(I^{<=k-1}, :, :, I^{>k+1})]^{2}
has rows (s, i_k) -> s + i_k r_{k-1} and columns (i_{k+1}, t) -> i_{k+1} + t n_{k+1}
(little-endian, Section 2.2).  A pivot row l adds (L[k-1][l mod r_{k-1}], l div r_{k-1})
to I^{<=k}; a pivot column c adds (c mod n_{k+1}, R[k+1][c div n_{k+1}]) to I^{>k}.

Readings of the paper taken here:
* Algorithm 5 residual: R = A(:, J) A(I, J)^{-1} A(I, :) - A (rows I, columns J),
  the skeleton of Appendix A; A(I,J)^{-1} applied by an LU solve.
* Random samples: max{rows, cols} distinct linear positions lin = row*cols + col
  drawn by Floyd's algorithm from the splitmix64 stream keyed
  (seed, TAG_UPDATE, sweep, k), sorted ascending; the bit is the top bit of the
  next draw of the same stream; bit 1 searches the row, bit 0 the column.
* Ties: among |R| values within tau = 1e-10 * (largest |entry| evaluated in the
  call so far) of the maximum, the lowest linear position wins.
* "If applicable update": the pair is added only if |R(l,t)| > tau, l is not in
  I, t is not in J and r_k < max_rank.
* Stopping test: relative Chebyshev-norm error max|X - X^| / max|X| over
  n_test = max(1000, 20 N max n) fixed multi-indices from the stream
  (seed, TAG_TEST); also stops when a whole sweep adds no pivot or after
  max_sweeps sweeps.
* Interpolation formula: C_k = F_k P_k^{-1} with F_k = X(I^{<=k-1}, :, I^{>k})
  unfolded to (r_{k-1} n_k) x r_k and P_k = X(I^{<=k}, I^{>k}) its row subset,
  applied by a direct LU solve.  The cores returned are those whose sampled
  error the stopping test measured last.  C_N = F_N.  (The QR form
  Q Q[J,:]^{-1} of F_k = Q R, equal in exact arithmetic, stays available.)
* Replay of decisions taken by another computation of the same residuals
  (the GPU path): a forced choice is accepted if its |R|, computed here, lies
  within the tie band of this computation's maximum widened by
  2 (C_NOISE + r_k) times the rounding noise of the step's residuals, which
  the oracle measures itself as the largest disagreement between three
  backward-stable FP64 evaluation orders of the same skeleton formula (r_k:
  the rank before the step, the length of the elimination).  Algorithm 5 takes an
  argmax of computed residuals, so an entry within rounding of the band edge
  is an equally valid choice; the add test |R| > tau is judged the same way.
  Nothing the other computation reports (its residual values) enters the
  check: only its choices.
* Initialisation (Algorithm 7): q_1, q_2 are full random multi-indices; a
  snapshot (all sets, max condition number of the half-sweep) is kept after
  every half-sweep and the one with the smallest maximum is returned (earliest
  within a relative band of 1e-12); the argmin over (j1, j2) takes the lowest
  j1 * n + j2 within a relative band of 1e-12; a singular 2x2 has condition +inf.
"""
import numpy as np

from . import rng as rngmod
from . import tt as ttmod

TIE_REL = 1e-10
COND_REL = 1e-12
# rounding allowance of a replayed choice, in units of the measured residual
# noise: C_NOISE + r_k (see update_cross)
C_NOISE = 4.0


class Entries:
    """Counted access to the tensor entries."""

    def __init__(self, fn, n):
        self.fn = fn
        self.n = list(n)
        self.N = len(n)
        self.count = 0

    def __call__(self, idx):
        idx = np.asarray(idx, dtype=np.int64).reshape(-1, self.N)
        self.count += idx.shape[0]
        if idx.shape[0] == 0:
            return np.zeros(0)
        return np.asarray(self.fn(idx), dtype=np.float64)


def _empty():
    return np.zeros((1, 0), dtype=np.int64)


def _cond2(M):
    """2-norm condition numbers of a stack of 2x2 matrices (SVD route)."""
    s = np.linalg.svd(M, compute_uv=False)
    with np.errstate(divide="ignore", invalid="ignore"):
        c = s[..., 0] / s[..., -1]
    c[~np.isfinite(c)] = np.inf
    c[s[..., -1] == 0] = np.inf
    return c


def _argmin_band(vals, rel):
    """Lowest position whose value is within a relative band of the minimum."""
    vals = np.asarray(vals, dtype=np.float64)
    m = np.min(vals)
    if not np.isfinite(m):
        return int(np.argmax(vals == m)) if np.any(vals == m) else 0
    cand = np.nonzero(vals <= m * (1.0 + rel))[0]
    return int(cand[0])


def _argmax_band(absvals, tau):
    """Lowest position whose |R| is within tau of the maximum; margin to the runner-up."""
    absvals = np.asarray(absvals, dtype=np.float64)
    m = float(np.max(absvals))
    cand = np.nonzero(absvals >= m - tau)[0]
    pos = int(cand[0])
    rest = np.delete(absvals, pos)
    second = float(np.max(rest)) if rest.size else 0.0
    margin = (m - second) / m if m > 0 else 0.0
    return pos, m, margin


def greedy_init(ent, seed, max_it=10, card=2):
    """Index initialisation (Algorithm 7); card = 1 gives one random multi-index."""
    N, n = ent.N, ent.n
    g = rngmod.keyed(seed, rngmod.TAG_INIT)
    L = [None] * (N + 1)
    R = [None] * (N + 1)
    L[0] = _empty()
    R[N] = _empty()
    if card == 1:
        q = [g.below(n[j]) for j in range(N)]
        for k in range(1, N):
            L[k] = np.array([q[:k]], dtype=np.int64)
            R[k] = np.array([q[k:]], dtype=np.int64)
        return L, R, {"max_cond": None, "snapshots": []}
    q1 = [g.below(n[j]) for j in range(N)]
    q2 = [g.below(n[j]) for j in range(N)]
    for k in range(1, N):
        R[k] = np.array([q1[k:], q2[k:]], dtype=np.int64)
    snaps = []
    for _ in range(max_it):
        cs = []
        for k in range(1, N):                    # left-to-right, dimension k-1 (0-based)
            nk = n[k - 1]
            a, b = (L[k - 1][0], L[k - 1][1]) if k > 1 else (L[0][0], L[0][0])
            c, c2 = R[k][0], R[k][1]
            j1, j2 = np.meshgrid(np.arange(nk), np.arange(nk), indexing="ij")
            j1, j2 = j1.ravel(), j2.ravel()
            P = j1.size

            def mk(left, j, right):
                return np.concatenate([np.tile(left, (P, 1)), j[:, None], np.tile(right, (P, 1))], axis=1)

            v00 = ent(mk(a, j1, c))
            v01 = ent(mk(a, j1, c2))
            v10 = ent(mk(b, j2, c))
            v11 = ent(mk(b, j2, c2))
            M = np.stack([np.stack([v00, v01], -1), np.stack([v10, v11], -1)], -2)
            cond = _cond2(M)
            allowed = (j1 != j2) if k == 1 else np.ones(P, bool)
            vals = np.where(allowed, cond, np.inf)
            pos = _argmin_band(vals, COND_REL)
            if not allowed[pos]:
                pos = int(np.nonzero(allowed)[0][0])
            cs.append(float(vals[pos]))
            L[k] = np.array([np.concatenate([a, [j1[pos]]]), np.concatenate([b, [j2[pos]]])], dtype=np.int64)
        snaps.append(([x.copy() if x is not None else None for x in L],
                      [x.copy() if x is not None else None for x in R], max(cs)))
        cs = []
        for k in range(N, 1, -1):                # right-to-left, dimension k-1 (0-based)
            nk = n[k - 1]
            a, b = L[k - 1][0], L[k - 1][1]
            c, c2 = (R[k][0], R[k][1]) if k < N else (R[N][0], R[N][0])
            j1, j2 = np.meshgrid(np.arange(nk), np.arange(nk), indexing="ij")
            j1, j2 = j1.ravel(), j2.ravel()
            P = j1.size

            def mk(left, j, right):
                return np.concatenate([np.tile(left, (P, 1)), j[:, None], np.tile(right, (P, 1))], axis=1)

            v00 = ent(mk(a, j1, c))
            v01 = ent(mk(a, j2, c2))
            v10 = ent(mk(b, j1, c))
            v11 = ent(mk(b, j2, c2))
            M = np.stack([np.stack([v00, v01], -1), np.stack([v10, v11], -1)], -2)
            cond = _cond2(M)
            allowed = (j1 != j2) if k == N else np.ones(P, bool)
            vals = np.where(allowed, cond, np.inf)
            pos = _argmin_band(vals, COND_REL)
            if not allowed[pos]:
                pos = int(np.nonzero(allowed)[0][0])
            cs.append(float(vals[pos]))
            R[k - 1] = np.array([np.concatenate([[j1[pos]], c]), np.concatenate([[j2[pos]], c2])], dtype=np.int64)
        snaps.append(([x.copy() if x is not None else None for x in L],
                      [x.copy() if x is not None else None for x in R], max(cs)))
    best = _argmin_band([s[2] for s in snaps], COND_REL)
    Lb, Rb, mc = snaps[best]
    return Lb, Rb, {"max_cond": mc, "snapshot": best, "snapshots": [s[2] for s in snaps],
                    "snapshot_sets": [(s[0], s[1]) for s in snaps]}


def _positions_left(L, k, n):
    """Row positions of I^{<=k} in the row space of super-core k (1-based k)."""
    rl = L[k - 1].shape[0]
    lookup = {tuple(e): s for s, e in enumerate(L[k - 1])}
    return np.array([lookup[tuple(e[:-1])] + e[-1] * rl for e in L[k]], dtype=np.int64)


def _positions_right(R, k, n, N):
    """Column positions of I^{>k} in the column space of super-core k."""
    nk1 = n[k]
    lookup = {tuple(e): t for t, e in enumerate(R[k + 1])}
    return np.array([e[0] + lookup[tuple(e[1:])] * nk1 for e in R[k]], dtype=np.int64)


def _supercore_index(L, R, k, n, rows, cols):
    """Full multi-indices for super-core positions (rows[i], cols[i])."""
    rl = L[k - 1].shape[0]
    nk1 = n[k]
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    left = L[k - 1][rows % rl]
    ik = (rows // rl)[:, None]
    i1 = (cols % nk1)[:, None]
    right = R[k + 1][cols // nk1]
    return np.concatenate([left, ik, i1, right], axis=1)


def _skeleton_residuals(P, AxJ, AIy, Axy):
    """Skeleton error R(x, y) = A(x, J) A(I, J)^{-1} A(I, y) - A(x, y) of the
    cross approximation (Appendix A) for paired positions (x_i, y_i).

    P = A(I, J) (r x r), AxJ (m x r), AIy (r x m), Axy (m,).  The same formula
    is evaluated in three FP64 orders, each backward stable:
      right:  A(x, J) [P^{-1} A(I, y)]   (LU with partial pivoting)
      left:   [A(x, J) P^{-1}] A(I, y)   (LU of P^T)
      qr:     A(x, J) [R^{-1} Q^T A(I, y)]  (Householder QR of P)
    Returns the right-order residuals and the largest disagreement between
    the three orders, which measures the FP64 rounding noise of this step's
    residuals (it grows with the conditioning of P).
    """
    right = np.einsum("mr,rm->m", AxJ, np.linalg.solve(P, AIy)) - Axy
    left = np.einsum("mr,rm->m", np.linalg.solve(P.T, AxJ.T).T, AIy) - Axy
    Q, Rq = np.linalg.qr(P)
    qr = np.einsum("mr,rm->m", AxJ, np.linalg.solve(Rq, Q.T @ AIy)) - Axy
    spread = max(float(np.max(np.abs(right - left))), float(np.max(np.abs(right - qr))),
                 float(np.max(np.abs(left - qr))))
    return right, spread


def update_cross(ent, L, R, k, sweep, seed, max_rank, forced=None):
    """One update cross step (Algorithm 5) on super-core k (1-based).

    The super-core unfolding A = [X(I^{<=k-1}, :, :, I^{>k+1})]^{2} is skeleton-
    approximated on the rows I and columns J given by I^{<=k}, I^{>k}.  The
    step (i) draws max(rows, cols) random positions, (ii) takes the one with
    the largest |R|, (iii) draws a bit and searches the sample's row (bit 1)
    or column (bit 0) of R for its largest |R|, and (iv) adds that position's
    row and column to I and J when |R| there exceeds tau and both are new.

    Returns a decision record and mutates L[k], R[k] when a pivot is added.
    With `forced` (the pivots another computation chose: sample_pos,
    pivot_row, pivot_col, added), the forced choices are taken instead, after
    checking that each lies within this computation's tie band, widened by
    (C_NOISE + r_k) times the rounding noise of the step's residuals measured
    here (_skeleton_residuals); no value reported by the other computation
    enters.
    """
    n = ent.n
    rl, rr = L[k - 1].shape[0], R[k + 1].shape[0]
    nk1 = n[k]
    rows, cols = rl * n[k - 1], nk1 * rr
    I = _positions_left(L, k, n)
    J = _positions_right(R, k, n, ent.N)
    rk = I.size

    def A(rr_, cc_):
        return ent(_supercore_index(L, R, k, n, np.asarray(rr_, np.int64), np.asarray(cc_, np.int64)))

    # (i) random positions of the unfolding (Floyd sample) and their residuals
    g = rngmod.keyed(seed, rngmod.TAG_UPDATE, sweep, k)
    ns = max(rows, cols)
    lin = np.array(g.floyd(rows * cols, ns), dtype=np.int64)
    srow, scol = lin // cols, lin % cols
    P = A(np.repeat(I, rk), np.tile(J, rk)).reshape(rk, rk)
    AsJ = A(np.repeat(srow, rk), np.tile(J, ns)).reshape(ns, rk)
    AIs = A(np.repeat(I, ns), np.tile(scol, rk)).reshape(rk, ns)
    As = A(srow, scol)
    seen = max(np.max(np.abs(P)), np.max(np.abs(AsJ)), np.max(np.abs(AIs)), np.max(np.abs(As)))
    Rs, noise = _skeleton_residuals(P, AsJ, AIs, As)
    tau = TIE_REL * seen
    p, m0, margin0 = _argmax_band(np.abs(Rs), tau)
    rec = {"sweep": sweep, "k": k, "rank_before": rk,
           "sample_pos": int(lin[p]), "sample_max": m0, "sample_margin": margin0}

    # (iii) the searched fibre through the chosen sample
    bit = g.bit()
    rec["bit"] = int(bit)
    if forced is not None:
        where = np.nonzero(lin == int(forced["sample_pos"]))[0]
        p_forced = int(where[0]) if where.size == 1 else p
    else:
        where, p_forced = None, p
    l, t = int(srow[p_forced]), int(scol[p_forced])
    if bit == 1:
        fib = np.arange(cols)
        AfJ = np.tile(A(np.full(rk, l), J), (cols, 1))
        AIf = A(np.repeat(I, cols), np.tile(fib, rk)).reshape(rk, cols)
        Af = A(np.full(cols, l), fib)
    else:
        fib = np.arange(rows)
        AfJ = A(np.repeat(fib, rk), np.tile(J, rows)).reshape(rows, rk)
        AIf = np.tile(A(I, np.full(rk, t))[:, None], (1, rows))
        Af = A(fib, np.full(rows, t))
    seen = max(seen, np.max(np.abs(AfJ)), np.max(np.abs(AIf)), np.max(np.abs(Af)))
    Rf, noise_f = _skeleton_residuals(P, AfJ, AIf, Af)
    noise = max(noise, noise_f)
    tau = TIE_REL * seen
    q, m1, margin1 = _argmax_band(np.abs(Rf), tau)
    # Rounding allowance of one FP64 computation of R by any elimination-based
    # solve with P: the worst-case backward error of elimination grows
    # linearly with its length r_k (gamma_{r_k} = r_k u / (1 - r_k u), Higham,
    # "Accuracy and Stability of Numerical Algorithms", 2nd ed., Thm 9.3),
    # while the measured spread of three orders reflects their typical error.
    band = (C_NOISE + rk) * noise

    def in_band(val, m):
        return val >= m - max(tau, 1e-9 * m) - 2.0 * band

    if forced is not None:
        rec["replay_sample_ok"] = bool(where.size == 1 and in_band(abs(Rs[p_forced]), m0))
        q_forced = int(forced["pivot_col"] if bit == 1 else forced["pivot_row"])
        rec["replay_search_ok"] = bool(0 <= q_forced < fib.size and in_band(abs(Rf[q_forced]), m1))
        q = q_forced if 0 <= q_forced < fib.size else q
    if bit == 1:
        t = q
    else:
        l = q
    val = abs(Rf[q])
    # (iv) add the pivot when it is significant and new
    fresh = (l not in set(I.tolist())) and (t not in set(J.tolist())) and rk < max_rank
    add = bool(val > tau and fresh)
    if forced is not None:
        # |R| within the rounding allowance of tau may be judged either way
        rec["replay_add_ok"] = bool(add == bool(forced["added"]) or (fresh and abs(val - tau) <= 2.0 * band))
        add = bool(forced["added"])
    rec.update({"pivot_row": l, "pivot_col": t, "pivot_abs": float(val), "search_margin": margin1,
                "tau": float(tau), "noise": float(noise), "added": add})
    if add:
        newL = np.concatenate([L[k - 1][l % rl], [l // rl]])
        newR = np.concatenate([[t % nk1], R[k + 1][t // nk1]])
        L[k] = np.vstack([L[k], newL[None, :]])
        R[k] = np.vstack([R[k], newR[None, :]])
    return rec


def fibre(ent, L, R, k):
    """F_k = X(I^{<=k-1}, :, I^{>k}) unfolded to (r_{k-1} n_k) x r_k (1-based k)."""
    N, n = ent.N, ent.n
    left = L[k - 1]
    right = R[k]
    rl, rr, nk = left.shape[0], right.shape[0], n[k - 1]
    rows = np.arange(rl * nk)
    s, ik = rows % rl, rows // rl
    idx = np.concatenate([np.repeat(left[s], rr, axis=0),
                          np.repeat(ik, rr)[:, None],
                          np.tile(right, (rl * nk, 1))], axis=1)
    return ent(idx).reshape(rl * nk, rr)


def interp_cores(ent, L, R, method="qr"):
    """Cores of the cross interpolant (interpolation formula of Appendix A).

    method "qr": C_k = Q Q[J,:]^{-1} from the thin QR F_k = Q R (final cores);
    method "lu": C_k = F_k P_k^{-1} by an LU solve (the sampled stopping test).
    """
    N, n = ent.N, ent.n
    cores = []
    for k in range(1, N + 1):
        F = fibre(ent, L, R, k)
        rl = L[k - 1].shape[0]
        if k < N:
            Jp = _positions_left(L, k, n)
            if method == "qr":
                Q, _ = np.linalg.qr(F)
                C = np.linalg.solve(Q[Jp, :].T, Q.T).T        # Q Q[J,:]^{-1}
            else:
                C = np.linalg.solve(F[Jp, :].T, F.T).T        # F P^{-1}
            cores.append(ttmod.from_g2(C, rl, n[k - 1], C.shape[1]))
        else:
            cores.append(ttmod.from_g2(F, rl, n[k - 1], 1))
    return cores


def test_points(seed, n, n_test):
    g = rngmod.keyed(seed, rngmod.TAG_TEST)
    return np.array([[g.below(nj) for nj in n] for _ in range(n_test)], dtype=np.int64)


def greedy_cross(ent, eps, seed=0, max_rank=256, max_sweeps=200, init_card=2, init_max_it=10,
                 n_test=None, forced=None):
    """TT greedy-cross outline (Algorithm 6) with the readings above.

    Returns (cores, info); info holds the final index sets, the decision log,
    the sweep count, the sampled error and the number of entry evaluations.
    """
    N, n = ent.N, ent.n
    L, R, init_info = greedy_init(ent, seed, init_max_it, init_card)
    if n_test is None:
        n_test = max(1000, 20 * N * max(n))
    tidx = test_points(seed, n, n_test)
    tval = ent(tidx)
    tmax = float(np.max(np.abs(tval)))

    def sampled_error():
        c = interp_cores(ent, L, R, method="lu")
        return float(np.max(np.abs(ttmod.evaluate(c, tidx) - tval)) / tmax), c

    log = []
    err, cores = sampled_error()
    errs = [err]
    sweep = 0
    fi = 0
    def keep_going():
        if forced is not None:          # replay: as many sweeps as the log holds
            return fi < len(forced)
        return err > eps and sweep < max_sweeps

    while keep_going():
        added = 0
        for k in range(1, N):
            f = None
            if forced is not None:
                f = forced[fi]
                fi += 1
            rec = update_cross(ent, L, R, k, sweep, seed, max_rank, forced=f)
            log.append(rec)
            added += int(rec["added"])
        sweep += 1
        err, cores = sampled_error()
        errs.append(err)
        if added == 0 and forced is None:
            break
    cores = interp_cores(ent, L, R, method="lu")
    info = {"L": L, "R": R, "log": log, "sweeps": sweep, "errors": errs, "error": err,
            "converged": err <= eps, "evals": ent.count, "init": init_info,
            "ranks": [1] + [L[k].shape[0] for k in range(1, N)] + [1]}
    return cores, info
