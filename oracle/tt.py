"""Tensor-train helpers (Sections 2.2 and 2.3).

Unfoldings use the little-endian flattening of Section 2.2, which is NumPy's
Fortran-order reshape: the unfolding X^{j} of an array with axes (i_1..i_N)
is reshape(X, (n_1...n_j, n_{j+1}...n_N), order="F").  For a core
G in R^{r0 x n x r1}:  G^{1} = reshape(G, (r0, n r1)),  G^{2} =
reshape(G, (r0 n, r1)), both in that order.
"""
import numpy as np


def unfold(X, j):
    shape = X.shape
    return np.reshape(X, (int(np.prod(shape[:j])), int(np.prod(shape[j:]))), order="F")


def g1(G):
    return np.reshape(G, (G.shape[0], G.shape[1] * G.shape[2]), order="F")


def g2(G):
    return np.reshape(G, (G.shape[0] * G.shape[1], G.shape[2]), order="F")


def from_g1(M, r0, n, r1):
    return np.reshape(M, (r0, n, r1), order="F")


def from_g2(M, r0, n, r1):
    return np.reshape(M, (r0, n, r1), order="F")


def ranks(cores):
    return [cores[0].shape[0]] + [G.shape[2] for G in cores]


def full(cores):
    """Entry formula of Section 2.3: sum over the rank indices of the product
    of core slices."""
    X = cores[0][0]                                    # (n_1, r_1)
    for G in cores[1:]:
        X = np.tensordot(X, G, axes=([-1], [0]))       # (..., n_k, r_k)
    return X[..., 0]


def evaluate(cores, idx):
    """TT entries at multi-indices idx (P, N)."""
    idx = np.asarray(idx, dtype=np.int64)
    v = cores[0][0, idx[:, 0], :]                      # (P, r_1)
    for k in range(1, len(cores)):
        v = np.einsum("pa,pab->pb", v, np.transpose(cores[k][:, idx[:, k], :], (1, 0, 2)))
    return v[:, 0]


def frob(cores):
    return float(np.linalg.norm(full(cores)))


def _trunc_rank(s, delta):
    """Smallest r' >= 1 with sqrt(sum_{i > r'} s_i^2) <= delta."""
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]     # tail[i] = ||s[i:]||
    for r in range(1, len(s) + 1):
        rest = tail[r] if r < len(s) else 0.0
        if rest <= delta:
            return r
    return len(s)


def tt_svd(X, eps):
    """TT-SVD (Oseledets 2011, Algorithm 1, cited in Section 2.3)."""
    n = X.shape
    N = len(n)
    delta = eps / np.sqrt(max(N - 1, 1)) * np.linalg.norm(X)
    cores = []
    C = np.asarray(X, dtype=np.float64)
    r_prev = 1
    for k in range(N - 1):
        C = np.reshape(C, (r_prev * n[k], -1), order="F")
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        r = _trunc_rank(s, delta)
        cores.append(np.reshape(U[:, :r], (r_prev, n[k], r), order="F"))
        C = s[:r, None] * Vt[:r]
        r_prev = r
    cores.append(np.reshape(C, (r_prev, n[-1], 1), order="F"))
    return cores


def tt_round(cores, eps, return_info=False):
    """TT-Round (Algorithm 1).

    Right-to-left orthogonalisation by thin QR of (G_i^{1})^T, pushing R^T into
    the left neighbour (new G_{i-1}^{2} = G_{i-1}^{2} R^T), then left-to-right
    truncated SVD of G_i^{2} with threshold delta = eps / sqrt(N-1) ||X||_F,
    pushing Sigma V^T into the right neighbour.  ||X||_F is taken as ||G_1||_F
    after the orthogonalisation sweep (equal in exact arithmetic).  The
    truncation keeps the smallest r' with the discarded tail norm <= delta.
    """
    G = [np.array(c, dtype=np.float64) for c in cores]
    N = len(G)
    for i in range(N - 1, 0, -1):
        r0, n, r1 = G[i].shape
        Q, R = np.linalg.qr(g1(G[i]).T)                 # (n r1, r'), (r', r0)
        rp = Q.shape[1]
        G[i] = from_g1(Q.T, rp, n, r1)
        a0, an, _ = G[i - 1].shape
        G[i - 1] = from_g2(g2(G[i - 1]) @ R.T, a0, an, rp)
    norm = float(np.linalg.norm(G[0]))
    delta = eps / np.sqrt(max(N - 1, 1)) * norm
    margins = []
    for i in range(N - 1):
        r0, n, r1 = G[i].shape
        U, s, Vt = np.linalg.svd(g2(G[i]), full_matrices=False)
        r = _trunc_rank(s, delta)
        margins.append(float(s[r - 1] / delta) if delta > 0 else np.inf)
        G[i] = from_g2(U[:, :r], r0, n, r)
        b0, bn, b1 = G[i + 1].shape
        G[i + 1] = from_g1((s[:r, None] * Vt[:r]) @ g1(G[i + 1]), r, bn, b1)
    if return_info:
        return G, {"norm": norm, "delta": delta, "margins": margins}
    return G


def random_tt(rng, n, ranks_inner, scale=1.0):
    r = [1] + list(ranks_inner) + [1]
    return [scale * rng.standard_normal((r[k], n[k], r[k + 1])) for k in range(len(n))]
