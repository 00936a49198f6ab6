"""PTTK stages (Section 3): offline Phase 3 (Algorithm 2), the core rounding
and gauge step that precedes it on the GPU path, the online stage
(Algorithm 3) and its theta-derivative, the apply K x ~ S H(theta) T^T x with
its backward pass, and PTTK-Global-1 (Algorithm 4).

Core numbering: cores[0..d-1] are the source cores G_1..G_d, cores[d..d+dt-1]
the parameter cores G_{d+1}..G_{d+dtheta}, cores[d+dt..D-1] the target cores
G_{d+dtheta+1}..G_D, where core d+dtheta+j belongs to target coordinate y_j.
"""
import numpy as np

from . import basis
from . import tt as ttmod


# ----------------------------------------------------------------- Phase 3
def factor_values(points, box, n):
    """U_i (or V_i) of Section 2.4: N x n Lagrange basis values per coordinate.

    points (N, d); box (d, 2).  Returns the list [U_1, ..., U_d].
    """
    pts = np.asarray(points, dtype=np.float64)
    return [basis.lagrange_values(pts[:, j], box[j, 0], box[j, 1], n) for j in range(pts.shape[1])]


def phase3_source(U, cores_s):
    """S <- U_1 G_1^{2}; S <- (U_i face-split S) G_i^{2}, i = 2..d (Algorithm 2).

    The face-splitting product's row p is kron(U_i[p], S[p]) (Section 2.1),
    whose index (k, a) -> a + k r is the little-endian row order of G_i^{2}.
    """
    S = U[0] @ ttmod.g2(cores_s[0])
    for i in range(1, len(cores_s)):
        FS = np.einsum("pk,pa->pka", U[i], S).reshape(S.shape[0], -1)   # kron(u, s)
        S = FS @ ttmod.g2(cores_s[i])
    return S


def phase3_target(V, cores_t):
    """T <- G_D^{1} V_d^T; T <- G_{D-i}^{1} (T khatri-rao V_{d-i}^T); T <- T^T (Algorithm 2).

    The Khatri-Rao product's column p is kron(T[:, p], V[p]) with index
    (b, k) -> k + b n, the little-endian column order of G^{1}.
    """
    d = len(cores_t)
    T = ttmod.g1(cores_t[d - 1]) @ V[d - 1].T
    for i in range(1, d):
        KR = np.einsum("bp,pk->bkp", T, V[d - 1 - i]).reshape(-1, T.shape[1])
        T = ttmod.g1(cores_t[d - 1 - i]) @ KR
    return T.T


def face_split(mats):
    """A_1 face-split A_2 face-split ... row by row (Section 2.1)."""
    out = mats[0]
    for M in mats[1:]:
        out = np.einsum("pa,pb->pab", out, M).reshape(out.shape[0], -1)
    return out


def phase3_explicit(U, V, cores_s, cores_t, n):
    """S = F_s L and T = F_t R with F_s = U_d face-split ... face-split U_1 and
    L = prod_i (I_{n^{d-i}} kron G_i^{2}) G_d^{2},
    R^T = G_{d+dt+1}^{1} prod_i (G_{d+dt+1+i}^{1} kron I_{n^i})  (Section 3.1)."""
    d = len(cores_s)
    Fs = face_split(U[::-1])
    Ft = face_split(V[::-1])
    Lm = np.eye(n ** d)
    for i in range(d - 1):
        Lm = Lm @ np.kron(np.eye(n ** (d - 1 - i)), ttmod.g2(cores_s[i]))
    Lm = Lm @ ttmod.g2(cores_s[d - 1])
    Rt = ttmod.g1(cores_t[0])
    for i in range(1, d):
        Rt = Rt @ np.kron(ttmod.g1(cores_t[i]), np.eye(n ** i))
    return Fs @ Lm, Ft @ Rt.T


# ----------------------------------------------------------- Phase 4-prime
def sign_fix_left(G, Gnext):
    """Make the largest-|.| entry of every column of G^{2} positive (lowest row
    on ties) and push the signs into the rows of the next core."""
    M = ttmod.g2(G)
    piv = np.argmax(np.abs(M), axis=0)
    sg = np.sign(M[piv, np.arange(M.shape[1])])
    sg[sg == 0] = 1.0
    G = ttmod.from_g2(M * sg[None, :], *G.shape)
    Gnext = Gnext * sg[:, None, None]
    return G, Gnext


def sign_fix_right(G, Gprev):
    """Same for the rows of G^{1}, pushing the signs into the previous core's columns."""
    M = ttmod.g1(G)
    piv = np.argmax(np.abs(M), axis=1)
    sg = np.sign(M[np.arange(M.shape[0]), piv])
    sg[sg == 0] = 1.0
    G = ttmod.from_g1(M * sg[:, None], *G.shape)
    Gprev = Gprev * sg[None, None, :]
    return G, Gprev


def round_and_gauge(cores, eps, d, dt):
    """TT-Round (Algorithm 1) of the cross cores, then gauge fixing.

    After rounding G_1..G_{D-1} are left-orthonormal.  The target cores
    G_D..G_{d+dt+1} are then right-orthonormalised (thin QR of (G^{1})^T) with
    R pushed into the left neighbour, so the last parameter core carries the
    norm.  Signs follow the largest-|.| rule on every orthonormal core.
    """
    G = ttmod.tt_round(cores, eps)
    D = len(G)
    for i in range(D - 1, d + dt - 1, -1):
        r0, n, r1 = G[i].shape
        Q, R = np.linalg.qr(ttmod.g1(G[i]).T)
        G[i] = ttmod.from_g1(Q.T, Q.shape[1], n, r1)
        a0, an, _ = G[i - 1].shape
        G[i - 1] = ttmod.from_g2(ttmod.g2(G[i - 1]) @ R.T, a0, an, Q.shape[1])
    for i in range(0, d + dt - 1):
        G[i], G[i + 1] = sign_fix_left(G[i], G[i + 1])
    for i in range(D - 1, d + dt - 1, -1):
        G[i], G[i - 1] = sign_fix_right(G[i], G[i - 1])
    return G


# ------------------------------------------------------------------ online
def online_H(param_cores, theta, boxes_theta, n):
    """H(theta) = H_1(theta_1) ... H_dt(theta_dt), H_j = G_{d+j} x_2 q^p_j(theta_j) (Algorithm 3)."""
    H = None
    for j, G in enumerate(param_cores):
        q = basis.lagrange_values(np.array(theta[j]), boxes_theta[j, 0], boxes_theta[j, 1], n)
        Hj = np.einsum("akb,k->ab", G, q)
        H = Hj if H is None else H @ Hj
    return H


def online_dH(param_cores, theta, boxes_theta, n):
    """dH/dtheta_j: factor j replaced by G_{d+j} x_2 dq^p_j/dtheta_j."""
    Hs, dHs = [], []
    for j, G in enumerate(param_cores):
        a, b = boxes_theta[j]
        q = basis.lagrange_values(np.array(theta[j]), a, b, n)
        dq = basis.lagrange_derivs(np.array(theta[j]), a, b, n)
        Hs.append(np.einsum("akb,k->ab", G, q))
        dHs.append(np.einsum("akb,k->ab", G, dq))
    out = []
    for j in range(len(param_cores)):
        M = None
        for i in range(len(param_cores)):
            F = dHs[i] if i == j else Hs[i]
            M = F if M is None else M @ F
        out.append(M)
    return out


# -------------------------------------------------------- apply / backward
def apply(S, H, T, x):
    """y = S (H (T^T x)) (the low-rank form of Section 1); x over targets."""
    return S @ (H @ (T.T @ x))


def apply_batched(S, Hs, T, X):
    """Y[:, b] = S H_b T^T X[:, b]."""
    W = T.T @ X
    Z = np.stack([Hs[b] @ W[:, b] for b in range(X.shape[1])], axis=1)
    return S @ Z, W


def backward_batched(S, Hs, dHs, T, X, G):
    """Gradients of L = sum_b <g_b, y_b>: dX_b = T H_b^T S^T g_b,
    dtheta_{b,j} = (S^T g_b)^T dH_{b,j} (T^T x_b)."""
    W = T.T @ X
    A = S.T @ G
    dX = np.stack([T @ (Hs[b].T @ A[:, b]) for b in range(X.shape[1])], axis=1)
    dth = np.array([[A[:, b] @ dHs[b][j] @ W[:, b] for j in range(len(dHs[b]))]
                    for b in range(X.shape[1])])
    return dX, dth


# ------------------------------------------------------------ Global case
def global_offline(S, T):
    """Thin QR of [S T] (Algorithm 4, offline part)."""
    Q, R = np.linalg.qr(np.hstack([S, T]))
    return Q, R


def global_online(R, H, rs, compress=False, eps=None):
    """Algorithm 4, online part, with H^ = [[0, H/2], [H^T/2, 0]] (symmetric
    part identity of Section 3.5).  Negative eigenvalues are dropped.
    Global-1 returns W = U Lambda U^T; Global-2 (compress) keeps the largest
    eigenvalues until the discarded tail is within eps ||R H^ R^T||_F and
    returns (U^, Lambda^)."""
    k = R.shape[0]
    Hh = np.zeros((k, k))
    Hh[:rs, rs:] = H / 2.0
    Hh[rs:, :rs] = H.T / 2.0
    M = R @ Hh @ R.T
    M = 0.5 * (M + M.T)
    lam, U = np.linalg.eigh(M)
    keep = lam > 0
    lam_p, U_p = lam[keep], U[:, keep]
    if not compress:
        return U_p @ np.diag(lam_p) @ U_p.T, int(np.sum(~keep))
    order = np.argsort(-lam_p)
    lam_p, U_p = lam_p[order], U_p[:, order]
    total = np.linalg.norm(M)
    r = len(lam_p)
    for rr in range(1, len(lam_p) + 1):
        if np.sqrt(np.sum(lam_p[rr:] ** 2)) <= eps * total:
            r = rr
            break
    return (U_p[:, :r], lam_p[:r]), int(np.sum(~keep))


# --------------------------------------------------- paper's Phase 4 (NEXT)
def phase4_paper(S, param_cores, T, eps):
    """TT-Round of [T^(1)(S), G_{d+1}, ..., G_{d+dt}, T^(3)(T^T)] (Algorithm 2, Phase 4)."""
    cores = [S[None, :, :]] + [np.array(G) for G in param_cores] + [T.T[:, :, None]]
    out = ttmod.tt_round(cores, eps)
    return out[0][0], out[1:-1], out[-1][:, :, 0].T


def storage_floats(Ns, Nt, ranks, n_param, d, dt):
    """N_s r_d + N_t r_{d+dt} + sum_j n r_{d+j-1} r_{d+j} (Section 3.2, storage)."""
    return Ns * ranks[d] + Nt * ranks[d + dt] + sum(n_param * ranks[d + j - 1] * ranks[d + j]
                                                  for j in range(1, dt + 1))
