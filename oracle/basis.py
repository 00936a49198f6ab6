"""Chebyshev interpolation basis (Section 2.4, "Multivariate Chebyshev
Interpolation").

* Chebyshev nodes of the first kind: the roots of T_n on [-1, 1],
  zeta_i = cos((2i - 1) pi / (2n)), i = 1..n (stored 0-based).
* The affine map phi_[a,b](x) = ((a - b)/2) x + (a + b)/2 as printed; it sends
  zeta_i (descending) to ascending eta_i.  Its inverse is
  t(x) = (2x - (a + b)) / (a - b).
* The basis polynomial phi^[a,b](eta_i, x) = 1/n + (2/n) sum_{k=1}^{n-1}
  T_k(zeta_i) T_k(t(x)), which Lemma 1 shows is the Lagrange polynomial of
  node i.  Here T_k(t) = cos(k arccos t), the definition given at the start of
  Section 2.4, evaluated directly (no recurrence).
* The basis-change matrix C[k, i] = (c_k / n) T_k(zeta_i), c_0 = 1, c_k = 2:
  sum_i f(eta_i) phi(eta_i, x) = sum_k (C f)_k T_k(t(x)), by regrouping the
  same sum.  C f is the Chebyshev coefficient vector (a DCT-II of f).
"""
import numpy as np


def cheb_nodes(n):
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.cos((2.0 * i - 1.0) * np.pi / (2.0 * n))


def affine(x, a, b):
    """phi_[a,b] : [-1,1] -> [a,b] as printed in Section 2.4."""
    return (a - b) / 2.0 * np.asarray(x, dtype=np.float64) + (a + b) / 2.0


def affine_inv(x, a, b):
    return (2.0 * np.asarray(x, dtype=np.float64) - (a + b)) / (a - b)


def grid_nodes(a, b, n):
    """eta_i = phi_[a,b](zeta_i), i = 1..n."""
    return affine(cheb_nodes(n), a, b)


def cheb_T_table(n, t):
    """Array [k, ...] of T_k(t) for k = 0..n-1."""
    t = np.clip(np.asarray(t, dtype=np.float64), -1.0, 1.0)
    ks = np.arange(n, dtype=np.float64)
    return np.cos(np.multiply.outer(ks, np.arccos(t)))


def cheb_dT_table(n, t):
    """Array [k, ...] of T_k'(t) = k U_{k-1}(t), k = 0..n-1.

    U_m are the Chebyshev polynomials of the second kind, from their
    defining recurrence U_0 = 1, U_1 = 2t, U_{m+1} = 2t U_m - U_{m-1}, which
    stays exact at the endpoints where the form sin((m+1)a)/sin(a) does not.
    """
    t = np.clip(np.asarray(t, dtype=np.float64), -1.0, 1.0)
    U = [np.ones_like(t), 2.0 * t]
    while len(U) < n:
        U.append(2.0 * t * U[-1] - U[-2])
    out = [np.zeros_like(t)] + [k * U[k - 1] for k in range(1, n)]
    return np.stack(out[:n], axis=0)


def basis_change(n):
    """C[k, i] = (c_k / n) T_k(zeta_i), the regrouping of the basis sum."""
    z = cheb_nodes(n)
    C = cheb_T_table(n, z) / n
    C[1:, :] *= 2.0
    return C


def lagrange_values(x, a, b, n):
    """q(x) = [phi^[a,b](eta_1, x), ..., phi^[a,b](eta_n, x)] for each x.

    Returns an array of shape x.shape + (n,).  This is the row vector
    q^s_i / q^p_i / q^t_i of Section 2.4 (the definition of the vectorised
    source, parameter and target polynomials).
    """
    z = cheb_nodes(n)
    t = affine_inv(x, a, b)
    Tz = cheb_T_table(n, z)             # [k, i]
    Tt = cheb_T_table(n, t)             # [k, ...]
    s = np.tensordot(Tt[1:], Tz[1:], axes=([0], [0]))  # [..., i]
    return 1.0 / n + 2.0 / n * s


def lagrange_derivs(x, a, b, n):
    """d/dx of lagrange_values: (2/n) sum_k T_k(zeta_i) T_k'(t) dt/dx."""
    z = cheb_nodes(n)
    t = affine_inv(x, a, b)
    Tz = cheb_T_table(n, z)
    dT = cheb_dT_table(n, t)
    s = np.tensordot(dT[1:], Tz[1:], axes=([0], [0]))
    return 2.0 / n * s * (2.0 / (a - b))


def lebesgue_function(x, n):
    """sum_k |phi^[-1,1](zeta_k, x)| (Lemma 1)."""
    return np.abs(lagrange_values(x, -1.0, 1.0, n)).sum(axis=-1)


# ----------------------------------------------- full coefficient tensor
def coefficient_tensor(M):
    """Chebyshev coefficient tensor of a grid tensor M (Section 2.4).

    Regrouping the multivariate interpolant sum_i M[i] prod_j phi(eta_{i_j}, .)
    by the Chebyshev-sum form of each basis polynomial gives
    sum_k A[k] prod_j T_{k_j}(t_j) with A = M x_1 C_1 x_2 C_2 ... x_D C_D,
    C_j = basis_change(n_j): a DCT-II along every mode.
    """
    A = np.asarray(M, dtype=np.float64)
    for j, nj in enumerate(A.shape):
        A = np.moveaxis(np.tensordot(basis_change(nj), A, axes=([1], [j])), 0, j)
    return A


def interpolant_coefficient_form(A, boxes, pts):
    """sum_k A[k] prod_j T_{k_j}(t_j(pts[:, j])) at points pts (P, D)."""
    pts = np.asarray(pts, dtype=np.float64)
    out = np.asarray(A, dtype=np.float64)[None]
    for j, (a, b) in enumerate(boxes):
        Tt = cheb_T_table(out.shape[1], affine_inv(pts[:, j], a, b))    # [k, p]
        out = np.einsum("pk...,kp->p...", out, Tt)
    return out


def interpolant_lagrange_form(M, boxes, pts):
    """sum_i M[i] prod_j phi^[a_j,b_j](eta_{i_j}, pts[:, j]) at points pts (P, D)."""
    pts = np.asarray(pts, dtype=np.float64)
    out = np.asarray(M, dtype=np.float64)[None]
    for j, (a, b) in enumerate(boxes):
        q = lagrange_values(pts[:, j], a, b, out.shape[1])               # [p, i]
        out = np.einsum("pi...,pi->p...", out, q)
    return out
