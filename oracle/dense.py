"""Dense truth and error metrics (Section 4, introduction).

relative error = ||K - K^||_p / ||K||_p, p in {2, F}; for matrices too large
to form, the same ratio on a uniformly subsampled set of rows and columns.
"""
import numpy as np

from . import kernels


def dense_K(kind, X, Y, theta, const=None):
    """[K]_{ij} = kappa(x_i, y_j; theta); rows are sources (Section 1)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    th = np.broadcast_to(np.asarray(theta, dtype=np.float64), (X.shape[0], Y.shape[0], len(theta)))
    return kernels.kappa(kind, X[:, None, :], Y[None, :, :], th, const)


def dense_dK(kind, X, Y, theta, const=None):
    """d K / d theta_j stacked on the last axis."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    th = np.broadcast_to(np.asarray(theta, dtype=np.float64), (X.shape[0], Y.shape[0], len(theta)))
    return kernels.dkappa_dtheta(kind, X[:, None, :], Y[None, :, :], th, const)


def rel_error(K, Khat, p="fro"):
    ordp = "fro" if p == "fro" else 2
    return float(np.linalg.norm(K - Khat, ord=ordp) / np.linalg.norm(K, ord=ordp))


def rel_fro(a, b):
    """||a - b||_F / ||b||_F for arrays of any shape."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))
