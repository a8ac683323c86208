"""FP64 reference of the dimension reduction of the streamed pipeline (test
infrastructure only).

Sec. 2.2 ("Using SVD to project to the best fit subspace") replaces each
piece by its best-fit low-dimensional approximation:
with A = U D V^T, keeping the top m singular values gives A_m, whose rows lie
in the span of the top m right singular vectors V_m.  A row's coordinates in
that span, y = x V_m, keep every squared distance between rows of A_m, so
k-means on the coordinates equals k-means on A_m (centers restricted to the
span, where optimal centers lie).

  * best_fit_basis(A, m)  -- V_m by the exact SVD (numpy / LAPACK);
  * best_fit_basis_weighted(A, w, m) -- V_m of the weighted point set
    (Sec. 2.3.2: the rows scaled by sqrt(w));
  * project(X, V)         -- X V in FP64;
  * rank_m_rows(A, m)     -- A V_m V_m^T, the rows of A_m.
"""
from __future__ import annotations

import numpy as np


def best_fit_basis(A, m: int) -> np.ndarray:
    """Top m right singular vectors of A as the columns of a d x m matrix."""
    A = np.asarray(A, np.float64)
    _, _, Vt = np.linalg.svd(A, full_matrices=False)
    return Vt[:m].T.copy()


def best_fit_basis_weighted(A, w, m: int) -> np.ndarray:
    """Top m right singular vectors of the weighted point set (Sec. 2.3.2):
    the matrix whose row i is sqrt(w_i) times row i of A has the same right
    singular vectors as the matrix holding w_i copies of row i."""
    A = np.asarray(A, np.float64)
    s = np.sqrt(np.asarray(w, np.float64)).reshape(-1, 1)
    return best_fit_basis(s * A, m)


def project(X, V) -> np.ndarray:
    """Coordinates X V of the rows of X in the basis V (FP64)."""
    return np.asarray(X, np.float64) @ np.asarray(V, np.float64)


def rank_m_rows(A, m: int) -> np.ndarray:
    """Rows of the best rank-m approximation A_m = A V_m V_m^T."""
    V = best_fit_basis(A, m)
    return project(A, V) @ V.T
