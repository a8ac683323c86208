"""Host-side basis for the streamed pipeline's dimension reduction (Sec. 2.2,
"Using SVD to project to the best fit subspace": each piece is replaced by its projection onto the top right singular vectors;
the paper computes them with a randomized SVD).

``top_right_singular_vectors`` is the randomized range finder with subspace
iteration of Halko, Martinsson & Tropp (2011, Alg. 4.4) followed by the exact
SVD of the small projected matrix (their Alg. 5.1), on a sample of rows.  The
projection itself runs on the GPU (``kmx_project``).
"""
from __future__ import annotations

import numpy as np


def top_right_singular_vectors(A, m: int, oversample: int = 10, power_iters: int = 2,
                               seed: int = 0) -> np.ndarray:
    """Approximate top m right singular vectors of A (rows x d) as a d x m
    float32 matrix with orthonormal columns."""
    A = np.asarray(A, dtype=np.float32)
    rng = np.random.default_rng(seed)
    ell = min(m + oversample, min(A.shape))
    Om = rng.standard_normal((A.shape[1], ell)).astype(np.float32)
    Q, _ = np.linalg.qr((A @ Om).astype(np.float64))
    for _ in range(power_iters):
        W, _ = np.linalg.qr((A.T @ Q.astype(np.float32)).astype(np.float64))
        Q, _ = np.linalg.qr((A @ W.astype(np.float32)).astype(np.float64))
    B = (Q.T.astype(np.float32) @ A).astype(np.float64)
    _, _, Vt = np.linalg.svd(B, full_matrices=False)
    return np.ascontiguousarray(Vt[:m].T.astype(np.float32))
