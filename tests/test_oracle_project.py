"""Pins of the projection reference: distances inside the span are kept, the
rank-m approximation is the best one (Eckart-Young), planted mistakes fail."""
import numpy as np
import pytest

from oracle import project as op


def _lowrank(n, d, r, seed, noise=0.0):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((r, d))
    Z = rng.standard_normal((n, r))
    return Z @ F + noise * rng.standard_normal((n, d))


def test_distances_preserved_for_points_in_the_span():
    A = _lowrank(300, 50, 6, 0)               # exactly rank 6
    V = op.best_fit_basis(A, 6)
    Y = op.project(A, V)
    i, j = np.triu_indices(60, 1)
    dA = np.sum((A[i] - A[j]) ** 2, axis=1)
    dY = np.sum((Y[i] - Y[j]) ** 2, axis=1)
    np.testing.assert_allclose(dY, dA, rtol=1e-9)
    np.testing.assert_allclose(V.T @ V, np.eye(6), atol=1e-12)


def test_rank_m_approximation_is_optimal():
    A = _lowrank(200, 30, 5, 1, noise=0.3)
    Am = op.rank_m_rows(A, 5)
    s = np.linalg.svd(A, compute_uv=False)
    # Eckart-Young: ||A - A_m||_F^2 = sum of the discarded squared singular values
    assert abs(np.sum((A - Am) ** 2) - np.sum(s[5:] ** 2)) <= 1e-8 * np.sum(s ** 2)
    # any other rank-5 projection does worse
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 5)))
    assert np.sum((A - A @ Q @ Q.T) ** 2) > np.sum((A - Am) ** 2)


def test_kmeans_cost_in_coordinates_equals_cost_in_span():
    A = _lowrank(150, 40, 4, 3, noise=0.2)
    V = op.best_fit_basis(A, 4)
    Am = op.rank_m_rows(A, 4)
    Y = op.project(A, V)
    C_span = Am[:5]                           # centers inside the span
    C_coord = op.project(C_span, V)
    cost_span = np.sum(np.min(((Am[:, None, :] - C_span[None]) ** 2).sum(-1), axis=1))
    cost_coord = np.sum(np.min(((Y[:, None, :] - C_coord[None]) ** 2).sum(-1), axis=1))
    assert abs(cost_span - cost_coord) <= 1e-9 * cost_span


def test_planted_mistakes_are_caught(monkeypatch):
    real = op.best_fit_basis
    # left instead of right singular vectors (first d entries of U's columns)
    monkeypatch.setattr(op, "best_fit_basis",
                        lambda A, m: np.linalg.svd(np.asarray(A, np.float64))[0][:A.shape[1], :m])
    with pytest.raises(AssertionError):
        test_rank_m_approximation_is_optimal()
    monkeypatch.setattr(op, "best_fit_basis", lambda A, m: real(A, m + 1)[:, 1:])  # drops the top one
    with pytest.raises(AssertionError):
        test_rank_m_approximation_is_optimal()


def test_weighted_basis_equals_replicated_rows():
    # Sec. 2.3.2: integer weights; the sqrt(w)-scaled matrix and the matrix
    # with w copies of every row have the same best-fit subspace (compared as
    # projectors, which removes the sign / rotation freedom)
    rng = np.random.default_rng(5)
    A = _lowrank(60, 12, 3, 4, noise=0.5)
    w = rng.integers(1, 6, 60)
    F = np.repeat(A, w, axis=0)
    for m in (1, 3, 5):
        Vw = op.best_fit_basis_weighted(A, w, m)
        Vf = op.best_fit_basis(F, m)
        np.testing.assert_allclose(Vw @ Vw.T, Vf @ Vf.T, atol=1e-9)
    # unit weights reduce to the plain basis
    V1 = op.best_fit_basis_weighted(A, np.ones(60), 3)
    V0 = op.best_fit_basis(A, 3)
    np.testing.assert_allclose(V1 @ V1.T, V0 @ V0.T, atol=1e-10)
    # scaling by w instead of sqrt(w) would not match the replicated rows
    Vbad = op.best_fit_basis(w.reshape(-1, 1) * A, 3)
    assert np.abs(Vbad @ Vbad.T - op.best_fit_basis(F, 3) @ op.best_fit_basis(F, 3).T).max() > 1e-3
