"""Pins of the router network's FP64 reference: central finite differences,
a hand-worked case and the Adam update written out by hand.  CPU only."""
import numpy as np
import pytest

from oracle import mlp


def _params(rng, d, H, k, scale=0.5):
    return (rng.normal(0, scale, (H, d)), rng.normal(0, 0.1, H),
            rng.normal(0, scale, (k, H)), rng.normal(0, 0.1, k))


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    d, H, k, B = 6, 5, 4, 7
    X = rng.normal(size=(B, d))
    y = rng.integers(0, k, B)
    P = list(_params(rng, d, H, k))
    L, *G = mlp.gradients(X, y, *P)
    assert abs(L - mlp.loss(X, y, *P)) < 1e-12
    for pi in range(4):
        it = np.nditer(P[pi], flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            h = 1e-6 * max(1.0, abs(P[pi][idx]))
            Pp = [p.copy() for p in P]
            Pm = [p.copy() for p in P]
            Pp[pi][idx] += h
            Pm[pi][idx] -= h
            fd = (mlp.loss(X, y, *Pp) - mlp.loss(X, y, *Pm)) / (2 * h)
            assert abs(fd - G[pi][idx]) <= 1e-6 * max(1.0, abs(fd)), (pi, idx, fd, G[pi][idx])


def test_hand_worked_single_unit():
    # d=1, H=1, k=2: a = 2x + 0, h = relu(a); z0 = h, z1 = 0.
    # x = 1, y = 0: z = (2, 0), p0 = e^2 / (e^2 + 1), loss = log(1 + e^-2).
    W1 = np.array([[2.0]]); b1 = np.array([0.0])
    W2 = np.array([[1.0], [0.0]]); b2 = np.array([0.0, 0.0])
    X = np.array([[1.0]]); y = np.array([0])
    L, dW1, db1, dW2, db2 = mlp.gradients(X, y, W1, b1, W2, b2)
    p0 = np.e ** 2 / (np.e ** 2 + 1)
    assert abs(L - np.log(1 + np.e ** -2)) < 1e-15
    # dz = (p0 - 1, 1 - p0); dW2 = dz^T h with h = 2; dh = dz . W2[:,0] = p0 - 1
    assert np.allclose(dW2, [[2 * (p0 - 1)], [2 * (1 - p0)]])
    assert np.allclose(db2, [p0 - 1, 1 - p0])
    assert np.allclose(dW1, [[(p0 - 1) * 1.0]]) and np.allclose(db1, [p0 - 1])
    # a dead ReLU passes no gradient
    L2, dW1b, db1b, _, _ = mlp.gradients(np.array([[-1.0]]), y, W1, b1, W2, b2)
    assert dW1b[0, 0] == 0 and db1b[0] == 0


def test_adam_first_step_moves_by_lr_times_sign():
    # after one step with zero state the bias-corrected update is lr * g / (|g| + eps)
    p = [np.array([1.0, -2.0, 0.5])]
    g = [np.array([0.3, -4.0, 0.0])]
    z = [np.zeros(3)]
    (q,), (m,), (v,) = mlp.adam_step(p, g, z, z, 1, lr=0.01)
    expect = p[0] - 0.01 * g[0] / (np.abs(g[0]) + 1e-8)
    assert np.allclose(q, expect, rtol=0, atol=1e-12)
    assert np.allclose(m, 0.1 * g[0]) and np.allclose(v, 0.001 * g[0] ** 2)


def test_training_learns_a_separable_labelling():
    rng = np.random.default_rng(1)
    k, d, H = 4, 3, 16
    means = rng.normal(0, 3, (k, d))
    y = rng.integers(0, k, 400)
    X = means[y] + 0.3 * rng.normal(size=(400, d))
    P = list(_params(rng, d, H, k, 0.3))
    m = [np.zeros_like(p) for p in P]
    v = [np.zeros_like(p) for p in P]
    L0 = mlp.loss(X, y, *P)
    for t in range(1, 301):
        L, *G = mlp.gradients(X, y, *P)
        P, m, v = mlp.adam_step(P, G, m, v, t, lr=1e-2)
    assert mlp.loss(X, y, *P) < 0.2 * L0
    assert np.mean(mlp.predict(X, *P) == y) > 0.95


def test_planted_gradient_mistake_is_caught(monkeypatch):
    real = mlp.gradients

    def no_relu_mask(X, y, W1, b1, W2, b2):
        L, dW1, db1, dW2, db2 = real(X, y, W1, b1, W2, b2)
        A, Hd, Z = mlp.forward(X, W1, b1, W2, b2)
        # forget the ReLU derivative in the first layer
        Zm = Z - Z.max(1, keepdims=True); E = np.exp(Zm); P = E / E.sum(1, keepdims=True)
        dZ = P.copy(); dZ[np.arange(len(y)), y] -= 1; dZ /= len(y)
        dA = dZ @ W2
        return L, dA.T @ X, dA.sum(0), dW2, db2

    monkeypatch.setattr(mlp, "gradients", no_relu_mask)
    with pytest.raises(AssertionError):
        test_gradients_match_central_differences()


def test_propose_hand_worked():
    # k = 20: quarter of j is (j mod 16) div 4 -> quarter 0 = {0..3, 16..19},
    # quarter 1 = {4..7}, quarter 2 = {8..11}, quarter 3 = {12..15}
    z = np.zeros((1, 20))
    z[0, [17, 2, 0, 19]] = [9.0, 8.0, 7.0, 7.0]      # 0 and 19 tie: 0 first
    z[0, 5] = 3.0
    z[0, 13] = -1.0
    got = mlp.propose(z)[0]
    assert got[:4].tolist() == [17, 2, 0, 19]
    assert got[4:8].tolist() == [5, 4, 6, 7]            # ties among zeros: index order
    assert got[12:16].tolist() == [12, 14, 15, 13]
    # a quarter with fewer than four centers pads with -1 (k = 6: quarter 1 = {4, 5})
    g6 = mlp.propose(np.arange(6, dtype=float)[None, :])[0]
    assert g6[4:8].tolist() == [5, 4, -1, -1] and g6[8:].tolist() == [-1] * 8


def test_propose_against_sorting_and_global_top_four():
    rng = np.random.default_rng(3)
    for k in (1, 7, 16, 37, 64):
        Z = rng.integers(-3, 4, size=(25, k)).astype(float)   # many ties
        P = mlp.propose(Z)
        quarter = (np.arange(k) % 16) // 4
        for r in range(Z.shape[0]):
            for q in range(4):
                J = np.nonzero(quarter == q)[0]
                # brute force: sort by (-logit, index)
                order = sorted(J.tolist(), key=lambda j: (-Z[r, j], j))[:4]
                assert P[r, 4 * q:4 * q + len(order)].tolist() == order
                assert (P[r, 4 * q + len(order):4 * q + 4] == -1).all()
            top4 = sorted(range(k), key=lambda j: (-Z[r, j], j))[:4]
            assert set(top4) <= set(P[r][P[r] >= 0].tolist())
