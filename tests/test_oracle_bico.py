"""Pins of the FP64 BICO oracle (oracle/bico.py) against facts that do not
come from it: a weighted insertion worked by hand (Sec. 2.3.1), the
clustering-feature identity against direct sums (Sec. 2.1), conservation of
weight and sums, the threshold invariant, and weighted insertion against
inserting the copies one by one under the plain rule of Sec. 2.1 (a copy
joins a feature when the feature's recomputed cost stays within T).  CPU only."""
import os

import numpy as np
import pytest

from oracle import bico as ob

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split()
                out[k] = float(v)
    return out


def test_weighted_insert_worked_example():
    g = _golden("bico_weighted_insert.txt")
    b = ob.Bico(1, 10, 0.01)
    b.insert_point(np.array([0.0], np.float32), 100.0)
    b.insert_point(np.array([0.02], np.float32), 50.0)
    (W, S, Q, ref, level) = b.features()
    assert len(W) == 2
    assert W[0] == g["parent_W"] and W[1] == g["child_W"]
    assert W[0] - 100 == g["joined"]
    x = np.float64(np.float32(0.02))
    np.testing.assert_allclose(S[:, 0], [33 * x, 17 * x], rtol=1e-15)
    np.testing.assert_allclose([S[0, 0], S[1, 0]], [g["parent_S"], g["child_S"]], rtol=1e-7)
    np.testing.assert_allclose(Q, [g["parent_Q"], g["child_Q"]], rtol=1e-7)
    assert level.tolist() == [1, int(g["child_level"])]
    # the joined feature stays within T, one more copy would not
    f = b.roots[0]
    assert f.cost() <= 0.01
    assert (f.Q + x * x) - (f.S[0] + x) ** 2 / (f.W + 1) > 0.01


def test_feature_cost_identity():
    # Sec. 2.1: Q - ||S||^2 / W is the sum of squared distances to the centroid
    rng = np.random.default_rng(0)
    for n, d in [(1, 3), (7, 5), (200, 17)]:
        P = rng.normal(size=(n, d)).astype(np.float32).astype(np.float64)
        w = rng.integers(1, 5, n).astype(np.float64)
        f = ob.Feature(P[0], w.sum(), (w[:, None] * P).sum(0), (w * (P * P).sum(1)).sum(), 1, None)
        mu = (w[:, None] * P).sum(0) / w.sum()
        direct = float((w * ((P - mu) ** 2).sum(1)).sum())
        assert abs(f.cost() - direct) <= 1e-9 * max(1.0, direct)


def _data(n, d, seed, sigma=1.0):
    rng = np.random.default_rng(seed)
    means = rng.uniform(-5, 5, size=(6, d))
    return (means[rng.integers(0, 6, n)] + sigma * rng.normal(size=(n, d))).astype(np.float32)


@pytest.mark.parametrize("weighted", [False, True])
def test_summary_invariants(weighted):
    n, d, m = 1500, 6, 60
    X = _data(n, d, 1)
    w = np.random.default_rng(2).integers(1, 6, n).astype(np.float64) if weighted else None
    b = ob.summarize(X, m, 1e-3, w)
    W, S, Q, ref, level = b.features()
    ww = np.ones(n) if w is None else w
    X64 = X.astype(np.float64)
    assert b.count == len(W) <= m
    assert b.rebuilds > 0
    assert W.sum() == ww.sum()
    np.testing.assert_allclose(S.sum(0), (ww[:, None] * X64).sum(0), rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(Q.sum(), (ww * (X64 * X64).sum(1)).sum(), rtol=1e-12)
    cost = Q - (S * S).sum(1) / W
    assert np.all(cost <= b.T * (1 + 1e-9))
    assert np.all(W > 0)
    # levels: a feature of level i > 1 sits below one of level i - 1
    for f in b.bfs():
        for g in f.kids:
            assert g.level == f.level + 1


class _CopyBico(ob.Bico):
    """Unweighted BICO that admits one copy when the feature's recomputed cost
    with it stays within T (the plain rule of Sec. 2.1)."""

    def insert_copy(self, x):
        x = np.asarray(x, np.float32)
        xd = x.astype(np.float64)
        q = ob._seqsum(xd * xd)
        siblings, parent, level = self.roots, None, 1
        while True:
            f, dd = self._closest(siblings, x)
            if f is None or dd > self.radius2(level):
                self._open(siblings, x, 1.0, xd, q, level, parent)
                break
            W, S, Q = f.W + 1, f.S + xd, f.Q + q
            if Q - ob._seqsum(S * S) / W <= self.T:
                f.W, f.S, f.Q = W, S, Q
                break
            siblings, parent, level = f.kids, f, level + 1


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_weighted_equals_copies(seed):
    # Sec. 2.3.1: w copies of x inserted as one weighted point give the
    # features that inserting the copies one at a time gives (no rebuild: m
    # is large, so every copy sees the same tree as the weighted point)
    rng = np.random.default_rng(seed)
    n, d = 300, 4
    X = _data(n, d, seed, sigma=0.05)
    w = rng.integers(1, 7, n)
    T0 = 0.5
    a = ob.summarize(X, 10 ** 6, T0, w.astype(np.float64))
    b = _CopyBico(d, 10 ** 6, T0)
    for i in range(n):
        for _ in range(int(w[i])):
            b.insert_copy(X[i])
    assert a.rebuilds == 0 and b.rebuilds == 0
    Wa, Sa, Qa, ra, la = a.features()
    Wb, Sb, Qb, rb, lb = b.features()
    assert len(Wa) == len(Wb)
    assert np.array_equal(Wa, Wb)
    assert np.array_equal(ra, rb) and np.array_equal(la, lb)
    np.testing.assert_allclose(Sa, Sb, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Qa, Qb, rtol=1e-12)
    # the copies descended somewhere (the test exercises w' < w)
    assert la.max() > 1
