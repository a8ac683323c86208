"""Pins of the FP64 oracle against facts that do not come from the oracle
itself: hand-worked examples, library routines, brute force, closed forms,
invariants stated in the paper and printed values.  CPU only."""
import itertools
import os

import numpy as np
import pytest
import scipy.spatial.distance as ssd
import scipy.stats

import synth
from oracle import kmeans as ok

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append(line.split())
    return rows


# --------------------------------------------------------------------------
# Random stream (reading S6)
# --------------------------------------------------------------------------
def test_splitmix64_reference_vectors():
    rows = _golden("splitmix64.txt")
    for seed, idx, val in rows:
        seed, idx, val = int(seed), int(idx), int(val)
        assert ok.splitmix64(seed, idx + 1)[idx] == val


def test_uniforms_are_53bit_fractions():
    u = ok.uniforms(0, 3)
    # 0xE220A8397B1DCDAF >> 11, divided by 2^53, computed by hand from the
    # reference output: 0xE220A8397B1DC / 2^53 with the low 11 bits dropped.
    assert u[0] == (16294208416658607535 >> 11) / 2.0 ** 53
    assert np.all((u >= 0) & (u < 1))


# --------------------------------------------------------------------------
# Distances and assignment (Sec. 1)
# --------------------------------------------------------------------------
def test_sqdist_hand_example():
    # Four points and two centers in the plane, distances worked by hand.
    X = np.array([[0, 0], [1, 0], [4, 4], [5, 3]], dtype=np.float32)
    C = np.array([[0, 1], [4, 3]], dtype=np.float32)
    D = ok.sqdist(X, C)
    expect = np.array([[1, 25], [2, 18], [25, 1], [29, 1]], dtype=np.float64)
    assert np.array_equal(D, expect)
    lab, d1, d2 = ok.assign(X, C)
    assert lab.tolist() == [0, 0, 1, 1]
    assert d1.tolist() == [1, 2, 1, 1]
    assert d2.tolist() == [25, 18, 25, 29]
    # cost = 1 + 2 + 1 + 1; new centers = means of the two pairs
    assert ok.cost(X, None, C) == 5.0
    Cn, W, S, Q = ok.update(X, None, lab, C)
    assert np.array_equal(Cn, np.array([[0.5, 0.0], [4.5, 3.5]]))
    assert W.tolist() == [2, 2]
    assert Q.tolist() == [1.0, 32.0 + 34.0]


def test_sqdist_matches_scipy_cdist():
    rng = np.random.default_rng(1)
    for n, k, d in [(50, 7, 3), (33, 1, 64), (20, 20, 129)]:
        X = rng.normal(size=(n, d)).astype(np.float32)
        C = rng.normal(size=(k, d)).astype(np.float32)
        ref = ssd.cdist(X.astype(np.float64), C.astype(np.float64), "sqeuclidean")
        np.testing.assert_allclose(ok.sqdist(X, C), ref, rtol=1e-13, atol=1e-12)


def test_assign_ties_go_to_lowest_index_and_k1():
    X = np.array([[0.0], [2.0]], dtype=np.float32)
    C = np.array([[1.0], [1.0], [3.0]], dtype=np.float32)
    lab, d1, d2 = ok.assign(X, C)
    assert lab.tolist() == [0, 0]          # centers 0 and 1 tie: lower index
    assert d1.tolist() == [1.0, 1.0] and d2.tolist() == [1.0, 1.0]
    lab, d1, d2 = ok.assign(X, C[:1])
    assert lab.tolist() == [0, 0] and np.all(np.isinf(d2))


# --------------------------------------------------------------------------
# Update step (Sec. 1 centroid step; Sec. 2 centroid; Sec. 2.1 features)
# --------------------------------------------------------------------------
def test_update_equals_bincount_means():
    rng = np.random.default_rng(2)
    n, d, k = 400, 5, 6
    X = rng.normal(size=(n, d)).astype(np.float32)
    w = rng.uniform(0.1, 3.0, size=n).astype(np.float32)
    lab = rng.integers(0, k, size=n)
    C_prev = rng.normal(size=(k, d))
    Cn, W, S, Q = ok.update(X, w, lab, C_prev)
    Wb = np.bincount(lab, weights=w.astype(np.float64), minlength=k)
    for t in range(d):
        Sb = np.bincount(lab, weights=w.astype(np.float64) * X[:, t], minlength=k)
        np.testing.assert_allclose(Cn[:, t], Sb / Wb, rtol=1e-13)
    np.testing.assert_allclose(W, Wb, rtol=1e-14)


def test_empty_cluster_keeps_previous_center():
    X = np.array([[0.0, 0.0], [1.0, 1.0]], dtype=np.float32)
    C_prev = np.array([[0.0, 0.0], [9.0, 9.0], [1.0, 1.0]])
    lab = np.array([0, 2])
    Cn, W, _, _ = ok.update(X, None, lab, C_prev)
    assert W.tolist() == [1, 0, 1]
    assert np.array_equal(Cn[1], C_prev[1])


def test_weighted_equals_replicated():
    # A point of integer weight w behaves as w copies (Sec. 2.3.1).
    rng = np.random.default_rng(3)
    n, d, k = 40, 3, 4
    X = rng.integers(-5, 6, size=(n, d)).astype(np.float32)
    w = rng.integers(1, 4, size=n)
    Xr = np.repeat(X, w, axis=0)
    C = rng.integers(-5, 6, size=(k, d)).astype(np.float32)
    lab, d1, _ = ok.assign(X, C)
    labr, d1r, _ = ok.assign(Xr, C)
    assert np.array_equal(np.repeat(lab, w), labr)
    assert ok.cost(X, w, C) == ok.cost(Xr, None, C)
    Cn, W, S, Q = ok.update(X, w, lab, C)
    Cr, Wr, Sr, Qr = ok.update(Xr, None, labr, C)
    np.testing.assert_allclose(Cn, Cr, rtol=1e-14)
    assert np.array_equal(W, Wr) and np.array_equal(S, Sr) and np.array_equal(Q, Qr)
    # seeding: with integer data every prefix is exact, so the same u picks a
    # copy of the same point (copies are laid out contiguously).
    for s in range(20):
        _, idx, _ = ok.seed(X, w, 3, s)
        _, idxr, _ = ok.seed(Xr, None, 3, s)
        owner = np.repeat(np.arange(n), w)
        assert np.array_equal(X[idx], Xr[idxr])
        assert np.array_equal(idx, owner[idxr])


def test_clustering_feature_identity():
    # sum ||x - c||^2 = |P| ||mu - c||^2 + sum ||x - mu||^2   (Sec. 2.1)
    rng = np.random.default_rng(4)
    n, d, k = 300, 7, 5
    X = rng.normal(size=(n, d)).astype(np.float32)
    w = rng.uniform(0.5, 2, size=n).astype(np.float32)
    C = rng.normal(size=(k, d))
    lab, d1, _ = ok.assign(X, C)
    W, S, Q = ok.clustering_features(X, w, lab, k)
    direct = float(np.sum(w.astype(np.float64) * d1))
    assert abs(ok.cost_from_features(W, S, Q, C) - direct) <= 1e-12 * direct
    # k = 1 closed form: cost(c) = cost(mu) + W ||mu - c||^2
    W1, S1, Q1 = ok.clustering_features(X, w, np.zeros(n, dtype=int), 1)
    mu = S1[0] / W1[0]
    c = rng.normal(size=d)
    lhs = ok.cost(X, w, c[None, :])
    rhs = ok.cost_at_centroids(W1, S1, Q1) + W1[0] * np.sum((mu - c) ** 2)
    assert abs(lhs - rhs) <= 1e-12 * lhs


def test_weighted_insertion_error_formula():
    # Adding w copies of x to a feature with s points and centroid mu raises
    # its error by s w / (s + w) ||x - mu||^2   (Sec. 2.3.1 derivation).
    rng = np.random.default_rng(5)
    for _ in range(20):
        s, d = int(rng.integers(1, 30)), int(rng.integers(1, 6))
        P = rng.normal(size=(s, d))
        x = rng.normal(size=d) * 3
        wgt = float(rng.uniform(0.5, 10))
        W0, S0, Q0 = ok.clustering_features(P, None, np.zeros(s, int), 1)
        Pw = np.vstack([P, x])
        ww = np.concatenate([np.ones(s), [wgt]])
        W1, S1, Q1 = ok.clustering_features(Pw, ww, np.zeros(s + 1, int), 1)
        inc = ok.cost_at_centroids(W1, S1, Q1) - ok.cost_at_centroids(W0, S0, Q0)
        mu = P.mean(0)
        expect = s * wgt / (s + wgt) * np.sum((x - mu) ** 2)
        assert abs(inc - expect) <= 1e-9 * max(1.0, expect)


# --------------------------------------------------------------------------
# Lloyd (Sec. 1): monotone cost, brute-force optimum, library cross-check
# --------------------------------------------------------------------------
def test_lloyd_cost_never_increases():
    rng = np.random.default_rng(6)
    for trial in range(100):
        n, d, k = int(rng.integers(5, 60)), int(rng.integers(1, 6)), int(rng.integers(1, 6))
        k = min(k, n)
        X = rng.normal(size=(n, d)).astype(np.float32)
        w = rng.uniform(0.1, 2, size=n).astype(np.float32) if trial % 2 else None
        C0 = X[rng.choice(n, k, replace=False)]
        res = ok.lloyd(X, w, C0, 15, f32_centers=False)
        c = res["cost"]
        assert np.all(c[1:] <= c[:-1] * (1 + 1e-12))


def _all_partitions_cost(X, k):
    n = X.shape[0]
    best = np.inf
    best_lab = None
    for lab in itertools.product(range(k), repeat=n):
        lab = np.array(lab)
        if len(set(lab.tolist())) != k:
            continue
        c = 0.0
        for j in range(k):
            P = X[lab == j].astype(np.float64)
            c += float(np.sum((P - P.mean(0)) ** 2))
        if c < best:
            best, best_lab = c, lab
    return best, best_lab


def test_lloyd_against_brute_force_optimum():
    rng = np.random.default_rng(7)
    for trial in range(12):
        n, k, d = int(rng.integers(4, 9)), int(rng.integers(2, 4)), 2
        X = rng.normal(size=(n, d)).astype(np.float32)
        opt, lab = _all_partitions_cost(X, k)
        # the optimal partition's centroids are a fixed point of Lloyd
        Copt = np.array([X[lab == j].astype(np.float64).mean(0) for j in range(k)])
        res = ok.lloyd(X, None, Copt, 5, f32_centers=False)
        assert abs(res["cost"][-1] - opt) <= 1e-12 * max(opt, 1e-300)
        assert np.all(np.abs(res["cost"] - opt) <= 1e-12 * max(opt, 1e-300))
        # any start ends at or above the optimum; the best of many seeds reaches it
        best = np.inf
        for s in range(40):
            C0, _, _ = ok.seed(X, None, k, s)
            r = ok.lloyd(X, None, C0, 30, f32_centers=False)
            assert r["cost"][-1] >= opt * (1 - 1e-12)
            best = min(best, r["cost"][-1])
        assert best <= opt * (1 + 1e-12)


def test_lloyd_matches_sklearn_on_tie_free_data():
    from sklearn.cluster import KMeans
    X, _ = synth.isotropic_mixture(600, 8, 5, seed=11)
    X64 = X.astype(np.float64)
    C0 = X64[[0, 1, 2, 3, 4]]
    T = 6
    res = ok.lloyd(X, None, C0, T, f32_centers=False)
    km = KMeans(n_clusters=5, init=C0, n_init=1, algorithm="lloyd", max_iter=T, tol=0.0)
    km.fit(X64)
    np.testing.assert_allclose(res["C"], km.cluster_centers_, rtol=1e-10, atol=1e-10)
    assert np.array_equal(res["labels"], km.labels_)
    assert abs(res["cost"][-1] - km.inertia_) <= 1e-9 * km.inertia_


def test_lloyd_early_stop_when_labels_stable():
    X, _ = synth.isotropic_mixture(300, 4, 3, seed=12)
    C0 = X[:3]
    res = ok.lloyd(X, None, C0, 50, tol=0.0)
    assert res["iters"] < 50
    fixed = ok.lloyd(X, None, C0, res["iters"])
    np.testing.assert_array_equal(res["C"], fixed["C"])


def test_lowerbound_closed_form_and_table2():
    # Small member of the family: Lloyd from the generating vertices' centroids
    # stays there with cost (delta^2/2)(n - k).
    delta, Delta = 100.0, 1000.0
    k, n = 5, 100
    X, lab = synth.lowerbound(k, n, delta, Delta)
    C = np.array([X[lab == j].mean(0) for j in range(k)])
    res = ok.lloyd(X, None, C, 3, f32_centers=False)
    closed = delta ** 2 / 2 * (n - k)
    assert np.all(np.abs(res["cost"] - closed) <= 1e-9 * closed)
    assert np.array_equal(res["labels"], lab)
    # the same closed form reproduces the optima printed in Table 2
    for kk, nn, dd, printed in _golden("lowerbound_table2.txt"):
        kk, nn, dd, printed = int(kk), int(nn), int(dd), float(printed)
        assert dd == kk + nn
        assert abs(delta ** 2 / 2 * (nn - kk) - printed) <= 1e-12 * printed


# --------------------------------------------------------------------------
# k-means++ (Sec. 1; weighted summary Sec. 2.2)
# --------------------------------------------------------------------------
def test_kmeanspp_hand_worked_line():
    # Points 0, 1, 3, 7, 15 on a line, unit weights, rng seed 0:
    #  u0 = 0.88330..., u1 = 0.43153..., u2 = 0.02643... (reference outputs / 2^64)
    #  round 0: prefix of weights 1..5 first exceeds 4.416 at index 4 (x = 15)
    #  round 1: D2 = 225,196,144,64,0 (M=629); target 271.4 -> index 1 (x = 1)
    #  round 2: D2 = 1,0,4,36,0 (M=41); target 1.08 -> prefix 1,1,5 -> index 2
    X = np.array([[0], [1], [3], [7], [15]], dtype=np.float32)
    C, idx, u = ok.seed(X, None, 3, 0)
    assert abs(u[0] - 0.8833) < 1e-4 and abs(u[1] - 0.4315) < 1e-4 and abs(u[2] - 0.02643) < 1e-4
    assert idx.tolist() == [4, 1, 2]
    assert C[:, 0].tolist() == [15.0, 1.0, 3.0]


def test_kmeanspp_zero_mass_falls_back_to_unchosen():
    X = np.array([[1, 1], [1, 1], [1, 1], [2, 2]], dtype=np.float32)
    C, idx, _ = ok.seed(X, None, 4, 3)
    assert sorted(idx.tolist()) == [0, 1, 2, 3]


def test_kmeanspp_zero_weight_never_chosen():
    rng = np.random.default_rng(8)
    X = rng.normal(size=(30, 3)).astype(np.float32)
    w = np.ones(30, dtype=np.float32)
    w[::3] = 0
    for s in range(30):
        _, idx, _ = ok.seed(X, w, 5, s)
        assert np.all(w[idx] > 0)


def test_kmeanspp_all_positive_weights_used_then_raises():
    # Sec. 2.3.1: a weight-w point stands for w copies, so zero-weight points
    # stand for nothing.  With exactly k positive weights (duplicates, zero D2
    # mass after a few rounds) every positive row is drawn; one more center
    # has no point left to be drawn from and must be refused, not invented.
    X = np.array([[1, 1], [1, 1], [4, 0], [1, 1], [9, 9]], dtype=np.float32)
    w = np.array([1, 0, 2, 3, 0], dtype=np.float32)
    for s in range(10):
        _, idx, _ = ok.seed(X, w, 3, s)
        assert sorted(idx.tolist()) == [0, 2, 3]
    with pytest.raises(ValueError):
        ok.seed(X, w, 4, 0)
    with pytest.raises(ValueError):
        ok.seed(X, np.zeros(5, np.float32), 1, 0)
    with pytest.raises(ValueError):
        ok.seed(X, np.array([1, -1, 1, 1, 1], np.float32), 2, 0)
    with pytest.raises(ValueError):
        ok.seed(X, np.array([1, np.nan, 1, 1, 1], np.float32), 2, 0)
    with pytest.raises(ValueError):
        ok.seed(X, None, 6, 0)


def test_kmeanspp_sampling_law_chi_square():
    # P(i0, i1) = w_i0 / sum w * w_i1 D2(i1, i0) / sum_j w_j D2(j, i0)
    X = np.array([[0, 0], [1, 0], [0, 2], [3, 3], [-2, 1], [5, -1]], dtype=np.float32)
    w = np.array([1, 2, 1, 3, 1, 2], dtype=np.float32)
    n = X.shape[0]
    N = 6000
    counts = np.zeros((n, n))
    for s in range(N):
        _, idx, _ = ok.seed(X, w, 2, 1000 + s)
        counts[idx[0], idx[1]] += 1
    X64 = X.astype(np.float64)
    w64 = w.astype(np.float64)
    expect = np.zeros((n, n))
    for a in range(n):
        D2 = np.sum((X64 - X64[a]) ** 2, axis=1)
        expect[a] = w64[a] / w64.sum() * (w64 * D2) / np.sum(w64 * D2)
    expect /= expect.sum()
    mask = expect > 0
    assert counts[~mask].sum() == 0
    stat = scipy.stats.chisquare(counts[mask], N * expect[mask])
    assert stat.pvalue > 1e-4


# --------------------------------------------------------------------------
# Sensitivity: plausible mistakes planted in the oracle must trip a pin.
# --------------------------------------------------------------------------
def _mutants():
    real = ok.sqdist

    def drop_last_coord(X, C, block=32):
        X = np.asarray(X, np.float64)[:, :-1] if np.asarray(X).shape[1] > 1 else np.asarray(X, np.float64)
        C = np.asarray(C, np.float64)[:, :X.shape[1]]
        return real(X, C, block)

    def sign_flip(X, C, block=32):
        return real(X, -np.asarray(C, np.float64), block)

    def transposed(X, C, block=32):
        X = np.asarray(X, np.float64)
        C = np.asarray(C, np.float64)
        return real(X[:, ::-1], C, block)

    return [drop_last_coord, sign_flip, transposed]


@pytest.mark.parametrize("mutant", _mutants(), ids=["drop_term", "sign", "transpose"])
def test_planted_distance_mistakes_are_caught(monkeypatch, mutant):
    monkeypatch.setattr(ok, "sqdist", mutant)
    with pytest.raises(AssertionError):
        test_sqdist_hand_example()


def test_planted_update_mistake_is_caught(monkeypatch):
    real = ok.clustering_features

    def unweighted(X, w, labels, k):
        return real(X, None, labels, k)

    monkeypatch.setattr(ok, "clustering_features", unweighted)
    with pytest.raises(AssertionError):
        test_update_equals_bincount_means()


def test_planted_seeding_mistake_is_caught(monkeypatch):
    def exclusive_prefix(mass, u):   # off by one: tests the prefix before adding
        total = float(np.sum(mass))
        run = 0.0
        for i, v in enumerate(mass):
            if run > u * total:
                return i
            run += v
        return len(mass) - 1

    monkeypatch.setattr(ok, "_inverse_cdf", exclusive_prefix)
    with pytest.raises(AssertionError):
        test_kmeanspp_hand_worked_line()
