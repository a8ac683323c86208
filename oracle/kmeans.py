"""FP64 CPU oracle for weighted k-means++ seeding and Lloyd's algorithm.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this module.  It shares no code
with the HIP library (``paper_1502_04265_amd``) and imports nothing from it.

Every function is the plain definition of what the method computes, written
for a reader who checks it against the paper by eye:

* k-means objective: sum over points of the squared Euclidean distance to the
  nearest center (Sec. 1, definition of the k-means problem); for weighted
  points each point counts w times (Sec. 1, coreset definition; Sec. 2.3.1,
  a weighted point stands for w copies).
* Lloyd's algorithm: alternate "assign every point to its closest center" and
  "replace each center by the centroid of its subset" (Sec. 1, Lloyd's
  algorithm and its footnote on stopping rules).
* Centroid mu(P) = sum x / |P| (Sec. 2, notation); weighted: sum w x / sum w.
* Clustering feature (|S|, sum x, sum x^T x) and the identity
  sum ||x-c||^2 = |P| ||mu(P)-c||^2 + sum ||x-mu(P)||^2 (Sec. 2.1).
* k-means++: first center uniformly at random, every further center drawn with
  probability proportional to the squared distance to the closest center
  chosen so far (Sec. 1, k-means++ paragraph), run on the weighted summary
  (Sec. 2.2, "Obtaining a solution").

Arithmetic: inputs are promoted exactly to float64; distances are direct
differences sum_i (x_i - c_i)^2 (no ||x||^2 - 2x.c + ||c||^2 expansion); all
sums are float64.  Readings where the paper is silent (tie-break, empty
cluster, weighted first draw, zero D^2 mass, inverse-CDF convention, random
number stream, stopping rule) are listed in the module constants below and
in the design notes.

Readings adopted where the paper is silent:
  S1  argmin ties go to the lowest center index.
  S2  an empty cluster keeps its previous center.
  S3  with weights, the first center is drawn with probability proportional
      to w_i (uniform when all weights are equal).
  S4  if the remaining D^2 mass is zero, draw by weight among the points not
      chosen yet.
  S5  inverse CDF: the first index whose inclusive prefix strictly exceeds
      u * total, u in [0, 1).
  S6  random numbers: SplitMix64 (Steele, Lea, Flood 2014), the r-th output
      mapped to (z >> 11) * 2^-53, r = 0 .. k-1.
  S8  stopping: a fixed number of iterations, or (tol >= 0) stop once the
      labels do not change or the relative cost decrease is <= tol.
  S9  the reported final cost is cost(C_T), from one more assignment.
"""
from __future__ import annotations

import numpy as np

_MASK64 = (1 << 64) - 1


# ----------------------------------------------------------------------------
# Random numbers (reading S6): SplitMix64, published by Steele, Lea and Flood
# (OOPSLA 2014).  Written out with Python integers so every step is visible.
# ----------------------------------------------------------------------------
def splitmix64(seed: int, count: int) -> list[int]:
    """The first ``count`` SplitMix64 outputs for state ``seed``."""
    state = seed & _MASK64
    out = []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & _MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        z = z ^ (z >> 31)
        out.append(z)
    return out


def uniforms(seed: int, count: int) -> np.ndarray:
    """u_r = (z_r >> 11) * 2^-53 in [0, 1), r = 0 .. count-1 (reading S6)."""
    return np.array([(z >> 11) * (2.0 ** -53) for z in splitmix64(seed, count)],
                    dtype=np.float64)


# ----------------------------------------------------------------------------
# Distances (Sec. 1: squared Euclidean distance).
# ----------------------------------------------------------------------------
def _f64(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float64)


def _weights(w, n: int) -> np.ndarray:
    if w is None:
        return np.ones(n, dtype=np.float64)
    return _f64(w).reshape(n)


def sqdist(X, C, block: int = 32) -> np.ndarray:
    """D[i, j] = sum_t (X[i, t] - C[j, t])^2, by direct differences in float64."""
    X = _f64(X)
    C = _f64(C)
    n, k = X.shape[0], C.shape[0]
    D = np.empty((n, k), dtype=np.float64)
    for s in range(0, n, block):
        diff = X[s:s + block, None, :] - C[None, :, :]
        D[s:s + block] = np.sum(diff * diff, axis=2)
    return D


def assign(X, C):
    """Assignment step of Lloyd's algorithm (Sec. 1).

    Returns (labels, d1, d2): labels[i] = argmin_j D(x_i, c_j) with ties to the
    lowest j (reading S1); d1 = that smallest distance; d2 = the second
    smallest over the other centers (+inf when k = 1).
    """
    D = sqdist(X, C)
    labels = np.argmin(D, axis=1)          # numpy argmin returns the first minimum
    rows = np.arange(D.shape[0])
    d1 = D[rows, labels]
    if D.shape[1] == 1:
        d2 = np.full(D.shape[0], np.inf)
    else:
        rest = D.copy()
        rest[rows, labels] = np.inf
        d2 = rest.min(axis=1)
    return labels.astype(np.int64), d1, d2


def cost(X, w, C) -> float:
    """Weighted k-means cost sum_i w_i min_j D(x_i, c_j) (Sec. 1, coreset cost)."""
    X = _f64(X)
    _, d1, _ = assign(X, C)
    return float(np.sum(_weights(w, X.shape[0]) * d1))


# ----------------------------------------------------------------------------
# Update step: weighted clustering features and centroids (Sec. 2, Sec. 2.1,
# Sec. 2.3.1 "new clustering feature (w, w x, w x^T x)").
# ----------------------------------------------------------------------------
def clustering_features(X, w, labels, k: int):
    """Per-cluster weighted clustering feature (W_j, S_j, Q_j).

    W_j = sum w_i, S_j = sum w_i x_i, Q_j = sum w_i ||x_i||^2 over a_i = j.
    Each cluster is summed by an explicit loop over its members.
    """
    X = _f64(X)
    n, d = X.shape
    w = _weights(w, n)
    labels = np.asarray(labels).reshape(n)
    W = np.zeros(k)
    S = np.zeros((k, d))
    Q = np.zeros(k)
    for j in range(k):
        members = np.nonzero(labels == j)[0]
        if members.size == 0:
            continue
        wm = w[members]
        xm = X[members]
        W[j] = np.sum(wm)
        S[j] = np.sum(wm[:, None] * xm, axis=0)
        Q[j] = np.sum(wm * np.sum(xm * xm, axis=1))
    return W, S, Q


def update(X, w, labels, C_prev):
    """Replace every center by the weighted centroid of its subset (Sec. 1).

    c_j = S_j / W_j when W_j > 0, else the previous center (reading S2).
    Returns (C_new float64, W, S, Q).
    """
    C_prev = _f64(C_prev)
    k = C_prev.shape[0]
    W, S, Q = clustering_features(X, w, labels, k)
    C_new = C_prev.copy()
    nonempty = W > 0
    C_new[nonempty] = S[nonempty] / W[nonempty, None]
    return C_new, W, S, Q


def cost_from_features(W, S, Q, C) -> float:
    """Cost of a fixed partition against centers C via the clustering-feature
    identity (Sec. 2.1): sum_{x in P_j} w||x - c_j||^2 = Q_j - 2 c_j.S_j + W_j||c_j||^2.
    """
    C = _f64(C)
    return float(np.sum(Q - 2.0 * np.sum(C * S, axis=1) + W * np.sum(C * C, axis=1)))


def cost_at_centroids(W, S, Q) -> float:
    """Cost of the partition against its own centroids: sum_j Q_j - ||S_j||^2 / W_j
    (Sec. 2.1 identity with c = mu(P_j))."""
    nz = W > 0
    return float(np.sum(Q[nz] - np.sum(S[nz] * S[nz], axis=1) / W[nz]))


# ----------------------------------------------------------------------------
# k-means++ seeding on weighted points (Sec. 1 k-means++; Sec. 2.2 run on the
# weighted summary; a weight-w point stands for w copies, Sec. 2.3.1).
# ----------------------------------------------------------------------------
def _inverse_cdf(mass: np.ndarray, u: float) -> int:
    """First index whose inclusive prefix of ``mass`` strictly exceeds u * total
    (reading S5).  The prefix is accumulated sequentially in index order.
    A draw from zero total mass is undefined and raises."""
    total = 0.0
    for v in mass:
        total += v
    if not total > 0.0:
        raise ValueError("inverse CDF of zero total mass")
    target = u * total
    run = 0.0
    last_positive = -1
    for i, v in enumerate(mass):
        run += v
        if v > 0:
            last_positive = i
        if run > target:
            return i
    # u * total rounds onto the total: the last index carrying mass.
    return last_positive


def seed(X, w, k: int, rng_seed: int):
    """Weighted k-means++ seeding.  Returns (C float64 k x d, idx int64 k, u).

    Round 0 draws i_0 with probability proportional to w_i (reading S3).
    Round r >= 1 draws i_r with probability proportional to w_i * D2_i, where
    D2_i is the squared distance of x_i to its closest chosen center; if that
    mass is zero, it draws by weight among the points not chosen yet (S4).
    The draws use u_r from SplitMix64 (S6) through the inverse CDF (S5).

    A weight-w point stands for w copies (Sec. 2.3.1), so a zero-weight point
    stands for none and k-means++ can only draw k centers from at least k
    points of positive weight: k > #{w_i > 0}, or a negative or non-finite
    weight, raises ValueError.
    """
    X = _f64(X)
    n = X.shape[0]
    w = _weights(w, n)
    if not np.all(np.isfinite(w)) or np.any(w < 0):
        raise ValueError("weights must be finite and >= 0")
    if not 1 <= k <= int(np.count_nonzero(w > 0)):
        raise ValueError(f"k = {k} needs 1 <= k <= #points of positive weight "
                         f"({int(np.count_nonzero(w > 0))})")
    u = uniforms(rng_seed, k)
    chosen = np.zeros(n, dtype=bool)
    idx = np.empty(k, dtype=np.int64)

    idx[0] = _inverse_cdf(w, u[0])
    chosen[idx[0]] = True
    D2 = sqdist(X, X[idx[0]][None, :])[:, 0]
    for r in range(1, k):
        mass = w * D2
        if np.sum(mass) > 0:
            i = _inverse_cdf(mass, u[r])
        else:
            i = _inverse_cdf(np.where(chosen, 0.0, w), u[r])
        idx[r] = i
        chosen[i] = True
        D2 = np.minimum(D2, sqdist(X, X[i][None, :])[:, 0])
    return X[idx].copy(), idx, u


# ----------------------------------------------------------------------------
# Lloyd's algorithm (Sec. 1 and its footnote).
# ----------------------------------------------------------------------------
def lloyd(X, w, C0, max_iter: int, tol: float = -1.0, f32_centers: bool = True):
    """Weighted Lloyd iterations from C0.

    Iteration t: assign against C_t (cost[t] = cost(C_t)), then C_{t+1} = the
    weighted centroids (empty clusters keep their center).  tol < 0 runs
    exactly max_iter iterations; tol >= 0 stops after iteration t when the
    labels equal those of iteration t-1 or the relative decrease of the cost
    is <= tol (footnote to Lloyd's algorithm, reading S8).  One more
    assignment gives cost[T] = cost(C_T) and the returned labels (S9).

    ``f32_centers`` stores each C_{t+1} as float32, the format in which centers
    cross the library boundary; the arithmetic itself stays float64.
    """
    X = _f64(X)
    n = X.shape[0]
    w = _weights(w, n)
    C = _f64(C0).copy()
    if f32_centers:
        C = C.astype(np.float32).astype(np.float64)
    cost_hist = []
    prev_labels = None
    iters = 0
    for t in range(max_iter):
        labels, d1, _ = assign(X, C)
        cost_hist.append(float(np.sum(w * d1)))
        C_new, _, _, _ = update(X, w, labels, C)
        if f32_centers:
            C_new = C_new.astype(np.float32).astype(np.float64)
        C = C_new
        iters = t + 1
        if tol >= 0:
            same = prev_labels is not None and np.array_equal(labels, prev_labels)
            small = t >= 1 and (cost_hist[-2] - cost_hist[-1]) <= tol * cost_hist[-2]
            if same or small:
                break
        prev_labels = labels
    labels, d1, d2 = assign(X, C)
    cost_hist.append(float(np.sum(w * d1)))
    return {"C": C, "labels": labels, "d1": d1, "d2": d2,
            "cost": np.array(cost_hist), "iters": iters}
