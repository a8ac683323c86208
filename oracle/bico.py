"""FP64 reference of the BICO summary (test infrastructure only).

BICO (Sec. 2.1) keeps clustering features CF = (W, S, Q) -- weight, weighted
sum of the points, weighted sum of their squared lengths -- in a tree of
spheres.  The cost of the points of a feature against its centroid S / W
follows from the identity of Sec. 2.1:  Q - ||S||^2 / W.  A point goes to the
feature whose reference point is closest among the children of the current
node; it opens a new feature when no reference lies within the level's
radius, joins the feature when the feature's cost stays within the threshold
T, and otherwise descends to that feature's children.  When there are more
than m features the threshold grows and the tree is rebuilt (Sec. 2.1, the
rebuilding step).  Weighted points follow Sec. 2.3.1: w copies of x open a
feature (w, w x, w ||x||^2) together, and at most w' of them join an existing
feature, the rest descending:
    w' = min(w, (sT - sc) / (s ||x - mu||^2 - T + c))   if s ||x - mu||^2 - T + c > 0,
    w' = w                                               otherwise,
with s = W, mu = S / W and c the feature's cost.

Readings where the paper leaves BICO's internals to its authors' publication:
  B1  the radius of level i (children of the root: level 1) is
      R_i = sqrt(T / 2^(3 + i)), the published BICO's choice;
  B2  "closest" is by the exact squared distance to the reference point;
      ties go to the oldest feature (creation order);
  B3  w' is rounded down (the paper's weights are integral: footnote to
      Sec. 2.3.2), and no copies join when it rounds to zero;
  B4  a rebuild doubles T and re-inserts every feature, in breadth-first order
      of the old tree (each level in creation order), into an empty tree: a
      feature follows its reference point down the tree like a point, merges
      into the closest feature within the radius when the merged cost stays
      within the new T, descends when it does not, and otherwise becomes a new
      feature with its (W, S, Q) and reference; rebuilds repeat while there
      are more than m features;
  B5  the starting threshold T_0 > 0 is an argument;
  B6  the summary is the features' centroids S / W with weights W, in
      breadth-first order.
Every sum over coordinates runs in index order (a sequential FP64 sum, the
order the library's host code uses), so both sides take each decision on the
same bits.
"""
from __future__ import annotations

import numpy as np


def _seqsum(v) -> float:
    """Sum of a FP64 vector in index order."""
    return float(np.cumsum(np.asarray(v, np.float64))[-1]) if len(v) else 0.0


def _sq(a, b) -> float:
    t = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    return _seqsum(t * t)


class Feature:
    __slots__ = ("ref", "W", "S", "Q", "kids", "level", "parent")

    def __init__(self, ref, W, S, Q, level, parent):
        self.ref = np.asarray(ref, np.float32).copy()
        self.W = float(W)
        self.S = np.asarray(S, np.float64).copy()
        self.Q = float(Q)
        self.kids = []
        self.level = level
        self.parent = parent

    def cost(self) -> float:
        """Q - ||S||^2 / W: the cost of the feature's points against their
        centroid (Sec. 2.1)."""
        return self.Q - _seqsum(self.S * self.S) / self.W


class Bico:
    """The summary: at most m features in R^d, threshold T."""

    def __init__(self, d: int, m: int, T0: float):
        if not T0 > 0:
            raise ValueError("the starting threshold must be positive")
        self.d = d
        self.m = m
        self.T = float(T0)
        self.roots = []          # level-1 features, creation order
        self.count = 0
        self.rebuilds = 0

    def radius2(self, level: int) -> float:
        """R_level^2 = T / 2^(3 + level) (reading B1)."""
        return self.T / 2.0 ** (3 + level)

    @staticmethod
    def _closest(cands, x):
        """The candidate whose reference is closest to x (the first, i.e. the
        oldest, among equal distances), with that squared distance; each
        distance is a sum in coordinate order."""
        if not cands:
            return None, None
        R = np.stack([f.ref for f in cands]).astype(np.float64)
        t = np.asarray(x, np.float64)[None, :] - R
        dd = np.cumsum(t * t, axis=1)[:, -1]
        i = int(np.argmin(dd))
        return cands[i], float(dd[i])

    def _open(self, siblings, ref, W, S, Q, level, parent):
        f = Feature(ref, W, S, Q, level, parent)
        siblings.append(f)
        self.count += 1
        return f

    def insert_point(self, x, w: float = 1.0):
        """w copies of x (Sec. 2.1; Sec. 2.3.1 for w != 1)."""
        x = np.asarray(x, np.float32)
        xd = x.astype(np.float64)
        q = _seqsum(xd * xd)
        siblings, parent, level = self.roots, None, 1
        w = float(w)
        while w > 0:
            f, dd = self._closest(siblings, x)
            if f is None or dd > self.radius2(level):
                self._open(siblings, x, w, w * xd, w * q, level, parent)
                break
            s, c = f.W, f.cost()
            mu = f.S / s
            D = _sq(xd, mu)
            den = s * D - self.T + c
            if den <= 0:
                wp = w
            else:
                wp = min(w, np.floor((s * self.T - s * c) / den))
            if wp > 0:
                f.W += wp
                f.S += wp * xd
                f.Q += wp * q
                w -= wp
            siblings, parent, level = f.kids, f, level + 1
        while self.count > self.m:
            self.rebuild()

    def bfs(self):
        out, layer = [], list(self.roots)
        while layer:
            out.extend(layer)
            layer = [g for f in layer for g in f.kids]
        return out

    def rebuild(self):
        """Double T and re-insert every feature into an empty tree (B4)."""
        old = self.bfs()
        self.T *= 2.0
        self.rebuilds += 1
        self.roots = []
        self.count = 0
        for f in old:
            siblings, parent, level = self.roots, None, 1
            while True:
                g, dd = self._closest(siblings, f.ref)
                if g is None or dd > self.radius2(level):
                    self._open(siblings, f.ref, f.W, f.S, f.Q, level, parent)
                    break
                W = g.W + f.W
                S = g.S + f.S
                Q = g.Q + f.Q
                if Q - _seqsum(S * S) / W <= self.T:
                    g.W, g.S, g.Q = W, S, Q
                    break
                siblings, parent, level = g.kids, g, level + 1

    def features(self):
        """(W, S, Q, ref, level) of every feature in breadth-first order."""
        fs = self.bfs()
        return (np.array([f.W for f in fs]), np.array([f.S for f in fs]).reshape(len(fs), self.d),
                np.array([f.Q for f in fs]), np.array([f.ref for f in fs]).reshape(len(fs), self.d),
                np.array([f.level for f in fs], np.int32))

    def coreset(self):
        """Centroids S / W and weights W (reading B6)."""
        W, S, _, _, _ = self.features()
        return S / W[:, None], W


def summarize(X, m: int, T0: float, w=None) -> Bico:
    """Insert the rows of X (with weights w) in order."""
    X = np.asarray(X, np.float32)
    b = Bico(X.shape[1], m, T0)
    for i in range(X.shape[0]):
        b.insert_point(X[i], 1.0 if w is None else float(w[i]))
    return b
