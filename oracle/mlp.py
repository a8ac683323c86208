"""FP64 reference of the candidate router's network (test infrastructure only).

The router is a two-layer perceptron d -> H (ReLU) -> k trained with softmax
cross-entropy on (point, label) pairs from earlier Lloyd iterations and
updated with Adam (Kingma & Ba 2015).  It is not part of the paper: the paper's
method only needs the exact assignment of Sec. 1, which the router's
certificate preserves.  This module is the plain definition the GPU kernels are
checked against; gradients are pinned by central finite differences in the
tests.

Shapes: W1 (H, d), b1 (H,), W2 (k, H), b2 (k,); X (B, d); y (B,) int.
"""
from __future__ import annotations

import numpy as np


def forward(X, W1, b1, W2, b2):
    """Returns (pre-activation A, hidden Hd, logits Z)."""
    X = np.asarray(X, np.float64)
    A = X @ np.asarray(W1, np.float64).T + np.asarray(b1, np.float64)
    Hd = np.maximum(A, 0.0)
    Z = Hd @ np.asarray(W2, np.float64).T + np.asarray(b2, np.float64)
    return A, Hd, Z


def loss(X, y, W1, b1, W2, b2) -> float:
    """Mean softmax cross-entropy of the labels y."""
    _, _, Z = forward(X, W1, b1, W2, b2)
    Zm = Z - Z.max(axis=1, keepdims=True)
    lse = np.log(np.sum(np.exp(Zm), axis=1))
    return float(np.mean(lse - Zm[np.arange(len(y)), np.asarray(y)]))


def gradients(X, y, W1, b1, W2, b2):
    """(loss, dW1, db1, dW2, db2) of the mean softmax cross-entropy, by the
    chain rule written out layer by layer."""
    X = np.asarray(X, np.float64)
    y = np.asarray(y)
    B = X.shape[0]
    A, Hd, Z = forward(X, W1, b1, W2, b2)
    Zm = Z - Z.max(axis=1, keepdims=True)
    E = np.exp(Zm)
    P = E / E.sum(axis=1, keepdims=True)
    L = float(np.mean(np.log(E.sum(axis=1)) - Zm[np.arange(B), y]))
    dZ = P.copy()
    dZ[np.arange(B), y] -= 1.0
    dZ /= B
    dW2 = dZ.T @ Hd
    db2 = dZ.sum(axis=0)
    dH = dZ @ np.asarray(W2, np.float64)
    dA = dH * (A > 0)
    dW1 = dA.T @ X
    db1 = dA.sum(axis=0)
    return L, dW1, db1, dW2, db2


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t is the 1-based step count).  Returns new params, m, v."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = beta1 * mm + (1 - beta1) * g
        vv = beta2 * vv + (1 - beta2) * g * g
        mhat = mm / (1 - beta1 ** t)
        vhat = vv / (1 - beta2 ** t)
        out_p.append(p - lr * mhat / (np.sqrt(vhat) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v


def propose(Z, per_quarter: int = 4):
    """Candidate proposals from logits Z (rows x k): for each quarter q of the
    centers (center j belongs to quarter (j mod 16) div 4), its per_quarter
    highest logits in decreasing order, ties to the lower index; -1 where a
    quarter has fewer centers.  Returns an int array rows x (4 per_quarter),
    quarter q in columns [q per_quarter, (q + 1) per_quarter).  Written as a
    plain repeated selection of the largest remaining logit of each quarter.
    """
    Z = np.asarray(Z, np.float64)
    rows, k = Z.shape
    out = np.full((rows, 4 * per_quarter), -1, dtype=np.int64)
    for r in range(rows):
        for q in range(4):
            members = [j for j in range(k) if (j % 16) // 4 == q]
            taken = []
            for slot in range(min(per_quarter, len(members))):
                best = -1
                for j in members:
                    if j in taken:
                        continue
                    if best < 0 or Z[r, j] > Z[r, best]:
                        best = j            # strict '>' keeps the lower index on ties
                taken.append(best)
                out[r, q * per_quarter + slot] = best
    return out


def predict(X, W1, b1, W2, b2):
    """Highest-logit class (lowest index on ties)."""
    _, _, Z = forward(X, W1, b1, W2, b2)
    return np.argmax(Z, axis=1)
