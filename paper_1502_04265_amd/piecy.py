"""piecy and piecy-mr (Sec. 2.2, Sec. 2.3): one pass over a stream of pieces,
each reduced to its best-fit subspace on the device, summarized by BICO on
the host (first-level search on the device), then weighted k-means++ and
Lloyd on the summary, on the device.

  piecy     (Sec. 2.2): one BICO instance takes every projected piece.
  piecy-mr  (Sec. 2.3): a Merge-and-Reduce tree of BICO instances; the
            instance of level l takes np inputs, then its summary is reduced
            to the best-fit subspace of its weighted points (Sec. 2.3.2: rows
            scaled by sqrt(w)) and enters the instance of level l + 1; at the
            end the summaries of all levels together are the summary of the
            stream.

A projected piece keeps its d coordinates (A_m = A V V^T: kmx_project gives
the coordinates Z = A V, kmx_lift the rows Z V^T), so that pieces with
different subspaces meet in one BICO instance.  The summary size m defaults
to 200 k (Sec. 2.2, "Parameters").  The starting threshold, which the paper
leaves to BICO, defaults to the smallest squared distance between a row of
the first projected piece and its closest other row among the first
min(m + 1, 16384) rows (found by the assignment step on the device).  The
dimension projected to is svd_dim rounded up to a multiple of 16 (at most
128), the widths the projection GEMM takes.
"""
from __future__ import annotations

import time
from typing import Iterable, Optional

import torch

from . import kmx


def project_piece(ctx: kmx.Context, A: torch.Tensor, svd_dim: int, w=None, seed: int = 0,
                  oversample: int = 16, power_iters: int = 2):
    """Rows of A reduced to the best-fit subspace of dimension svd_dim (of
    the weighted rows when w is given), as d-dimensional rows."""
    A = A.contiguous()
    n, d = A.shape
    r = subspace_dim(svd_dim)
    l = (r + oversample + 15) // 16 * 16
    if l > min(n, d) or r >= d:
        return A                      # too few rows or columns to reduce
    V, _ = ctx.range_basis(A, r, w=w, oversample=oversample, power_iters=power_iters, seed=seed)
    return ctx.lift(ctx.project(A, V), V)


def subspace_dim(svd_dim: int) -> int:
    """The dimension projected to: svd_dim rounded up to a multiple of 16 in
    [16, 128] (the widths the projection GEMM takes)."""
    return min(128, max(16, (int(svd_dim) + 15) // 16 * 16))


def initial_threshold(ctx: kmx.Context, Y: torch.Tensor, m: int) -> float:
    """Smallest positive squared distance between one of the first rows of Y
    and its closest other row among them."""
    s = int(min(Y.shape[0], m + 1, 16384))
    S = Y[:s].contiguous()
    if s < 2:
        return 1.0
    _, _, d2, _ = ctx.assign(S, S, prec="fp32")
    v = d2.cpu().numpy()
    v = v[v > 0]
    return float(v.min()) if v.size else 1.0


class _Clock:
    """Wall seconds per stage (the device is synchronized at each stage end)."""

    def __init__(self, dev):
        self.dev = dev
        self.s = {"reduce_s": 0.0, "bico_s": 0.0, "kmeans_s": 0.0}

    def run(self, key, fn, *a, **kw):
        t = time.perf_counter()
        out = fn(*a, **kw)
        torch.cuda.synchronize(self.dev)
        self.s[key] += time.perf_counter() - t
        return out


def _finish(ctx, clock, P, w, k, lloyd_iters, seed, prec, stats):
    def km():
        C0, _ = ctx.seed(P, k, w=w, rng_seed=seed)
        return ctx.lloyd(P, C0, lloyd_iters, w=w, prec=prec)
    C, lab, hist, it = clock.run("kmeans_s", km)
    r = dict(C=C, P=P, w=w, cost_hist=hist, iters=it)
    r.update(clock.s)
    r.update(stats)
    return r


def piecy(ctx: kmx.Context, pieces: Iterable[torch.Tensor], k: int, svd_dim: int,
          m: Optional[int] = None, T0: Optional[float] = None, lloyd_iters: int = 20,
          seed: int = 0, prec: str = "fp32", progress=None):
    """Sec. 2.2: every projected piece enters one BICO instance.  Returns a
    dict with the centers C, the summary (P, w), the Lloyd cost history on the
    summary, the BICO statistics and the wall seconds of the stages (reduce_s:
    range finder + projection + lift, bico_s: insertion and summary, kmeans_s:
    k-means++ and Lloyd on the summary).  progress(piece, rows, stats), when
    given, is called after each piece."""
    m = 200 * k if m is None else int(m)
    b = None
    clock = None
    rows = 0
    for q, A in enumerate(pieces):
        if clock is None:
            clock = _Clock(A.device)
        Y = clock.run("reduce_s", project_piece, ctx, A, svd_dim, seed=seed + q)
        if b is None:
            b = kmx.Bico(ctx, Y.shape[1], m, T0 if T0 is not None else initial_threshold(ctx, Y, m))
        clock.run("bico_s", b.insert, Y)
        rows += Y.shape[0]
        if progress:
            progress(q, rows, b.stats())
    P, w = clock.run("bico_s", b.coreset)
    st = b.stats()
    st["rows"] = rows
    return _finish(ctx, clock, P, w, k, lloyd_iters, seed, prec, {"bico": [st]})


def piecy_mr(ctx: kmx.Context, pieces: Iterable[torch.Tensor], k: int, svd_dim: int,
             np_: int = 4, m: Optional[int] = None, T0: Optional[float] = None,
             lloyd_iters: int = 20, seed: int = 0, prec: str = "fp32", progress=None):
    """Sec. 2.3: a Merge-and-Reduce tree of BICO instances of degree np_."""
    m = 200 * k if m is None else int(m)
    levels = []        # [Bico, inputs taken]
    T_start = [T0]
    done = []          # statistics of the instances that handed on their summary
    clock = [None]

    def new_bico(d, Y):
        if T_start[0] is None:
            T_start[0] = initial_threshold(ctx, Y, m)
        return kmx.Bico(ctx, d, m, T_start[0])

    def push(level, Y, w, tag):
        if len(levels) <= level:
            levels.append([new_bico(Y.shape[1], Y), 0])
        clock[0].run("bico_s", levels[level][0].insert, Y, w)
        levels[level][1] += 1
        if levels[level][1] == np_:
            b = levels[level][0]
            P, wP = clock[0].run("bico_s", b.coreset)
            st = b.stats()
            st["level"] = level
            done.append(st)
            levels[level] = [new_bico(Y.shape[1], Y), 0]
            # the summary's weighted best-fit subspace (Sec. 2.3.2)
            Y2 = clock[0].run("reduce_s", project_piece, ctx, P, svd_dim, w=wP,
                              seed=seed + 7919 * (level + 1) + tag)
            push(level + 1, Y2.contiguous(), wP.contiguous(), tag)

    for q, A in enumerate(pieces):
        if clock[0] is None:
            clock[0] = _Clock(A.device)
        Y = clock[0].run("reduce_s", project_piece, ctx, A, svd_dim, seed=seed + q)
        push(0, Y, None, q)
        if progress:
            progress(q, None, levels[0][0].stats())
    parts, wparts, live = [], [], []
    for lv, (b, cnt) in enumerate(levels):
        if cnt == 0:
            continue
        P, wP = clock[0].run("bico_s", b.coreset)
        st = b.stats()
        st["level"] = lv
        live.append(st)
        parts.append(P)
        wparts.append(wP)
    P = torch.cat(parts).contiguous()
    w = torch.cat(wparts).contiguous()
    return _finish(ctx, clock[0], P, w, k, lloyd_iters, seed, prec,
                   {"bico": live, "handed_on": done})
