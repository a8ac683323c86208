"""The delta update against the full update and the oracle.

After the first update of a Lloyd run, the clustering features of an
iteration are formed from the previous iteration's by removing and adding the
rows whose label changed (Sec. 2.1: features add under union and subtract
under removal).  Every sum of the update is exact on a fixed-point grid, so:
  * the centers after update t of kmx_lloyd equal, bit for bit, those of the
    standalone kmx_update (every row summed) of the labels and centers of
    iteration t - 1, and the costs are the same bits as kmx_cost's;
  * a cluster that loses all of its members keeps its center;
  * the delta path is the one taken when few rows change (kmx_update_stats).
"""
import sys

import numpy as np
import pytest

import synth
from oracle import kmeans as ok

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_04265_amd import kmx
    return kmx.Context(0)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _chain(ctx, X, C0, T, prec, w=None):
    """For t = 1..T: kmx_lloyd(t) against kmx_update of lloyd(t - 1)'s labels
    and centers; returns the update statistics of every run."""
    stats = []
    Cp, labp, histp, _ = ctx.lloyd(X, C0, 0, w=w, prec=prec)
    for t in range(1, T + 1):
        Ct, labt, histt, it = ctx.lloyd(X, C0, t, w=w, prec=prec)
        assert it == t
        stats.append(ctx.update_stats())
        Cu, _, _ = ctx.update(X, labp, Cp, w=w)
        assert torch.equal(Ct, Cu), f"t={t}: delta and full centers differ"
        assert histt[:t] == histp[:t], (t, histt, histp)
        ct = ctx.cost(X, Ct, w=w, prec=prec)
        assert ct == histt[t], (t, ct, histt[t])
        Cp, labp, histp = Ct, labt, histt
    return stats


@pytest.mark.parametrize("n,d,k,weighted,prec", [
    (20000, 64, 50, False, "bf16"), (7001, 45, 23, True, "fp32"), (4000, 512, 300, False, "fp8"),
    (3000, 1000, 12, True, "bf16"), (5000, 3, 7, False, "fp32"), (2500, 1300, 9, True, "fp32")])
def test_delta_equals_full_update(ctx, n, d, k, weighted, prec):
    say(f"delta vs full n={n} d={d} k={k} w={weighted} {prec}")
    X, _, _ = synth.router_mixture(n, d, max(k // 2, 2), seed=d + k)
    w = synth.lognormal_weights(n, seed=k) if weighted else None
    Xd, wd = _dev(X), (None if w is None else _dev(w))
    C0, _ = ctx.seed(Xd, k, w=wd, rng_seed=5)
    stats = _chain(ctx, Xd, C0, 6, prec, wd)
    say(f"  (changed, delta) of the final updates: {stats}")
    assert any(dl for _, dl in stats), "no update took the delta path"
    ref = ok.lloyd(X, w, C0.cpu().numpy(), 6)
    Cg, lab, hist, _ = ctx.lloyd(Xd, C0, 6, w=wd, prec=prec)
    np.testing.assert_allclose(hist, ref["cost"], rtol=1e-6)
    bad = (lab.cpu().numpy() != ref["labels"]) & ~((ref["d2"] - ref["d1"]) < 1e-6 * ref["d2"])
    assert not bad.any()


def _emptying_case():
    # small 2-D data with many centers: find (by the oracle) a run in which a
    # cluster with members at some iteration has none at the next
    for seed in range(200):
        rng = np.random.default_rng(seed)
        X = rng.normal(size=(400, 2)).astype(np.float32)
        X[:200] += 3.0
        C = np.concatenate([X[rng.choice(400, 30, replace=False)],
                            rng.normal(size=(10, 2)).astype(np.float32) * 4.0])
        Cd = C.astype(np.float64)
        prevW = None
        for t in range(8):
            lab, _, _ = ok.assign(X, Cd)
            W = np.bincount(lab, minlength=len(C))
            if prevW is not None and np.any((prevW > 0) & (W == 0)):
                return X, C, t
            prevW = W
            Cd = ok.update(X, None, lab, Cd)[0].astype(np.float32).astype(np.float64)
    return None


def test_delta_cluster_emptied(ctx):
    case = _emptying_case()
    assert case is not None, "no run with a cluster emptied after the first iteration"
    X, C, t_empty = case
    say(f"cluster emptied at iteration {t_empty}")
    Xd, Cd = _dev(X), _dev(C)
    _chain(ctx, Xd, Cd, t_empty + 2, "fp32")
    ref = ok.lloyd(X, None, C, t_empty + 2)
    Cg, lab, hist, _ = ctx.lloyd(Xd, Cd, t_empty + 2, prec="fp32")
    assert np.array_equal(lab.cpu().numpy(), ref["labels"])
    np.testing.assert_allclose(Cg.cpu().numpy(), ref["C"], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(hist, ref["cost"], rtol=1e-6)


def test_delta_large(ctx):
    # 2,000,000 rows: the delta path over long segments and many chunks
    say("delta vs full n=2e6 d=64 k=100")
    n, d, k = 2_000_000, 64, 100
    Xg, _, _ = synth.router_mixture_device(n, d, k, seed=3)
    w = torch.from_numpy(synth.lognormal_weights(n, seed=3)).to("cuda:0")
    C0, _ = ctx.seed(Xg, k, rng_seed=1)
    for wd in (None, w):
        stats = _chain(ctx, Xg, C0, 4, "bf16", wd)
        say(f"  weighted={wd is not None}: {stats}")
        assert stats[-1][1]
    del Xg
    torch.cuda.empty_cache()
