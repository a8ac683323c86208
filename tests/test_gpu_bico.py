"""BICO with the first-level search on the device (kmx_bico_*) against the
FP64 oracle (oracle/bico.py), the lift of projected coordinates (kmx_lift),
and piecy / piecy-mr end to end (Sec. 2.2, Sec. 2.3).

BICO's decisions are comparisons of FP64 sums taken in coordinate order on
both sides, and the device's argmin is exact (the host compares in FP64 when
the device's two closest distances are too near), so the summaries must be
identical: the same features in the same order, the same weights and sums.
End to end, piecy and piecy-mr on the paper's LowerBound family must reach
the optimum of the family, (delta^2 / 2)(n - k), which is the value Table 2
prints for BICO at k = 10 and k = 50 (tests/golden/lowerbound_table2.txt).
"""
import os
import sys

import numpy as np
import pytest

import synth
from oracle import bico as ob
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


def _mixture(n, d, seed, sigma):
    rng = np.random.default_rng(seed)
    means = rng.uniform(-5, 5, size=(8, d))
    return (means[rng.integers(0, 8, n)] + sigma * rng.normal(size=(n, d))).astype(np.float32)


@pytest.mark.parametrize("n,d,m,T0,wkind,sigma", [
    (3000, 8, 60, 1e-3, None, 1.0), (2500, 5, 40, 0.5, "int", 0.05), (2000, 37, 100, 1e-2, None, 0.5),
    (1500, 6, 30, 1e-4, "lognormal", 1.0), (1200, 3, 200, 1e-2, "zeros", 0.3)])
def test_bico_matches_oracle(ctx, n, d, m, T0, wkind, sigma):
    from paper_1502_04265_amd import kmx
    say(f"bico n={n} d={d} m={m} T0={T0} w={wkind}")
    X = _mixture(n, d, n + d, sigma)
    rng = np.random.default_rng(d)
    w = None
    if wkind == "int":
        w = rng.integers(1, 6, n).astype(np.float32)
    elif wkind == "lognormal":
        w = synth.lognormal_weights(n, seed=d)
    elif wkind == "zeros":
        w = rng.integers(0, 3, n).astype(np.float32)
    ref = ob.summarize(X, m, T0, None if w is None else w.astype(np.float64))
    b = kmx.Bico(ctx, d, m, T0)
    h = n // 3                      # two insert calls
    b.insert(_dev(X[:h]), None if w is None else _dev(w[:h]))
    b.insert(_dev(X[h:]), None if w is None else _dev(w[h:]))
    st = b.stats()
    say(f"  {st}; oracle: {ref.count} features, T = {ref.T}, {ref.rebuilds} rebuilds")
    assert st["count"] == ref.count and st["rebuilds"] == ref.rebuilds and st["T"] == ref.T
    assert st["gpu_rows"] > 0
    W, S, Q, R, L = b.features()
    Wo, So, Qo, Ro, Lo = ref.features()
    assert np.array_equal(L, Lo)
    assert np.array_equal(R, Ro)
    assert np.array_equal(W, Wo)
    assert np.array_equal(S, So)
    assert np.array_equal(Q, Qo)
    P, wP = b.coreset()
    np.testing.assert_array_equal(P.cpu().numpy(), (So / Wo[:, None]).astype(np.float32))
    np.testing.assert_array_equal(wP.cpu().numpy(), Wo.astype(np.float32))


def test_bico_first_level_outgrows_its_device_buffer(ctx):
    # thousands of first-level features: the device copy of their references
    # is reallocated several times while blocks are queried, and every
    # reallocation must upload all of them again
    from paper_1502_04265_amd import kmx
    n, d, m = 4000, 64, 1500
    say(f"bico n={n} d={d} m={m}, growing first level")
    X = _mixture(n, d, 11, 1.0)
    ref = ob.summarize(X, m, 20.0)
    b = kmx.Bico(ctx, d, m, 20.0)
    b.insert(_dev(X))
    st = b.stats()
    say(f"  {st}")
    W, S, Q, R, L = b.features()
    Wo, So, Qo, Ro, Lo = ref.features()
    assert st["rebuilds"] == ref.rebuilds and st["count"] == ref.count
    assert np.array_equal(W, Wo) and np.array_equal(S, So) and np.array_equal(R, Ro)
    assert np.array_equal(L, Lo)
    assert st["host_scans"] < n // 100


def test_bico_wide_rows(ctx):
    # d > 1024: the device search takes the every-center path
    from paper_1502_04265_amd import kmx
    n, d, m = 700, 1500, 40
    say(f"bico wide n={n} d={d} m={m}")
    X = _mixture(n, d, 5, 0.2)
    ref = ob.summarize(X, m, 1.0)
    b = kmx.Bico(ctx, d, m, 1.0)
    b.insert(_dev(X))
    W, S, Q, R, L = b.features()
    Wo, So, Qo, Ro, Lo = ref.features()
    assert b.stats()["rebuilds"] == ref.rebuilds > 0
    assert np.array_equal(W, Wo) and np.array_equal(S, So) and np.array_equal(R, Ro)


def test_bico_argument_errors(ctx):
    from paper_1502_04265_amd import kmx
    with pytest.raises(kmx.KmxError) as e:
        kmx.Bico(ctx, 4, 10, 0.0)
    assert e.value.status == 1
    with pytest.raises(kmx.KmxError) as e:
        kmx.Bico(ctx, 4, 0, 1.0)
    assert e.value.status == 1
    b = kmx.Bico(ctx, 4, 10, 1.0)
    with pytest.raises(ValueError):
        b.insert(_dev(np.zeros((5, 3), np.float32)))
    w = np.ones(5, np.float32)
    w[3] = -1.0
    with pytest.raises(kmx.KmxError) as e:
        b.insert(_dev(np.zeros((5, 4), np.float32)), _dev(w))
    assert e.value.status == 1


@pytest.mark.parametrize("rows,m,d", [(1000, 16, 300), (777, 64, 1001), (4100, 128, 64)])
def test_lift_matches_oracle(ctx, rows, m, d):
    rng = np.random.default_rng(rows)
    Z = rng.normal(size=(rows, m)).astype(np.float32)
    V = rng.normal(size=(d, m)).astype(np.float32)
    Y = ctx.lift(_dev(Z), _dev(V)).cpu().numpy().astype(np.float64)
    ref = Z.astype(np.float64) @ V.astype(np.float64).T
    bound = (m + 2) * 2.0 ** -23 * (np.abs(Z.astype(np.float64)) @ np.abs(V.astype(np.float64)).T)
    assert np.all(np.abs(Y - ref) <= bound)


def _lowerbound_optimum(k, n):
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "lowerbound_table2.txt")):
        f = line.split("#")[0].split()
        if len(f) == 4 and int(f[0]) == k and int(f[1]) == n:
            return float(f[3])
    raise KeyError((k, n))


@pytest.mark.parametrize("k,mr", [(10, False), (10, True), (50, True)])
def test_piecy_lowerbound_reaches_table2(ctx, k, mr):
    # Sec. 3 LowerBound at the sizes of Table 2 (n = 10,000, d = n + k), pieces
    # of 1,000 rows projected to max(16, k) dimensions (at least k, Sec. 2.2
    # "Parameters": a summary mixing many clusters must keep them apart); the
    # centers from the summary must give the family's optimum on the full data
    from paper_1502_04265_amd import piecy
    n = 10_000
    printed = _lowerbound_optimum(k, n)
    X, _ = synth.lowerbound(k, n)
    Xd = _dev(X.astype(np.float32))
    pieces = (Xd[s:s + 1000] for s in range(0, n, 1000))
    say(f"piecy{'-mr' if mr else ''} LowerBound k={k} n={n} d={n + k}")
    svd = max(16, k)
    if mr:
        r = piecy.piecy_mr(ctx, pieces, k, svd, np_=4, lloyd_iters=10, seed=1)
    else:
        r = piecy.piecy(ctx, pieces, k, svd, lloyd_iters=10, seed=1)
    cost = ctx.cost(Xd, r["C"])
    say(f"  summary of {r['P'].shape[0]} points, weight {float(r['w'].sum()):.1f}, "
        f"cost {cost:.6e} (printed {printed:.4e}); {r['bico']}")
    assert abs(float(r["w"].double().sum().item()) - n) <= 1e-3
    assert abs(cost - printed) <= 1e-6 * printed
    del Xd
    torch.cuda.empty_cache()


def test_piecy_structured_with_noise(ctx):
    # StructuredWithNoise (Sec. 3): the centers from the summary cost at most
    # 5 % more on the full data than Lloyd from k-means++ on the full data
    from paper_1502_04265_amd import piecy
    k = 8
    X = synth.structured_with_noise(k, 2000, 300, 15, seed=2)
    Xd = _dev(X)
    pieces = [Xd[s:s + 4000] for s in range(0, X.shape[0], 4000)]
    for mr in (False, True):
        fn = piecy.piecy_mr if mr else piecy.piecy
        r = fn(ctx, iter(pieces), k, 32, lloyd_iters=20, seed=3, m=400) if not mr else \
            fn(ctx, iter(pieces), k, 32, np_=2, lloyd_iters=20, seed=3, m=400)
        c_summary = ctx.cost(Xd, r["C"])
        C0, _ = ctx.seed(Xd, k, rng_seed=3)
        C, _, hist, _ = ctx.lloyd(Xd, C0, 30, prec="fp32")
        c_full = ctx.cost(Xd, C)
        say(f"  SWN {'piecy-mr' if mr else 'piecy'}: summary {r['P'].shape[0]} points, cost "
            f"{c_summary:.6e} vs full-data Lloyd {c_full:.6e}")
        assert abs(float(r["w"].double().sum().item()) - X.shape[0]) <= 1e-2
        assert c_summary <= 1.05 * c_full
