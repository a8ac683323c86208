"""Batched Lloyd (many uneven weighted instances, one persistent assignment
launch per iteration, the iteration replayed as a HIP graph) through the C ABI.

  * against independent single-instance runs of the library from the same
    centers: identical labels, bitwise identical centers and per-iteration
    costs within 1e-12 relative (every replay of the captured iteration is
    compared with an eager run);
  * against the FP64 oracle on weighted instances: labels exact outside the
    1e-6 top-2 margin band, centroids 1e-5, cost 1e-6;
  * the autotuner: tuned shapes give the same results, its cache round-trips.
"""
import json
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


def _instances(ctx, count, seed, n_range=(200, 30000), k_range=(2, 200)):
    descs = synth.uneven_instances(count, seed=seed, n_range=n_range, k_range=k_range)
    probs = []
    for i, desc in enumerate(descs):
        X, w = synth.instance(desc)
        Xd, wd = _dev(X), _dev(w)
        C0, _ = ctx.seed(Xd, desc["k"], w=wd, rng_seed=i)
        probs.append({"X": Xd, "C": C0, "w": wd, "host": (X, w)})
    return descs, probs


def test_batched_matches_single_runs(ctx):
    iters = 6
    descs, probs = _instances(ctx, 24, seed=1)
    say("batched: " + ", ".join(f"({d['n']},{d['d']},{d['k']})" for d in descs))
    res = ctx.lloyd_batched(probs, iters)
    for i, p in enumerate(probs):
        C, lab, hist, it = ctx.lloyd(p["X"], p["C"], iters, w=p["w"], prec="bf16")
        Cb, labb, histb = res[i]
        assert torch.equal(lab, labb), i
        assert torch.equal(C, Cb), i
        np.testing.assert_allclose(histb, hist, rtol=1e-12, err_msg=str(i))


def test_batched_reuses_grouped_copies_until_invalidated(ctx):
    # a second call on the same problems reuses the grouped rows, weights and
    # row statistics; after new contents at the same addresses (which the
    # binding notices from the tensors' version counters and reports with
    # kmx_invalidate), the results are those of a fresh context
    from paper_1502_04265_amd import kmx
    iters = 3
    descs, probs = _instances(ctx, 8, seed=5)
    r1 = ctx.lloyd_batched(probs, iters)
    r2 = ctx.lloyd_batched(probs, iters)
    for a, b in zip(r1, r2):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
        np.testing.assert_array_equal(a[2], b[2])
    for p in probs:
        p["X"].mul_(1.5)
        p["w"].add_(0.25)
    r3 = ctx.lloyd_batched(probs, iters)
    r4 = kmx.Context(0).lloyd_batched(probs, iters)
    changed = 0
    for a, b, c in zip(r3, r4, r1):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
        np.testing.assert_array_equal(a[2], b[2])
        changed += int(not torch.equal(a[0], c[0]))
    assert changed == len(probs)


def test_batched_matches_oracle(ctx):
    iters = 4
    descs, probs = _instances(ctx, 6, seed=2, n_range=(300, 3000), k_range=(3, 40))
    res = ctx.lloyd_batched(probs, iters)
    for i, p in enumerate(probs):
        X, w = p["host"]
        C0 = p["C"].cpu().numpy()
        ref = ok.lloyd(X, w, C0, iters)
        Cb, labb, histb = res[i]
        np.testing.assert_allclose(histb, ref["cost"], rtol=1e-6)
        lab_o, d1, d2 = ok.assign(X, ref["C"])
        bad = (labb.cpu().numpy() != lab_o) & ~((d2 - d1) < 1e-6 * d2)
        assert not bad.any()
        G = Cb.cpu().numpy().astype(np.float64)
        for j in range(C0.shape[0]):
            assert np.linalg.norm(G[j] - ref["C"][j]) <= 1e-5 * max(np.linalg.norm(ref["C"][j]), 1e-3)


def test_batched_edge_cases(ctx):
    rng = np.random.default_rng(4)
    probs = []
    # k == n, tiny n, duplicated points, d = 16 and d = 512 in one batch
    for (n, d, k) in [(7, 16, 7), (1, 32, 1), (40, 512, 3), (500, 16, 5), (130, 128, 64)]:
        X = rng.normal(size=(n, d)).astype(np.float32)
        if n >= 40:
            X[n // 2:] = X[: n - n // 2]
        probs.append({"X": _dev(X), "C": _dev(X[:k].copy())})
    res = ctx.lloyd_batched(probs, 3)
    for p, (Cb, labb, histb) in zip(probs, res):
        C, lab, hist, _ = ctx.lloyd(p["X"], p["C"], 3, prec="bf16")
        assert torch.equal(lab, labb) and torch.equal(C, Cb)
        np.testing.assert_allclose(histb, hist, rtol=1e-12)
    res0 = ctx.lloyd_batched(probs, 0)
    for p, (Cb, labb, histb) in zip(probs, res0):
        assert torch.equal(Cb, p["C"]) and len(histb) == 1


def test_batched_autotuner(ctx, tmp_path):
    descs, probs = _instances(ctx, 12, seed=3)
    base = ctx.lloyd_batched(probs, 3)
    cache = str(tmp_path / "tiles.jsonl")
    assert ctx.batched_autotune(probs, cache) is False
    lines = [json.loads(l) for l in open(cache)]
    assert lines and all(len(e["ms"]) == 3 and 0 <= e["variant"] < 3 for e in lines)
    tuned = ctx.lloyd_batched(probs, 3)
    for (C0, l0, h0), (C1, l1, h1) in zip(base, tuned):
        assert torch.equal(C0, C1) and torch.equal(l0, l1)
        np.testing.assert_allclose(h1, h0, rtol=1e-12)
    from paper_1502_04265_amd import kmx
    other = kmx.Context(0)
    assert other.batched_autotune(probs, cache) is True
    for e in lines:
        k_rep = {0: 10, 1: 50, 2: 150}[e["kclass"]]
        assert other.batched_tiles(e["d"], k_rep)[0] == e["tile"]


def test_seed_batched_matches_oracle_and_single(ctx):
    # k-means++ of uneven weighted instances in one batched call: every
    # instance's indices equal the FP64 oracle's (oracle.kmeans.seed with the
    # instance's own seed) and those of kmx_seed on it alone; the centers are
    # exact copies of the chosen rows.  Instances include weights with zeros,
    # no weights, n = k, k = 1, strided rows and d above the batched Lloyd's 512.
    say("seed batched")
    rng = np.random.default_rng(41)
    shapes = [(1500, 16, 12, True), (3000, 40, 30, False), (777, 100, 7, True), (5, 3, 5, False),
              (2100, 8, 1, True), (4200, 64, 25, True), (1200, 700, 4, False), (900, 33, 17, True)]
    probs, host, seeds = [], [], []
    for i, (n, d, k, weighted) in enumerate(shapes):
        X, _ = synth.isotropic_mixture(n, d, max(k, 2), seed=100 + i)
        w = synth.lognormal_weights(n, seed=100 + i) if weighted else None
        if w is not None:
            w[::4] = 0.0
        Xd = _dev(X)
        if i == 5:   # strided rows: a view into a wider buffer
            wide = torch.zeros((n, d + 7), dtype=torch.float32, device="cuda:0")
            wide[:, :d] = Xd
            Xd = wide[:, :d]
        probs.append({"X": Xd, "k": k, "w": None if w is None else _dev(w)})
        host.append((X, w, k))
        seeds.append(int(rng.integers(0, 2 ** 63)))
    out = ctx.seed_batched(probs, seeds)
    for i, ((C, idx), (X, w, k), sd) in enumerate(zip(out, host, seeds)):
        _, idx_o, _ = ok.seed(X, w, k, sd)
        got = idx.cpu().numpy().tolist()
        assert got == idx_o.tolist(), (i, got, idx_o.tolist())
        assert np.array_equal(C.cpu().numpy(), X[idx_o]), i
        Cs, idx_s = ctx.seed(probs[i]["X"], k, w=probs[i]["w"], rng_seed=sd)
        assert idx_s.cpu().numpy().tolist() == got, i
    # a problem asking for more centers than rows of positive weight
    bad = [{"X": probs[0]["X"], "k": 3, "w": torch.zeros(1500, device="cuda:0")}]
    with pytest.raises(RuntimeError):
        ctx.seed_batched(bad, [1])
