"""The larger workloads at their full sizes, through the C ABI, in the launch
configurations bench.py times:

  * rotated mixture (n = 1,000,000, d = 1000, k = 50): k-means++ and three
    Lloyd iterations in FP32, BF16 and FP8; every precision returns the same
    labels, centers and cost history; sampled rows against the oracle's
    assignment, three clusters' centroids against the oracle's update on
    their rows;
  * streamed (10,000,000 rows of d = 4096 in 153 chunks of 65,536 -> 64):
    sampled projected rows against the oracle's projection within the FP32
    accumulation bound, then the same cross-precision identity and sampled
    labels;
  * 256 uneven weighted instances (sum n = 26.7 M): two batched iterations
    against independent single-instance runs (identical labels, bitwise
    identical centers) and sampled labels of three instances against the
    oracle.

Labels are compared with the oracle outside its 1e-6 relative top-2 margin
band, centroids to 1e-5 relative.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import kmeans as ok
from oracle import project as op

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


def _check_sampled(lab_rows, Xs, C, what):
    lab_o, d1, d2 = ok.assign(Xs, C)
    bad = (lab_rows != lab_o) & ~((d2 - d1) < 1e-6 * d2)
    assert not bad.any(), f"{what}: {int(bad.sum())} sampled rows differ"


def _three_precisions(ctx, X, C0, iters):
    out = {}
    for prec in ("fp32", "bf16", "fp8"):
        C, lab, hist, it = ctx.lloyd(X, C0, iters, prec=prec, labels=True)
        say(f"  {prec}: cost {hist[-1]:.9e}, re-check {ctx.assign_stats()}")
        out[prec] = (C, lab, hist, it)
    C32, l32, h32, _ = out["fp32"]
    for prec in ("bf16", "fp8"):
        C, lab, hist, _ = out[prec]
        assert torch.equal(lab, l32), prec
        assert torch.equal(C, C32), prec
        assert hist == h32, prec
    return out["fp32"]


def test_rotated_mixture_full_size(ctx):
    n, d, k, iters = 1_000_000, 1000, 50, 3
    say("rotated mixture n=1e6 d=1000 k=50")
    X, _ = synth.rotated_mixture_device(n, d, k, seed=0, device="cuda:0")
    C0, _ = ctx.seed(X, k, rng_seed=0)
    C, lab, hist, it = _three_precisions(ctx, X, C0, iters)
    assert it == iters
    assert all(hist[t + 1] <= hist[t] * (1 + 1e-12) for t in range(len(hist) - 1))
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(n, 2000, replace=False))
    ridx = torch.from_numpy(rows).to("cuda:0")
    Ch = C.cpu().numpy()
    _check_sampled(lab[ridx].cpu().numpy(), X[ridx].cpu().numpy(), Ch, "rotated labels")
    # the update of C_T on the final labels, three clusters against the oracle
    Cn, W, _ = ctx.update(X, lab, C)
    labh = lab.cpu().numpy()
    for j in (0, k // 2, k - 1):
        members = np.nonzero(labh == j)[0]
        Xj = X[torch.from_numpy(members).to("cuda:0")].cpu().numpy()
        ref = Xj.astype(np.float64).mean(axis=0)
        got = Cn[j].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(got - ref) <= 1e-5 * max(np.linalg.norm(ref), 1e-3), j
        assert float(W[j].item()) == float(len(members))
    del X
    torch.cuda.empty_cache()


def test_streamed_full_size(ctx):
    d_in, r, k, rows, n, iters = 4096, 64, 100, 65536, 10_000_000, 3
    nchunks = (n + rows - 1) // rows
    say(f"streamed {nchunks} chunks of {rows} x {d_in} -> {r}")
    dev = "cuda:0"
    F = torch.from_numpy(synth.lowrank_factors(d_in, r, seed=0)).to(dev)
    sample = torch.cat([synth.lowrank_chunk_device(rows, F, seed=0, chunk=1_000_000 + c,
                                                   device=dev) for c in range(2)])[:100_000]
    Vd, _ = ctx.range_basis(sample.contiguous(), r, oversample=16, power_iters=1, seed=0)
    V = Vd.cpu().numpy()
    del sample
    Y = torch.empty((nchunks * rows, r), dtype=torch.float32, device=dev)
    rng = np.random.default_rng(3)
    worst = 0.0
    for c in range(nchunks):
        Xc = synth.lowrank_chunk_device(rows, F, seed=0, chunk=c, device=dev)
        ctx.project(Xc, Vd, out=Y[c * rows:(c + 1) * rows])
        if c % 16 == 0:
            pick = np.sort(rng.choice(rows, 16, replace=False))
            Xs = Xc[torch.from_numpy(pick).to(dev)].cpu().numpy()
            Ys = Y[c * rows + torch.from_numpy(pick).to(dev)].cpu().numpy().astype(np.float64)
            Yo = op.project(Xs, V)
            bound = (d_in + 2) * 2.0 ** -23 * (np.abs(Xs.astype(np.float64)) @ np.abs(V.astype(np.float64)))
            assert np.all(np.abs(Ys - Yo) <= bound + 1e-30), c
            worst = max(worst, float(np.max(np.abs(Ys - Yo) / (bound + 1e-30))))
    say(f"  projection: worst sampled error {worst:.3f} of its bound")
    del Xc
    C0, _ = ctx.seed(Y, k, rng_seed=0)
    C, lab, hist, it = _three_precisions(ctx, Y, C0, iters)
    pick = torch.from_numpy(np.sort(rng.choice(Y.shape[0], 2000, replace=False))).to(dev)
    _check_sampled(lab[pick].cpu().numpy(), Y[pick].cpu().numpy(), C.cpu().numpy(),
                   "streamed labels")
    del Y
    torch.cuda.empty_cache()


def test_batched_full_size(ctx):
    iters = 2
    descs = synth.uneven_instances(256, seed=0)
    say(f"batched 256 instances, sum n = {sum(d['n'] for d in descs)}")
    probs = []
    for desc in descs:
        X, w = synth.instance_device(desc, device="cuda:0")
        C0 = X[:desc["k"]].contiguous()           # first k rows as the start
        probs.append({"X": X, "C": C0, "w": w})
    res = ctx.lloyd_batched(probs, iters)
    for i, p in enumerate(probs):
        C, lab, hist, _ = ctx.lloyd(p["X"], p["C"], iters, w=p["w"], prec="bf16")
        Cb, labb, histb = res[i]
        assert torch.equal(lab, labb), i
        assert torch.equal(C, Cb), i
        np.testing.assert_allclose(histb, hist, rtol=1e-12)
    rng = np.random.default_rng(5)
    for i in (0, 127, 255):
        Cb, labb, _ = res[i]
        X = probs[i]["X"]
        pick = torch.from_numpy(np.sort(rng.choice(X.shape[0], min(1000, X.shape[0]),
                                                   replace=False))).to("cuda:0")
        _check_sampled(labb[pick].cpu().numpy(), X[pick].cpu().numpy(), Cb.cpu().numpy(),
                       f"instance {i}")
    del probs, res
    torch.cuda.empty_cache()


def test_headline_fp8_step_against_oracle(ctx):
    # n = 4,000,000, d = 512, k = 1000 (means N(0, 4I), sigma in [0.5, 1.5]),
    # k-means++ seed 0, the FP8 path bench.py times: one Lloyd iteration.
    # The oracle recomputes, on the host in FP64, the clustering features of
    # the GPU's partitions (Sec. 2.1): all 1000 centroids of C_1 against the
    # oracle's update of the labels against C_0 (1e-5 relative), cost(C_0) and
    # cost(C_1) against the clustering-feature identity on the same labels
    # (1e-6 relative); labels of 20,000 sampled rows against the oracle's
    # assignment outside the 1e-6 top-2 band.
    say("headline step n=4e6 d=512 k=1000 (fp8) against the oracle")
    n, d, k = 4_000_000, 512, 1000
    Xg, _, _ = synth.router_mixture_device(n, d, k, seed=0)
    C0, _ = ctx.seed(Xg, k, rng_seed=0)
    lab0, _, _, _ = ctx.assign(Xg, C0, prec="fp8", want_d=False)
    C1, lab1, hist, it = ctx.lloyd(Xg, C0, 1, prec="fp8", labels=True)
    assert it == 1
    X = Xg.cpu().numpy()
    L0, L1 = lab0.cpu().numpy(), lab1.cpu().numpy()
    C0h = C0.cpu().numpy().astype(np.float64)
    C1h = C1.cpu().numpy().astype(np.float64)
    del Xg
    torch.cuda.empty_cache()
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(n, 20000, replace=False))
    _check_sampled(L0[rows], X[rows], C0h, "labels against C_0")
    _check_sampled(L1[rows], X[rows], C1h, "labels against C_1")
    say("  oracle update of the GPU's labels")
    Cn, W, S, Q = ok.update(X, None, L0, C0h)
    nonempty = W > 0
    say(f"  {int(nonempty.sum())} non-empty clusters")
    for j in range(k):
        scale = max(np.linalg.norm(Cn[j]), 1e-3)
        assert np.linalg.norm(C1h[j] - Cn[j]) <= 1e-5 * scale, j
    cost0 = ok.cost_from_features(W, S, Q, C0h)
    assert abs(hist[0] - cost0) <= 1e-6 * cost0, (hist[0], cost0)
    W1, S1, Q1 = ok.clustering_features(X, None, L1, k)
    cost1 = ok.cost_from_features(W1, S1, Q1, C1h)
    assert abs(hist[1] - cost1) <= 1e-6 * cost1, (hist[1], cost1)
    say(f"  cost(C_0) {hist[0]:.9e} vs {cost0:.9e}; cost(C_1) {hist[1]:.9e} vs {cost1:.9e}")


@pytest.mark.parametrize("k,n", [(10, 10000), (50, 10000)])
def test_lowerbound_table2_optimum_on_gpu(ctx, k, n):
    # The paper's LowerBound family (Sec. 3) at the sizes of Table 2 (d =
    # k + n = 10010 and 10050: rows wider than the GEMM, the exact
    # every-center path).  Lloyd started at the clusters' centroids is a fixed
    # point whose cost is the optimum (delta^2 / 2)(n - k) that Table 2 prints
    # (4.995e7 and 4.975e7, tests/golden/lowerbound_table2.txt); the GPU's
    # k-means++ draws the oracle's rows.
    import os
    say(f"LowerBound k={k} n={n} d={k + n}")
    gold = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "lowerbound_table2.txt")):
        if line.strip() and not line.startswith("#"):
            kk, nn, dd, printed = line.split()
            gold[(int(kk), int(nn))] = (int(dd), float(printed))
    d, printed = gold[(k, n)]
    X, lab = synth.lowerbound(k, n)
    assert X.shape[1] == d
    X32 = X.astype(np.float32)
    Xd = torch.from_numpy(X32).to("cuda:0")
    C0 = np.stack([X32[lab == j].astype(np.float64).mean(axis=0) for j in range(k)])
    for prec in ("fp32", "bf16", "fp8"):
        C, labg, hist, it = ctx.lloyd(Xd, torch.from_numpy(C0.astype(np.float32)).to("cuda:0"),
                                      3, prec=prec)
        say(f"  {prec}: cost {hist}")
        assert it == 3
        assert np.array_equal(labg.cpu().numpy(), lab)
        for c in hist:
            assert abs(c - printed) <= 1e-3 * printed      # printed to 4 digits
            assert abs(c - 0.5 * 100.0 ** 2 * (n - k)) <= 1e-6 * printed
    # k-means++ on the GPU draws the oracle's rows (FP64 D2 on both sides)
    Cg, idx = ctx.seed(Xd, k, rng_seed=7)
    _, idx_o, _ = ok.seed(X32, None, k, 7)
    assert idx.cpu().numpy().tolist() == idx_o.tolist()
    cost_g = ctx.cost(Xd, Cg)
    assert abs(cost_g - ok.cost(X32, None, Cg.cpu().numpy())) <= 1e-6 * cost_g
