"""The randomized range finder on the GPU (kmx_range_basis) against the exact
best-fit subspace of the FP64 oracle (Sec. 2.2, "Computation of the SVD";
Sec. 2.3.2 for weighted points).

The basis is unique only as a subspace (sign and rotation freedom inside
degenerate singular values), so the comparisons are:
  * orthonormal columns (V^T V = I within FP32 rounding);
  * principal angles to the oracle's top-r subspace on data with a clear
    spectral gap (largest sine below 1e-3);
  * Eckart-Young: the residual of projecting onto V is within 1e-3 relative
    of the optimal sum of the discarded squared singular values;
  * singular values of the sample against the oracle's;
  * the weighted variant against the oracle's weighted basis, and the
    sqrt(w) reading against the rows replicated w times.
"""
import sys

import numpy as np
import pytest

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


def lowrank(n, d, r, seed, noise):
    # singular values 100 .. 50 (geometric) on a random rank-r subspace, plus
    # Gaussian noise far below the smallest of them
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, r)))
    V, _ = np.linalg.qr(rng.standard_normal((d, r)))
    s = 100.0 * 0.5 ** (np.arange(r) / max(r - 1, 1))
    return ((U * s) @ V.T + noise * rng.standard_normal((n, d))).astype(np.float32)


def max_sine(V1, V2):
    s = np.linalg.svd(V1.T @ V2, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - s.min() ** 2)))


@pytest.mark.parametrize("n,d,r,ov,q", [(20000, 500, 16, 16, 2), (8000, 1000, 64, 16, 1),
                                        (3001, 200, 20, 12, 2), (50000, 130, 32, 0, 3)])
def test_range_basis_matches_best_fit_subspace(ctx, n, d, r, ov, q):
    say(f"range basis n={n} d={d} r={r} oversample={ov} power={q}")
    A = lowrank(n, d, r, seed=n + d, noise=0.01)
    V, sig = ctx.range_basis(torch.from_numpy(A).cuda(), r, oversample=ov, power_iters=q, seed=3)
    V = V.cpu().numpy().astype(np.float64)
    assert V.shape == (d, r)
    np.testing.assert_allclose(V.T @ V, np.eye(r), atol=2e-5)
    Vo = op.best_fit_basis(A, r)
    sn = max_sine(V, Vo)
    s = np.linalg.svd(A.astype(np.float64), compute_uv=False)
    A64 = A.astype(np.float64)
    resid = np.sum((A64 - (A64 @ V) @ V.T) ** 2)
    opt = np.sum(s[r:] ** 2)
    say(f"  max sine {sn:.2e}; residual {resid:.6e} vs optimum {opt:.6e}; "
        f"sigma_1 {sig[0]:.6f} vs {s[0]:.6f}")
    assert sn < 1e-3
    assert resid <= opt * (1 + 1e-3) + 1e-6 * np.sum(s ** 2)
    np.testing.assert_allclose(sig, s[:r], rtol=1e-4)


def test_range_basis_weighted(ctx):
    # weights log-normal (coreset-like) and integer ones: the sqrt(w) reading
    n, d, r = 12000, 300, 16
    say("range basis, weighted")
    A = lowrank(n, d, r, seed=7, noise=0.002)
    rng = np.random.default_rng(8)
    w = np.exp(rng.normal(0, 1, n)).astype(np.float32)
    V, _ = ctx.range_basis(torch.from_numpy(A).cuda(), r, w=torch.from_numpy(w).cuda(),
                           oversample=16, power_iters=2, seed=1)
    V = V.cpu().numpy().astype(np.float64)
    Vo = op.best_fit_basis_weighted(A, w, r)
    assert max_sine(V, Vo) < 1e-3
    # integer weights against the replicated rows
    wi = rng.integers(1, 4, 2000).astype(np.float32)
    B = A[:2000]
    Vi, _ = ctx.range_basis(torch.from_numpy(B).cuda(), r, w=torch.from_numpy(wi).cuda(),
                            oversample=16, power_iters=2, seed=2)
    F = np.repeat(B, wi.astype(int), axis=0)
    assert max_sine(Vi.cpu().numpy().astype(np.float64), op.best_fit_basis(F, r)) < 1e-3
    # zero weights remove rows
    wz = np.ones(n, np.float32)
    wz[n // 2:] = 0.0
    Vz, _ = ctx.range_basis(torch.from_numpy(A).cuda(), r, w=torch.from_numpy(wz).cuda(), seed=4)
    assert max_sine(Vz.cpu().numpy().astype(np.float64), op.best_fit_basis(A[:n // 2], r)) < 1e-3


def test_range_basis_streamed_workload_sample(ctx):
    # the streamed workload's basis: a 100,000-row sample of rank-64 signal in
    # d = 4096 plus N(0, 0.05^2) noise, r = 64; the subspace the GPU finds
    # projects the sample within 1e-3 of the optimum
    import synth
    say("range basis, streamed workload sample")
    F = torch.from_numpy(synth.lowrank_factors(4096, 64, seed=0)).cuda()
    A = torch.cat([synth.lowrank_chunk_device(65536, F, seed=0, chunk=1_000_000 + c,
                                              device="cuda:0") for c in range(2)])[:100000]
    V, sig = ctx.range_basis(A.contiguous(), 64, oversample=16, power_iters=1, seed=0)
    Vd = V.double()
    Ad = A.double()
    resid = float(((Ad - (Ad @ Vd) @ Vd.T) ** 2).sum())
    total = float((Ad ** 2).sum())
    # the noise floor: 100,000 x (4096 - 64) entries of variance 0.05^2
    floor = 100000 * (4096 - 64) * 0.05 ** 2
    say(f"  residual {resid:.6e}, noise floor {floor:.6e}, total {total:.6e}")
    assert resid <= floor * 1.01
    np.testing.assert_allclose((Vd.T @ Vd).cpu().numpy(), np.eye(64), atol=2e-5)


def test_range_basis_argument_checks(ctx):
    from paper_1502_04265_amd import kmx
    A = torch.zeros((100, 50), device="cuda")
    with pytest.raises(kmx.KmxError) as e:
        ctx.range_basis(A, 120)
    assert e.value.status == 4
    with pytest.raises(kmx.KmxError) as e:
        ctx.range_basis(A[:20], 8)                # l = 32 > n = 20
    assert e.value.status == 1
    with pytest.raises(kmx.KmxError) as e:
        ctx.range_basis(A, 8)                     # no direction at all
    assert e.value.status == 1
