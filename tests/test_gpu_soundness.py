"""Soundness of the assignment's error flag, as a property over many rows.

A row the first GEMM pass does not flag keeps the GEMM's label without any
re-check, so a flag that misses a row whose top-2 margin lies inside the
GEMM's true error shows up as a label that differs from the FP64 oracle's.
Here 2,000,000 rows per precision (FP32, BF16, FP8) are assigned and every
label is compared with the oracle's argmin (Sec. 1), outside the 1e-6
relative top-2 band.  Half of the rows are built as near ties: the midpoint
of two centers moved along their difference by a relative 1e-9 .. 1e-1 and
orthogonally by up to three center spreads, so the margins span the rounding
error of every precision; the rest are mixture rows.  The second data set
adds a common offset of norm 40 to points and centers, which makes the
GEMM's cancellation (||x||^2 - 2 x.c + ||c||^2 form) and the quantization
error larger relative to the margins.
"""
import sys

import numpy as np
import pytest

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


def near_tie_rows(C, n, rng, spread):
    k, d = C.shape
    a = rng.integers(0, k, n)
    b = (a + rng.integers(1, k, n)) % k
    ca, cb = C[a].astype(np.float64), C[b].astype(np.float64)
    diff = cb - ca
    dn = np.linalg.norm(diff, axis=1, keepdims=True)
    u = diff / dn
    z = rng.normal(size=(n, d))
    z -= np.sum(z * u, axis=1, keepdims=True) * u            # orthogonal to c_b - c_a
    z *= (rng.uniform(0, 3 * spread, (n, 1)) / np.maximum(np.linalg.norm(z, axis=1,
                                                                          keepdims=True), 1e-30))
    delta = np.sign(rng.uniform(-1, 1, (n, 1))) * 10.0 ** rng.uniform(-9, -1, (n, 1)) * dn
    return (0.5 * (ca + cb) + z + delta * u).astype(np.float32)


def dataset(seed, n, d, k, offset):
    rng = np.random.default_rng(seed)
    C = rng.normal(0, 2.0, (k, d))
    m = rng.normal(size=d)
    m *= offset / np.linalg.norm(m)
    C = (C + m).astype(np.float32)
    half = n // 2
    X1 = near_tie_rows(C, half, rng, 2.0)
    comp = rng.integers(0, k, n - half)
    X2 = (C[comp] + rng.normal(0, rng.uniform(0.3, 3.0, (n - half, 1)), (n - half, d))
          ).astype(np.float32)
    X = np.concatenate([X1, X2])
    X = X[rng.permutation(n)]
    return np.ascontiguousarray(X), C


@pytest.mark.parametrize("offset", [0.0, 40.0])
def test_unflagged_rows_are_exact(ctx, offset):
    n, d, k = 2_000_000, 64, 32
    say(f"soundness n={n} d={d} k={k} offset={offset}")
    X, C = dataset(17 + int(offset), n, d, k, offset)
    lab_o, d1, d2 = ok.assign(X, C)
    exempt = (d2 - d1) < 1e-6 * d2
    say(f"  rows inside the 1e-6 band: {int(exempt.sum())}")
    Xd = torch.from_numpy(X).cuda()
    Cd = torch.from_numpy(C).cuda()
    for prec in ("fp32", "bf16", "fp8"):
        lab, _, _, nf = ctx.assign(Xd, Cd, prec=prec, want_d=False)
        g = lab.cpu().numpy()
        bad = (g != lab_o) & ~exempt
        say(f"  {prec}: flagged by the first pass {nf}, re-check lists {ctx.assign_stats()}, "
            f"labels differing outside the band {int(bad.sum())}")
        assert not bad.any(), f"{prec}: {int(bad.sum())} rows differ from FP64"
