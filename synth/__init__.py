"""Seeded synthetic input generators shared by the tests, the bench and the oracle
checks.  This module holds none of the k-means arithmetic: it only draws points
and weights.  Every array is float32 (the format the library consumes) unless
stated otherwise.

Families:
  * ``isotropic_mixture``  -- K spherical Gaussians, means uniform in a cube
    (the small plain-method workload: n=10,000, d=64, K=10, means in [-10,10]^d).
  * ``rotated_mixture``    -- Gaussians with random-rotation covariances whose
    eigenvalues are log-uniform (n=1e6, d=1000, K=50 workload).
  * ``router_mixture``     -- means N(0, 4I), sigma_c uniform in [0.5, 1.5]
    (n=4e6, d=512, K=1000 workload); ``router_mixture_device`` draws the same
    family on a GPU with torch so 8 GB never crosses PCIe.
  * ``lowerbound``         -- the k-means++ worst-case family of Sec. 3
    (simplex of simplices).
  * ``structured_with_noise`` and ``random_cube`` -- the other two generated
    families of Sec. 3.
  * ``uneven_instances``   -- many independent weighted problems with
    log-normal(0,1) weights (coreset-like inputs).

Mixture membership: row i belongs to component i mod K (equal counts).
"""
from __future__ import annotations

import numpy as np


def _rng(seed):
    return np.random.default_rng(np.random.SeedSequence(seed))


def isotropic_mixture(n: int, d: int, K: int, seed: int = 0, lo: float = -10.0,
                      hi: float = 10.0, sigma: float = 1.0):
    """Rows mu_{i mod K} + sigma * N(0, I); means uniform in [lo, hi]^d."""
    rng = _rng(seed)
    means = rng.uniform(lo, hi, size=(K, d))
    comp = np.arange(n) % K
    X = means[comp] + sigma * rng.standard_normal((n, d))
    return X.astype(np.float32), means


def haar_rotation(d: int, rng) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the
    signs of R's diagonal folded into Q (Mezzadri 2007)."""
    A = rng.standard_normal((d, d))
    Q, R = np.linalg.qr(A)
    return Q * np.sign(np.diag(R))[None, :]


def rotated_mixture(n: int, d: int, K: int, seed: int = 0, lo: float = -5.0,
                    hi: float = 5.0, log10_eig=(-2.0, 0.0), chunk: int = 65536):
    """Rows mu_c + R_c diag(sqrt(lambda_c)) z, c = i mod K, with R_c Haar,
    lambda_{c,j} = 10^U[log10_eig], means uniform in [lo, hi]^d."""
    rng = _rng(seed)
    means = rng.uniform(lo, hi, size=(K, d))
    factors = []
    for _ in range(K):
        R = haar_rotation(d, rng)
        lam = 10.0 ** rng.uniform(log10_eig[0], log10_eig[1], size=d)
        factors.append((R * np.sqrt(lam)[None, :]).astype(np.float32))
    X = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        comp = np.arange(s, e) % K
        Z = rng.standard_normal((e - s, d)).astype(np.float32)
        for c in range(K):
            rows = np.nonzero(comp == c)[0]
            if rows.size:
                X[s + rows] = means[c].astype(np.float32) + Z[rows] @ factors[c].T
    return X, means


def rotated_mixture_device(n: int, d: int, K: int, seed: int = 0, lo: float = -5.0,
                           hi: float = 5.0, log10_eig=(-2.0, 0.0), device="cuda"):
    """Same family as ``rotated_mixture`` (means, rotations and eigenvalues
    from the host RNG in the same order) with the N(0, I) draws made on the
    device by torch's seeded Philox generator.  Returns (X device float32,
    means)."""
    import torch
    rng = _rng(seed)
    means = rng.uniform(lo, hi, size=(K, d))
    X = torch.empty((n, d), dtype=torch.float32, device=device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) + 0x7A7E)
    for c in range(K):
        R = haar_rotation(d, rng)
        lam = 10.0 ** rng.uniform(log10_eig[0], log10_eig[1], size=d)
        Ft = torch.from_numpy((R * np.sqrt(lam)[None, :]).T.astype(np.float32)).to(device)
        m = (n - c + K - 1) // K if c < n else 0
        if m == 0:
            continue
        Z = torch.randn(m, d, generator=g, device=device)
        X[c::K] = torch.from_numpy(means[c].astype(np.float32)).to(device) + Z @ Ft
    return X, means


def router_mixture(n: int, d: int, K: int, seed: int = 0, mean_std: float = 2.0,
                   sig_lo: float = 0.5, sig_hi: float = 1.5):
    """Rows mu_c + sigma_c N(0, I), c = i mod K; mu_c ~ N(0, mean_std^2 I),
    sigma_c ~ U[sig_lo, sig_hi]."""
    rng = _rng(seed)
    means = rng.normal(0.0, mean_std, size=(K, d))
    sig = rng.uniform(sig_lo, sig_hi, size=K)
    comp = np.arange(n) % K
    X = means[comp] + sig[comp, None] * rng.standard_normal((n, d))
    return X.astype(np.float32), means, sig


def router_mixture_device(n: int, d: int, K: int, seed: int = 0, device="cuda",
                          mean_std: float = 2.0, sig_lo: float = 0.5,
                          sig_hi: float = 1.5, chunk: int = 1 << 18):
    """Same family as ``router_mixture`` but the N(0, I) noise is drawn on the
    device by torch's seeded Philox generator (means and sigmas come from the
    host RNG, so a host copy of any row can be rebuilt from them only with the
    device noise).  Returns (X device float32, means, sig)."""
    import torch
    rng = _rng(seed)
    means = rng.normal(0.0, mean_std, size=(K, d))
    sig = rng.uniform(sig_lo, sig_hi, size=K)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) + 0x5EED)
    mu_t = torch.as_tensor(means, dtype=torch.float32, device=device)
    sg_t = torch.as_tensor(sig, dtype=torch.float32, device=device)
    X = torch.empty((n, d), dtype=torch.float32, device=device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        comp = torch.arange(s, e, device=device) % K
        z = torch.randn((e - s, d), generator=g, device=device, dtype=torch.float32)
        X[s:e] = mu_t[comp] + sg_t[comp, None] * z
    return X, means, sig


def lowerbound(k: int, n: int, delta: float = 100.0, Delta: float = 1000.0):
    """The simplex-of-simplices family used as the k-means++ lower-bound
    instance (Sec. 3, LowerBound): a k-vertex simplex in the first k coordinates
    and, at each vertex, an (n/k)-vertex simplex on its own block of the next n
    coordinates.  Reading: both simplices have edge lengths Delta and delta,
    i.e. vertex v of a simplex of edge a sits at (a / sqrt 2) e_v.
    Returns (X float64 n x (k+n), labels of the generating vertex)."""
    assert n % k == 0
    m = n // k
    X = np.zeros((n, k + n))
    lab = np.repeat(np.arange(k), m)
    big = Delta / np.sqrt(2.0)
    small = delta / np.sqrt(2.0)
    for i in range(n):
        X[i, lab[i]] = big
        X[i, k + i] = small
    return X, lab


def structured_with_noise(ell: int, y: int, d: int, x: int, seed: int = 0,
                          Delta: float = 10.0, delta: float = 0.5):
    """StructuredWithNoise (Sec. 3): ell clusters of y points; cluster i picks x
    coordinates at random, draws them uniform in [-Delta, Delta] and the other
    coordinates uniform in [-delta, delta]."""
    rng = _rng(seed)
    X = rng.uniform(-delta, delta, size=(ell * y, d))
    for i in range(ell):
        dims = rng.choice(d, size=x, replace=False)
        X[i * y:(i + 1) * y][:, dims] = rng.uniform(-Delta, Delta, size=(y, x))
    return X.astype(np.float32)


def random_cube(n: int, d: int, seed: int = 0, Delta: float = 10.0):
    """Random family (Sec. 3): points uniform in [-Delta, Delta]^d."""
    return _rng(seed).uniform(-Delta, Delta, size=(n, d)).astype(np.float32)


def lognormal_weights(n: int, seed: int = 0):
    """Coreset-like weights w ~ LogNormal(0, 1), float32."""
    return _rng(seed).lognormal(0.0, 1.0, size=n).astype(np.float32)


def uneven_instances(count: int = 256, seed: int = 0, n_range=(1000, 200000),
                     d_choices=(16, 32, 64, 128, 256, 512), k_range=(5, 200),
                     scale: float = 1.0):
    """Descriptors of independent weighted problems: n_i ~ U{n_range} (times
    ``scale``), d_i ~ U(d_choices), k_i ~ U{k_range}.  Points come from
    ``instance(desc)``."""
    rng = _rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1) * scale)
        n = max(n, 1)
        d = int(rng.choice(d_choices))
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        k = min(k, n)
        out.append({"n": n, "d": d, "k": k, "seed": (seed, i)})
    return out


def instance(desc):
    """Points (k_i Gaussian components, means U[-10,10]^d, sigma 1) and
    log-normal(0,1) weights for one descriptor of ``uneven_instances``."""
    rng = _rng(list(desc["seed"]))
    n, d, k = desc["n"], desc["d"], desc["k"]
    means = rng.uniform(-10, 10, size=(k, d))
    comp = np.arange(n) % k
    X = (means[comp] + rng.standard_normal((n, d))).astype(np.float32)
    w = rng.lognormal(0.0, 1.0, size=n).astype(np.float32)
    return X, w


def lowrank_factors(d: int, r: int = 64, seed: int = 0):
    """Gaussian factor matrix F (r x d, float32) of the streamed high-dimensional
    workload: rows are z F + noise with z ~ N(0, I_r)."""
    return _rng([seed, 0x10F]).standard_normal((r, d)).astype(np.float32)


def lowrank_chunk(rows: int, F, seed: int = 0, chunk: int = 0, noise: float = 0.05):
    """Chunk ``chunk`` of the streamed workload: rows z F + noise N(0, noise^2 I),
    z ~ N(0, I_r) (float32)."""
    rng = _rng([seed, 0xC4, chunk])
    Z = rng.standard_normal((rows, F.shape[0])).astype(np.float32)
    return (Z @ F + noise * rng.standard_normal((rows, F.shape[1])).astype(np.float32)
            ).astype(np.float32)


def lowrank_chunk_device(rows: int, F_dev, seed: int = 0, chunk: int = 0, noise: float = 0.05,
                         device="cuda"):
    """Same family as ``lowrank_chunk``, drawn on the device by torch's seeded
    Philox generator (a different stream than the host version)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed((int(seed) * 1_000_003 + int(chunk)) & 0x7FFFFFFFFFFFFFFF)
    Z = torch.randn(rows, F_dev.shape[0], generator=g, device=device)
    X = Z @ F_dev
    X.add_(torch.randn(rows, F_dev.shape[1], generator=g, device=device), alpha=noise)
    return X


def instance_device(desc, device="cuda"):
    """Same family as ``instance`` with the noise and the weights drawn on the
    device by torch's seeded Philox generator (means from the host RNG)."""
    import torch
    rng = _rng(list(desc["seed"]))
    n, d, k = desc["n"], desc["d"], desc["k"]
    means = torch.from_numpy(rng.uniform(-10, 10, size=(k, d)).astype(np.float32)).to(device)
    g = torch.Generator(device=device)
    g.manual_seed(int(rng.integers(0, 2 ** 62)))
    comp = torch.arange(n, device=device) % k
    X = means[comp] + torch.randn(n, d, generator=g, device=device)
    w = torch.exp(torch.randn(n, generator=g, device=device))
    return X.contiguous(), w.contiguous()
