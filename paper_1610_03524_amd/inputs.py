"""Seeded synthetic inputs with the shapes of the benchmark configurations.

This module only draws symbols; it holds none of the construction's
arithmetic, and both the oracle tests and the GPU library consume it.  The
paper has no datasets (its results are bounds), so every workload is
synthetic; the recipes follow the five configurations:

* ``c1_uniform``    n = 2^20 uint8, sigma = 256, uniform i.i.d.        (seed 1)
* ``c2_zipf``       n = 2^28 uint32, sigma = 2^16, Zipf(s=1.1) over a
                    seed-permuted alphabet                              (seed 2)
* ``c3_geometric``  n = 2^26 uint16, sigma = 4096, geometric(p=0.01)
                    truncated at 4095                                   (seed 3)
* ``c4_batch``      8192 uint32 sequences, n log-uniform in [2^10, 2^22],
                    sigma log-uniform in [4, 2^20], uniform symbols     (seed 4)
* ``c5_requests``   Poisson build arrivals from the c4 mix plus query
                    batches                                             (seed 5)
"""
from __future__ import annotations

import numpy as np

ZIPF_CHUNK = 1 << 24


def c1_uniform(n: int = 1 << 20, sigma: int = 256, seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, sigma, n, dtype=np.uint8 if sigma <= 256 else np.uint32)


def zipf_tables(sigma: int = 1 << 16, s: float = 1.1, seed: int = 2):
    """(permutation of the alphabet, cdf of rank k ~ k^-s)"""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(sigma)
    w = np.arange(1, sigma + 1, dtype=np.float64) ** -s
    cdf = np.cumsum(w) / w.sum()
    return rng, perm, cdf


def c2_zipf(n: int = 1 << 28, sigma: int = 1 << 16, s: float = 1.1, seed: int = 2,
            device=None):
    """Zipf symbols as uint32.  Uniforms are drawn in fixed chunks of 2^24
    from one PCG64 stream; rank = searchsorted(cdf, u, 'right') clipped to
    sigma-1; symbol = perm[rank].  With ``device`` the per-chunk lookup runs
    in torch on that device (same float64 comparisons, same result) and a
    device tensor is returned."""
    rng, perm, cdf = zipf_tables(sigma, s, seed)
    if device is None:
        out = np.empty(n, dtype=np.uint32)
        for a in range(0, n, ZIPF_CHUNK):
            b = min(n, a + ZIPF_CHUNK)
            u = rng.random(b - a)
            r = np.minimum(np.searchsorted(cdf, u, side="right"), sigma - 1)
            out[a:b] = perm[r]
        return out
    import torch
    tcdf = torch.from_numpy(cdf).to(device)
    tperm = torch.from_numpy(perm.astype(np.int64)).to(device)
    out = torch.empty(n, dtype=torch.int32, device=device)
    for a in range(0, n, ZIPF_CHUNK):
        b = min(n, a + ZIPF_CHUNK)
        u = torch.from_numpy(rng.random(b - a)).to(device)
        r = torch.clamp(torch.searchsorted(tcdf, u, right=True), max=sigma - 1)
        out[a:b] = tperm[r].to(torch.int32)
    return out


def c3_geometric(n: int = 1 << 26, sigma: int = 4096, p: float = 0.01, seed: int = 3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    k = rng.geometric(p, n) - 1
    return np.minimum(k, sigma - 1).astype(np.uint16)


def c4_sizes(count: int = 8192, seed: int = 4):
    """(n_i, sigma_i, child seed sequences) of the batched configuration."""
    ss = np.random.SeedSequence(seed)
    m = np.random.default_rng(ss)
    n = np.floor(2.0 ** m.uniform(10, 22, count)).astype(np.int64)
    sig = np.clip(np.floor(2.0 ** m.uniform(2, 20, count)), 4, 1 << 20).astype(np.int64)
    children = ss.spawn(count)
    return n, sig, children


def c4_sequence(n: int, sigma: int, child) -> np.ndarray:
    return np.random.default_rng(child).integers(0, sigma, n, dtype=np.uint32)


def c4_batch(count: int = 8192, seed: int = 4, limit: int | None = None):
    """Yield (S_i, sigma_i) for the first ``limit`` (default all) sequences."""
    n, sig, children = c4_sizes(count, seed)
    k = count if limit is None else min(limit, count)
    for i in range(k):
        yield c4_sequence(int(n[i]), int(sig[i]), children[i]), int(sig[i])


def c5_requests(rate: float, horizon_s: float, seed: int = 5, count: int = 8192):
    """Poisson build arrivals at ``rate``/s (sizes from the c4 mix, drawn in
    arrival order) and query-batch arrivals at max(10, rate/10)/s over
    ``horizon_s`` seconds.  Returns (build_times, build_ids, query_times)."""
    rng = np.random.default_rng(seed)
    nb = rng.poisson(rate * horizon_s)
    bt = np.sort(rng.uniform(0, horizon_s, nb))
    ids = rng.integers(0, count, nb)
    qrate = max(10.0, rate / 10.0)
    nq = rng.poisson(qrate * horizon_s)
    qt = np.sort(rng.uniform(0, horizon_s, nq))
    return bt, ids, qt
