"""Alphabets of 21 to 32 key bits (sigma up to 2^32 - 1).

The wavelet matrix over such keys runs its first passes with 32-bit keys in
LDS (more than 16 key bits left), then 16- and 8-bit ones; balanced and
multiary trees over more than 20 key bits take their runs from symbol counts
read back to the host.  Every image is compared byte for byte with the
oracle's, and queries over 32 levels with brute force on S (from a stable
argsort of S: no array as long as the alphabet)."""
import numpy as np
import pytest

from gpu_util import assert_same, gpu_image, oracle_image, to_device
from paper_1610_03524_amd import binding as B

pytestmark = pytest.mark.gpu

U32MAX = 0xFFFFFFFF
U64MAX = 0xFFFFFFFFFFFFFFFF
WIDE = [(1 << 20) + 1, (1 << 24) + 3, (1 << 31) + 1, (1 << 32) - 1]


def wide_patterns(n, sigma, rng):
    yield "uniform", rng.integers(0, sigma, n, dtype=np.uint64).astype(np.uint32)
    if n > 1:
        yield "equal", np.full(n, sigma - 1, dtype=np.uint32)
        yield "sorted", np.sort(rng.integers(0, sigma, n, dtype=np.uint64)).astype(np.uint32)
        rare = np.zeros(n, dtype=np.uint32)
        rare[n // 2] = sigma - 1
        yield "one_rare", rare
        # a few symbols spread over the key space: almost every run is empty
        few = rng.integers(0, sigma, 7, dtype=np.uint64)
        yield "few_symbols", few[rng.integers(0, 7, n)].astype(np.uint32)


@pytest.mark.parametrize("sigma", WIDE)
def test_matrix_over_wide_alphabets(sigma):
    rng = np.random.default_rng(sigma % 1000003)
    for n in (0, 1, 4097, 70001):
        for name, S in wide_patterns(n, sigma, rng):
            o = oracle_image(B.KIND_WM, S, sigma)
            # automatic passes (8 key bits each) and passes of 5 key bits
            for tune in (None, B.make_tuning(tau=5)):
                assert_same(gpu_image(B.KIND_WM, S, sigma, tune=tune), o,
                            f"sigma={sigma} n={n} {name} tau={'auto' if tune is None else 5}")


@pytest.mark.parametrize("kind,D", [(B.KIND_WT, 0), (B.KIND_MULTIARY, 2), (B.KIND_MULTIARY, 4)])
@pytest.mark.parametrize("sigma", [(1 << 20) + 1, (1 << 24) + 3])
def test_trees_over_wide_alphabets(kind, D, sigma):
    rng = np.random.default_rng(sigma % 1000003 + 7 * kind + D)
    for n in (1, 4097, 70001):
        for name, S in wide_patterns(n, sigma, rng):
            assert_same(gpu_image(kind, S, sigma, D=D), oracle_image(kind, S, sigma, D=D),
                        f"kind={kind} D={D} sigma={sigma} n={n} {name}")


def brute_queries(S, sigma, pos, c, i, k):
    n = S.size
    order = np.argsort(S, kind="stable")   # positions of every symbol, in order
    so = S[order]
    acc = np.where(pos < n, S[np.minimum(pos, n - 1)].astype(np.uint64), np.uint64(U32MAX))
    rk = np.zeros(c.size, dtype=np.uint64)
    sl = np.zeros(c.size, dtype=np.uint64)
    for q in range(c.size):
        cc = int(c[q])
        lo, hi = np.searchsorted(so, cc, side="left"), np.searchsorted(so, cc, side="right")
        at = order[lo:hi]
        if i[q] >= n:
            rk[q] = U64MAX
        else:
            rk[q] = 0 if cc >= sigma else np.searchsorted(at, i[q], side="right")
        kk = int(k[q])
        sl[q] = at[kk - 1] if (cc < sigma and 1 <= kk <= at.size) else U64MAX
    return acc, rk, sl


@pytest.mark.parametrize("kind,D,sigma", [(B.KIND_WM, 0, (1 << 32) - 1), (B.KIND_WM, 0, (1 << 31) + 1),
                                          (B.KIND_WT, 0, (1 << 24) + 3), (B.KIND_MULTIARY, 4, (1 << 24) + 3)])
def test_queries_over_wide_alphabets(kind, D, sigma):
    import torch
    rng = np.random.default_rng(D + kind + sigma % 9973)
    for name, S in wide_patterns(70001, sigma, rng):
        n, m = S.size, 2000
        img, _ = B.build(kind, to_device(S), sigma, arity_log2=D)
        present = np.unique(S)
        absent = rng.integers(0, sigma, 16, dtype=np.uint64)
        above = np.array([sigma, U32MAX] if sigma < U32MAX else [U32MAX], dtype=np.uint64)
        pick = rng.random(m)
        c = np.where(pick < 0.8, present[rng.integers(0, present.size, m)],
                     np.where(pick < 0.95, absent[rng.integers(0, absent.size, m)],
                              above[rng.integers(0, above.size, m)])).astype(np.uint64)
        pos = rng.integers(0, n + 3, m).astype(np.uint64)
        i = rng.integers(0, n + 3, m).astype(np.uint64)
        so = np.sort(S)
        cnt = np.searchsorted(so, c, side="right") - np.searchsorted(so, c, side="left")
        k = (rng.random(m) * (cnt + 3)).astype(np.uint64)
        c32 = c.astype(np.uint32)
        ga = B.access(img, torch.from_numpy(pos.view(np.int64)).cuda()).cpu().numpy().view(np.uint32)
        gr = B.rank(img, torch.from_numpy(c32.view(np.int32)).cuda(), torch.from_numpy(i.view(np.int64)).cuda())
        gs = B.select(img, torch.from_numpy(c32.view(np.int32)).cuda(), torch.from_numpy(k.view(np.int64)).cuda())
        ba, br, bs = brute_queries(S, sigma, pos, c32, i, k)
        assert np.array_equal(ga.astype(np.uint64), ba), f"access {name}"
        assert np.array_equal(gr.cpu().numpy().view(np.uint64), br), f"rank {name}"
        assert np.array_equal(gs.cpu().numpy().view(np.uint64), bs), f"select {name}"
