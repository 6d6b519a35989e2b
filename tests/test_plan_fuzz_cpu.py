"""The host-only sizing calls (wt_plan, wt_batch_plan) over random and extreme
arguments: sizes and alphabets up to and past 2^32, every kind and arity,
invalid symbol widths and tunings.  Each call returns OK or an argument /
limit code (no crash, no other code), and an accepted plan is consistent:
1..32 levels, no level longer than n, an image at least as large as its
header and level records, figures that fit the device."""
import random

import numpy as np
import pytest

from paper_1610_03524_amd import binding as B

NS = [0, 1, 2, 63, 64, 65, 511, 512, 513, 8191, 8192, 8193, (1 << 20) + 1, 1 << 28, (1 << 31) + 7,
      (1 << 32) - 8193, (1 << 32) - 8192, (1 << 32) - 1, 1 << 32]
SIGMAS = [0, 1, 2, 3, 4, 5, 255, 256, 257, 4096, 65535, 65536, 65537, (1 << 20) + 1, 1 << 24, (1 << 31) + 1,
          (1 << 32) - 1]
REFUSALS = (B.WT_EINVAL, B.WT_EUNSUP, B.WT_ENOSPC, B.WT_ERANGE)


@pytest.mark.parametrize("seed", range(3))
def test_plan_over_random_and_extreme_arguments(seed):
    rng = random.Random(seed)
    accepted = 0
    for _ in range(600):
        kind = rng.choice([B.KIND_WM, B.KIND_WT, B.KIND_MULTIARY, B.KIND_SHAPED])
        n = rng.choice(NS) if rng.random() < 0.7 else rng.randrange(0, 1 << 32)
        sigma = rng.choice(SIGMAS) if rng.random() < 0.7 else rng.randrange(1, 1 << 32)
        sb = rng.choice([1, 2, 4, 3, 0])
        tune = None
        if rng.random() < 0.5:
            tune = B.make_tuning(tau=rng.choice([0, 1, 2, 5, 8, 9]), tile=rng.choice([0, 1, 16, 1 << 20]),
                                 blocks=rng.choice([0, 1, 2, 1000, 1 << 31]))
        shape = None
        if kind == B.KIND_SHAPED:
            if not 1 <= sigma <= 4096:
                continue
            counts = np.array([rng.randrange(0, 50) for _ in range(sigma)], dtype=np.uint64)
            if not counts.any():
                continue
            codes, lens = B.huffman_codes(counts)
            shape = B.make_shape(codes=codes, code_len=lens, counts=counts)
        elif kind == B.KIND_MULTIARY:
            shape = B.make_shape(arity_log2=rng.choice([0, 1, 2, 3, 4, 5]))
        try:
            info = B.plan(kind, n, sigma, sb, shape=shape, tune=tune)
        except B.WaveletError as e:
            assert e.code in REFUSALS, (kind, n, sigma, sb, e.code)
            continue
        accepted += 1
        nl = info.nlevels
        what = (kind, n, sigma, sb)
        assert 1 <= nl <= 32 and info.n == n, what
        assert all(info.level_n[l] <= n for l in range(nl)), what
        assert 256 + 64 * nl <= info.out_bytes < (1 << 48) and info.workspace_bytes < (1 << 50), what
    assert accepted > 100


@pytest.mark.parametrize("seed", range(2))
def test_batch_plan_over_random_and_extreme_arguments(seed):
    rng = random.Random(100 + seed)
    for _ in range(60):
        descs = []
        for i in range(rng.choice([1, 2, 5, 64, 300])):
            d = B.wt_seq_desc()
            d.S, d.n = 256 * (i + 1), rng.choice([0, 1, 64, 8193, 1 << 20, (1 << 32) - 1, 1 << 32,
                                                  rng.randrange(0, 1 << 22)])
            d.sigma = rng.choice([0, 1, 2, 255, 65537, (1 << 32) - 1, rng.randrange(1, 1 << 20)])
            d.sym_bytes = rng.choice([1, 2, 4, 3])
            d.out, d.out_bytes = 256 * (i + 1) + (1 << 40), rng.choice([0, 1 << 30, 1 << 40])
            d.tau = rng.choice([0, 1, 8, 9])
            descs.append(d)
        try:
            ws = B.batch_plan(B.KIND_WM, descs, B.make_tuning(tile=rng.choice([0, 1, 8, 1 << 20])))
            assert 0 <= ws < (1 << 50)
        except B.WaveletError as e:
            assert e.code in REFUSALS, e.code
