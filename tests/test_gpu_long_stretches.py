"""Stored select answers of long stretches (Sec. 5.1, "Select": Clark's rule
of storing every answer of a long range).  Levels of 2^20 bits and more whose
512-one (or zero) stretches span 2^20 bits or more: every build path writes
the oracle's image byte for byte (pool included), and selects through the
pool equal brute force on S."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same, gpu_image, oracle_image, to_device
from paper_1610_03524_amd import binding as B
from test_gpu_batch import run_batch
from test_oracle_pins import LONG, long_stretch_bits

pytestmark = pytest.mark.gpu


def select_all_long(img_t, S, sym):
    """select of every ordinal of `sym` (1-based k) on the device against
    the positions of `sym` in S"""
    import torch
    pos = np.flatnonzero(S == sym)
    if not pos.size:
        return
    k = np.arange(1, pos.size + 1, dtype=np.int64)
    c = np.full(pos.size, sym, dtype=np.int32)
    got = B.select(img_t, torch.from_numpy(c).cuda(), torch.from_numpy(k).cuda()).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, pos.astype(np.uint64)), f"select of symbol {sym}"


def skewed(n, seed):
    """4 symbols, symbol 0 about 99.95 %: the top level's ones are sparse"""
    rng = np.random.default_rng(seed)
    S = np.zeros(n, dtype=np.uint8)
    rare = rng.choice(n, 1500, replace=False)
    S[rare] = rng.integers(1, 4, rare.size)
    return S


@pytest.mark.parametrize("case", ["ones", "zeros", "random", "edge"])
@pytest.mark.parametrize("kind", [B.KIND_WM, B.KIND_WT])
def test_binary_sequences(case, kind):
    rng = np.random.default_rng(7)
    n = 1000 + 2 * LONG - 1 if case == "edge" else (1 << 21) + 300000
    S = long_stretch_bits(case, n, rng)
    got = gpu_image(kind, S, 2)
    assert_same(got, oracle_image(kind, S, 2), f"{case} kind {kind}")
    import torch
    img_t = torch.from_numpy(got).cuda()
    for sym in (0, 1):
        select_all_long(img_t, S, sym)


@pytest.mark.parametrize("kind,levelwise", [(B.KIND_WM, False), (B.KIND_WT, False), (B.KIND_WM, True),
                                            (B.KIND_WT, True)])
def test_skewed_four_symbols(kind, levelwise):
    """matrix passes (span directories) and level-by-level builds (one
    directory per level) on a sequence whose top level is sparse"""
    import torch
    S = skewed((1 << 21) + 4321, 11)
    tune = B.make_tuning(flags=B.FLAG_LEVELWISE) if levelwise else None
    got = gpu_image(kind, S, 4, tune=tune)
    assert_same(got, oracle_image(kind, S, 4), f"kind {kind} levelwise {levelwise}")
    img_t = torch.from_numpy(got).cuda()
    for sym in range(4):
        select_all_long(img_t, S, sym)


def test_shaped_tree_with_a_sparse_level():
    import torch
    S = skewed((1 << 21) + 99, 12)
    counts = np.bincount(S, minlength=4).astype(np.uint64)
    codes, lens = oracle.huffman(counts)
    got = gpu_image(B.KIND_SHAPED, S, 4, codes=codes, lens=lens)
    assert_same(got, oracle_image(oracle.KIND_SHAPED, S, 4, codes=codes, lens=lens), "shaped")
    img_t = torch.from_numpy(got).cuda()
    for sym in range(4):
        select_all_long(img_t, S, sym)


def test_batch_with_long_stretches():
    """a batch mixing levels with pool slots (n >= 2^20) and without"""
    rng = np.random.default_rng(13)
    seqs = [(skewed((1 << 20) + 17, 14), 4), (rng.integers(0, 300, 5000).astype(np.uint16), 300),
            (long_stretch_bits("ones", (1 << 21) + 300000, rng), 2), (np.zeros(3, dtype=np.uint8), 1),
            (long_stretch_bits("zeros", (1 << 21) + 300000, rng), 2)]
    imgs = run_batch(seqs)
    for k, ((S, sigma), img) in enumerate(zip(seqs, imgs)):
        assert_same(img, oracle_image(B.KIND_WM, S, sigma), f"sequence {k}")
