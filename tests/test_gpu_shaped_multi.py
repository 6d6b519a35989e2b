"""Shaped multiary trees: codewords of D-bit digits (Sec. 4.3 carries the
arbitrary shape over to multiary trees).  Every image equals the oracle's
byte for byte and every query equals brute force on S, on both build paths:
matrix passes over padded codewords with digit levels gathered to tree
order (D = 2, 4; the default), and level by level (every D; on request)."""
import numpy as np
import pytest

import dary
import oracle
from gpu_util import assert_same, to_device
from paper_1610_03524_amd import binding as B
from test_gpu_queries import run_queries

pytestmark = pytest.mark.gpu


def build_both(S, sigma, D, lens, codes, levelwise=False):
    import torch
    counts = np.bincount(S.astype(np.int64), minlength=sigma).astype(np.uint64)
    tune = B.make_tuning(flags=B.FLAG_LEVELWISE) if levelwise else None
    img, info = B.build(B.KIND_SHAPED, to_device(S), sigma, arity_log2=D, codes=codes, code_len=lens, counts=counts,
                        tune=tune)
    torch.cuda.synchronize()
    assert B.check(img) == B.WT_OK
    assert info.nlevels == int(lens.max()) and info.arity_log2 == D
    return img, oracle.build_image(oracle.KIND_SHAPED, S, sigma, D, codes=codes, lens=lens)


@pytest.mark.parametrize("levelwise", [False, True])
@pytest.mark.parametrize("D", [2, 3, 4])
@pytest.mark.parametrize("dt,sigma", [(np.uint8, 200), (np.uint16, 4096), (np.uint32, 70000)])
def test_huffman_shaped_multiary_equals_oracle(D, dt, sigma, levelwise):
    """d-ary Huffman codes of a geometric sequence, every symbol width"""
    if D == 3 and not levelwise:
        pytest.skip("3-bit digits are built level by level only")
    rng = np.random.default_rng(7 * D + sigma)
    n = 200003
    S = np.minimum(rng.geometric(0.01, n) - 1, sigma - 1).astype(dt)
    lens = dary.huffman_lengths(np.bincount(S.astype(np.int64), minlength=sigma), D)
    codes = dary.canonical(lens, D)
    img, want = build_both(S, sigma, D, lens, codes, levelwise)
    assert_same(img.cpu().numpy(), want, f"D={D} sigma={sigma} levelwise={levelwise}")
    run_queries(img, S, sigma, rng)


@pytest.mark.parametrize("levelwise", [False, True])
@pytest.mark.parametrize("D", [2, 4])
def test_shaped_multiary_long_levels(D, levelwise):
    """levels of 2^20 digits and more (stored select answers do not apply to
    digit levels; the counters and digit samples span several 2^20 blocks),
    a skewed alphabet whose deep levels are short"""
    rng = np.random.default_rng(50 + D)
    n, sigma = (1 << 21) + 333, 3000
    S = np.minimum(rng.geometric(0.02, n) - 1, sigma - 1).astype(np.uint16)
    lens = dary.huffman_lengths(np.bincount(S.astype(np.int64), minlength=sigma), D)
    codes = dary.canonical(lens, D)
    img, want = build_both(S, sigma, D, lens, codes, levelwise)
    assert_same(img.cpu().numpy(), want, f"D={D} levelwise={levelwise}")
    run_queries(img, S, sigma, rng)


@pytest.mark.parametrize("D", [2, 3, 4])
@pytest.mark.parametrize("seed", range(4))
def test_random_codes_shaped_multiary(D, seed):
    """random prefix-free codes over digits, up to 32 bits, with codewords
    for absent symbols (empty nodes), across sizes from one symbol up"""
    rng = np.random.default_rng(1000 * D + seed)
    for n in (1, 97, 5000, 70001):
        sigma = int(rng.integers(2, 3000))
        S = np.minimum(rng.geometric(0.003, n) - 1, sigma - 1).astype(np.uint16)
        lens = dary.random_lengths(sigma, D, rng)
        codes = dary.canonical(lens, D)
        for levelwise in ((True,) if D == 3 else (False, True)):
            img, want = build_both(S, sigma, D, lens, codes, levelwise)
            assert_same(img.cpu().numpy(), want,
                        f"D={D} seed={seed} n={n} sigma={sigma} h={int(lens.max())} levelwise={levelwise}")
            run_queries(img, S, sigma, rng, m=1500)
