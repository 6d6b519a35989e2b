"""Huffman codewords computed on the device (one workgroup): equal, symbol by
symbol, to the oracle's canonical codes and to the library's host rule, on
counts with ties, absent symbols, a single symbol, skewed and flat
distributions, and lengths past 32 bits (refused through the status word)."""
import numpy as np
import pytest

import oracle
from gpu_util import to_device
from paper_1610_03524_amd import binding as B

pytestmark = pytest.mark.gpu


def dev_codes(counts):
    import torch
    c = torch.from_numpy(np.asarray(counts, dtype=np.uint64).view(np.int64)).cuda()
    codes, lens, st = B.huffman_codes_dev(c)
    torch.cuda.synchronize()
    return codes.cpu().numpy().view(np.uint64), lens.cpu().numpy().view(np.uint32), int(st.cpu()[0])


def count_cases():
    rng = np.random.default_rng(31)
    yield np.array([5], dtype=np.uint64)                        # one symbol
    yield np.array([0, 0, 7, 0], dtype=np.uint64)               # one present among absent
    yield np.array([3, 3, 3, 3, 3, 3], dtype=np.uint64)         # all tied
    yield np.array([1, 1, 2, 3, 5, 8, 13, 21], dtype=np.uint64)
    yield np.zeros(17, dtype=np.uint64)                         # nothing present
    for sigma in (2, 3, 100, 1000, 4096):
        for _ in range(3):
            yield rng.integers(0, 50, sigma).astype(np.uint64)
            yield np.bincount(np.minimum(rng.geometric(0.01, 200000) - 1, sigma - 1), minlength=sigma).astype(np.uint64)
            w = rng.integers(1, 5, sigma).astype(np.uint64)
            w[rng.random(sigma) < 0.3] = 0
            yield w


def test_device_huffman_equals_oracle_and_host_rule():
    for k, counts in enumerate(count_cases()):
        dc, dl, st = dev_codes(counts)
        assert st == B.WT_OK, k
        oc, ol = oracle.huffman(counts)
        hc, hl = B.huffman_codes(counts)
        assert np.array_equal(dl, ol) and np.array_equal(dl, hl), f"case {k}: lengths"
        m = ol > 0
        assert np.array_equal(dc[m], oc[m]) and np.array_equal(dc[m], hc[m]), f"case {k}: codes"
        assert not dc[~m].any()


def test_device_huffman_refuses_lengths_past_32_bits():
    # Fibonacci weights make one code per symbol longer: 40 symbols need
    # lengths far past 32, which both rules refuse
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    counts = np.array(fib, dtype=np.uint64)
    dc, dl, st = dev_codes(counts)
    assert st == B.WT_EUNSUP and not dl.any() and not dc.any()
    with pytest.raises(B.WaveletError) as e:
        B.huffman_codes(counts)
    assert e.value.code == B.WT_EUNSUP


def test_device_codes_shape_a_tree_equal_to_the_oracle():
    """the device counts and codes shape a Huffman tree equal to the oracle's
    (counts, codes and lengths stay on the device until the plan needs them)"""
    import torch
    rng = np.random.default_rng(5)
    S = np.minimum(rng.geometric(0.02, 300001) - 1, 3999).astype(np.uint16)
    St = to_device(S)
    counts_d = B.symbol_counts(St, 4000)
    codes_d, lens_d, st_d = B.huffman_codes_dev(counts_d)
    torch.cuda.synchronize()
    assert int(st_d.cpu()[0]) == B.WT_OK
    counts = counts_d.cpu().numpy().view(np.uint64)
    codes = codes_d.cpu().numpy().view(np.uint64)
    lens = lens_d.cpu().numpy().view(np.uint32)
    img, _ = B.build(B.KIND_SHAPED, St, 4000, codes=codes, code_len=lens, counts=counts)
    torch.cuda.synchronize()
    oc, ol = oracle.huffman(oracle.symbol_counts(S, 4000))
    want = oracle.build_image(oracle.KIND_SHAPED, S, 4000, codes=oc, lens=ol)
    assert np.array_equal(img.cpu().numpy(), want)
