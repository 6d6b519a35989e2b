"""Parity at the full sizes of the benchmark configurations, in the launch
configuration bench.py times (default tuning; the tuned pass width for the
batch).  Where the oracle finishes in seconds (C1, C3, sampled C4 sequences)
the images are compared with the oracle's byte for byte; for the 2^28-symbol
matrix (C2) the checks are sampled outputs computed one by one from S and
properties that hold at any size."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same, gpu_image, oracle_image, shaped_codes, to_device
from imagewalk import MatrixWalk
from paper_1610_03524_amd import binding as B
from paper_1610_03524_amd import inputs

pytestmark = pytest.mark.gpu

SEL_STRIDE = 4096


def test_c2_full_size_matrix():
    """C2: 2^28 uint32 Zipf symbols, sigma 2^16; per-level zero counts equal
    the bit counts of S, sampled directory entries and select samples equal
    counts over the level words, and sampled access / rank equal S and counts
    over S"""
    import torch
    n, sigma = 1 << 28, 1 << 16
    S = inputs.c2_zipf(n=n, sigma=sigma, seed=2, device="cuda")
    info = B.plan(B.KIND_WM, n, sigma, 4)
    out = torch.empty(info.out_bytes, dtype=torch.uint8, device="cuda")
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device="cuda")
    assert B.build_into(B.KIND_WM, S, sigma, out, ws) == B.WT_OK
    torch.cuda.synchronize()
    assert B.check(out) == B.WT_OK
    img = out.cpu().numpy()
    Sh = S.cpu().numpy().view(np.uint32)
    del out, ws
    L = info.nlevels
    assert L == 16
    walk = MatrixWalk(img, L)
    rng = np.random.default_rng(28)
    for l in range(L):
        nl, zeros, ones, _, roff, s0off, s1off, nsel = walk.lv[l]
        assert nl == n
        want_zeros = int(np.count_nonzero(((Sh >> np.uint32(L - 1 - l)) & np.uint32(1)) == 0))
        assert zeros == want_zeros and ones == n - want_zeros, f"level {l} zero count"
        w = walk.words(l)
        ones_before = np.zeros(w.size + 1, dtype=np.int64)
        ones_before[1:] = np.cumsum(np.bitwise_count(w))
        # rank directory: zeros before every sampled superblock and sub-block
        for k in rng.integers(0, n // 512, 64):
            d = img[roff + 16 * k:roff + 16 * k + 16].view(np.uint64)
            assert int(d[0]) == 512 * k - ones_before[8 * k], f"level {l} superblock {k}"
            for q in range(1, 8):
                rel = (int(d[1]) >> (9 * (q - 1))) & 511
                assert rel == 64 * q - int(ones_before[8 * k + q] - ones_before[8 * k])
        # select samples: the (4096 j)-th one / zero (0-based ordinal)
        sel1 = img[s1off:s1off + 8 * nsel].view(np.uint64)
        sel0 = img[s0off:s0off + 8 * nsel].view(np.uint64)
        for j in rng.integers(0, max(1, ones // SEL_STRIDE), 8):
            p = int(sel1[j])
            assert walk.bit(l, p) == 1 and p - walk.rank0(l, p) == SEL_STRIDE * j
        for j in rng.integers(0, max(1, zeros // SEL_STRIDE), 8):
            p = int(sel0[j])
            assert walk.bit(l, p) == 0 and walk.rank0(l, p) == SEL_STRIDE * j
    for i in rng.integers(0, n, 512):
        assert walk.access(int(i)) == int(Sh[i]), f"access({i})"
    for c_src, i in zip(rng.integers(0, n, 6), rng.integers(0, n, 6)):
        c = int(Sh[c_src])
        assert walk.rank(c, int(i)) == int(np.count_nonzero(Sh[:i + 1] == c)), f"rank({c}, {i})"


def test_c1_full_size_balanced_tree():
    S = inputs.c1_uniform()
    assert_same(gpu_image(B.KIND_WT, S, 256), oracle_image(B.KIND_WT, S, 256), "C1")


@pytest.mark.parametrize("shape", ["huffman", "4-ary"])
def test_c3_full_size_trees(shape):
    S = inputs.c3_geometric()
    sigma = 4096
    if shape == "huffman":
        (gc, gl), (oc, ol) = shaped_codes(S, sigma)
        g = gpu_image(B.KIND_SHAPED, S, sigma, codes=gc, lens=gl)
        o = oracle_image(B.KIND_SHAPED, S, sigma, codes=oc, lens=ol)
    else:
        g = gpu_image(B.KIND_MULTIARY, S, sigma, 2)
        o = oracle_image(B.KIND_MULTIARY, S, sigma, 2)
    assert_same(g, o, f"C3 {shape}")


def test_c4_full_batch_sampled_sequences():
    """the whole C4 batch in one call; a sample of its sequences (the
    largest, the smallest, the widest alphabet and random ones) equals the
    oracle byte for byte"""
    import torch
    from paper_1610_03524_amd import tune as T
    ns, sig, children = inputs.c4_sizes()
    count = ns.size
    dev_S, descs, imgs = [], [], []
    for i in range(count):
        S = inputs.c4_sequence(int(ns[i]), int(sig[i]), children[i])
        St = to_device(S)
        tau = T.choose_tau(S.size, int(sig[i]))
        ob = B.plan(B.KIND_WM, S.size, int(sig[i]), 4, tune=B.make_tuning(tau=tau)).out_bytes
        img = torch.empty(ob, dtype=torch.uint8, device="cuda")
        d = B.wt_seq_desc()
        d.S, d.n, d.sigma, d.sym_bytes, d.out, d.out_bytes, d.tau = St.data_ptr(), S.size, int(sig[i]), 4, \
            img.data_ptr(), ob, tau
        dev_S.append(St)
        descs.append(d)
        imgs.append(img)
    ws = torch.empty(B.batch_plan(B.KIND_WM, descs), dtype=torch.uint8, device="cuda")
    assert B.batch_build(B.KIND_WM, descs, ws) == B.WT_OK
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    pick = {int(np.argmax(ns)), int(np.argmin(ns)), int(np.argmax(sig))} | set(int(x) for x in rng.integers(0, count, 9))
    for i in sorted(pick):
        S = inputs.c4_sequence(int(ns[i]), int(sig[i]), children[i])
        assert_same(imgs[i].cpu().numpy(), oracle.build_image(oracle.KIND_WM, S, int(sig[i])), f"C4 sequence {i}")
