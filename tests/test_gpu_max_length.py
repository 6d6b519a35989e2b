"""Sequences of n = 2^32 - 1 symbols, the longest the library takes.

Cut into chunks one per resident workgroup, such a sequence gives chunks
that together cover 2^32 keys or more, so chunk ends, tile starts and chunk
lengths must not wrap in 32 bits (one chunk of it would not fit 32 bits at
all).  The oracle cannot build 4 G symbols in a test's time; the checks are
properties that hold at any size: level 0 of either kind is the top key bit
of S in input order, word for word; every level's zero count; access at
sampled positions (every chunk boundary and the tail included) equals S;
rank and select agree with counts over S."""
import numpy as np
import pytest

from paper_1610_03524_amd import binding as B

pytestmark = pytest.mark.gpu

N = (1 << 32) - 1
SIGMA = 4            # two levels, built by one pass of 2-bit digits
STEP = 1 << 26       # symbols per piece of the host-side checks (multiple of 64)


@pytest.fixture(scope="module")
def seq():
    """S on the device, and the count of every symbol in every STEP-piece"""
    import torch
    g = torch.Generator(device="cuda").manual_seed(31)
    S = torch.randint(0, SIGMA, (N,), dtype=torch.uint8, device="cuda", generator=g)
    pieces = torch.stack([torch.bincount(S[a:a + STEP].to(torch.int32), minlength=SIGMA)
                          for a in range(0, N, STEP)]).cpu().numpy().astype(np.int64)
    yield S, pieces
    del S
    torch.cuda.empty_cache()


def count_upto(S, pieces, c, i):
    """occurrences of c in S[0..i]"""
    p = (i + 1) // STEP
    rest = int((S[p * STEP:i + 1] == c).sum()) if (i + 1) % STEP else 0
    return int(pieces[:p, c].sum()) + rest


@pytest.mark.parametrize("kind", [B.KIND_WM, B.KIND_WT])
def test_longest_sequence(seq, kind):
    import torch
    S, pieces = seq
    img, info = B.build(kind, S, SIGMA)
    torch.cuda.synchronize()
    assert B.check(img) == B.WT_OK
    lv = img[256:256 + 64 * 2].cpu().numpy().view(np.uint64).reshape(2, 8)   # n_l, zeros, ones, bits_off, ...
    assert int(lv[0, 0]) == N and int(lv[1, 0]) == N
    # level 0: bit 1 of every symbol in input order, 64 symbols a word, LSB first
    off = int(lv[0, 3])
    words = img[off:off + 8 * ((N + 63) // 64)].view(torch.int64)
    shifts = torch.arange(64, device="cuda", dtype=torch.int64)
    for a in range(0, N, STEP):
        m = min(N, a + STEP) - a
        bits = ((S[a:a + m] >> 1) & 1).to(torch.int64)
        if m % 64:
            bits = torch.nn.functional.pad(bits, (0, 64 - m % 64))
        packed = (bits.view(-1, 64) << shifts).sum(dim=1)
        assert torch.equal(packed, words[a // 64:a // 64 + packed.numel()]), f"level 0 from symbol {a}"
    total = pieces.sum(axis=0)
    assert int(lv[0, 1]) == int(total[0] + total[1]), "zeros of level 0"
    assert int(lv[1, 1]) == int(total[0] + total[2]), "zeros of level 1"
    # access: every boundary of the chunks of the library's geometry, the
    # tail, and random positions
    rng = np.random.default_rng(kind)
    C = 1 << 22          # chunk length of 1024 chunks over 2^32 - 1 keys
    edges = np.concatenate([np.arange(C, N, C) + d for d in (-2, -1, 0, 1)])
    pos = np.unique(np.concatenate([edges, np.arange(N - 300, N), rng.integers(0, N, 4096)])).astype(np.int64)
    got = B.access(img, torch.from_numpy(pos).cuda()).cpu().numpy().view(np.uint32)
    want = S[torch.from_numpy(pos).cuda()].cpu().numpy()
    assert np.array_equal(got, want), f"access: {np.count_nonzero(got != want)} of {pos.size} wrong"
    # rank at sampled positions, and select of the occurrence found there
    ip = np.concatenate([[0, N - 1, N - 2, N - C, N - C - 1], rng.integers(0, N, 12)]).astype(np.int64)
    cs = S[torch.from_numpy(ip).cuda()].cpu().numpy().astype(np.int64)
    ranks = np.array([count_upto(S, pieces, int(c), int(i)) for c, i in zip(cs, ip)], dtype=np.int64)
    gr = B.rank(img, torch.from_numpy(cs.astype(np.int32)).cuda(), torch.from_numpy(ip).cuda()).cpu().numpy()
    assert np.array_equal(gr, ranks), "rank"
    gs = B.select(img, torch.from_numpy(cs.astype(np.int32)).cuda(), torch.from_numpy(ranks).cuda()).cpu().numpy()
    assert np.array_equal(gs, ip), "select of the occurrence at each sampled position"
    del img
    torch.cuda.empty_cache()
