"""Sequences of n = 2^32 - 1 symbols, the longest the library takes.

Cut into chunks one per resident workgroup, such a sequence gives chunks
that together cover 2^32 keys or more, so chunk ends, tile starts and chunk
lengths must not wrap in 32 bits (one chunk of it would not fit 32 bits at
all).  The oracle cannot build 4 G symbols in a test's time; the checks are
properties that hold at any size: level 0 of a matrix or binary tree is the
top key bit of S in input order, and the one level of a 4-ary tree over four
symbols is S itself as 2-bit digits, word for word; every binary level's
zero count; access at sampled positions (every chunk boundary and the tail
included) equals S; rank and select agree with counts over S."""
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


def packed_words(S, a, m, D, digit):
    """the words of a level holding `digit`(S[a:a+m]) in input order, D bits a
    symbol, 64 / D symbols a word, LSB first (m a multiple of 64 / D or the
    end of S)"""
    import torch
    P = 64 // D
    v = digit(S[a:a + m]).to(torch.int64)
    if m % P:
        v = torch.nn.functional.pad(v, (0, P - m % P))
    shifts = torch.arange(0, 64, D, device="cuda", dtype=torch.int64)
    return (v.view(-1, P) << shifts).sum(dim=1)


@pytest.mark.parametrize("kind,D", [(B.KIND_WM, 0), (B.KIND_WT, 0), (B.KIND_MULTIARY, 2)])
def test_longest_sequence(seq, kind, D):
    import torch
    S, pieces = seq
    img, info = B.build(kind, S, SIGMA, arity_log2=D)
    torch.cuda.synchronize()
    assert B.check(img) == B.WT_OK
    nl = int(img[28:32].cpu().numpy().view(np.uint32)[0])
    lv = img[256:256 + 64 * nl].cpu().numpy().view(np.uint64).reshape(nl, 8)   # n_l, zeros, ones, bits_off, ...
    assert nl == (1 if D == 2 else 2) and all(int(x) == N for x in lv[:, 0])
    # level 0 in input order: the top key bit of every symbol (binary), or
    # every symbol as one 2-bit digit (4-ary)
    bits = 2 if D == 2 else 1
    digit = (lambda x: x) if D == 2 else (lambda x: (x >> 1) & 1)
    off = int(lv[0, 3])
    words = img[off:off + 8 * ((N * bits + 63) // 64)].view(torch.int64)
    per = STEP * bits // 64
    for a in range(0, N, STEP):
        got = packed_words(S, a, min(N, a + STEP) - a, bits, digit)
        assert torch.equal(got, words[a // STEP * per:a // STEP * per + got.numel()]), f"level 0 from symbol {a}"
    if D != 2:
        total = pieces.sum(axis=0)
        assert int(lv[0, 1]) == int(total[0] + total[1]), "zeros of level 0"
        assert int(lv[1, 1]) == int(total[0] + total[2]), "zeros of level 1"
    # access: every boundary of the chunks of the library's geometry, the
    # tail, and random positions
    rng = np.random.default_rng(kind + D)
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


def test_longest_sequence_in_a_batch(seq):
    """The batched build over the longest sequence and a short one: the long
    image equals the single build's byte for byte (its properties are checked
    above), the short one the oracle's"""
    import torch
    import oracle
    S, _ = seq
    small = np.random.default_rng(5).integers(0, 300, 100003).astype(np.uint32)
    Ss = torch.from_numpy(small.view(np.int32)).cuda()
    single, _ = B.build(B.KIND_WM, S, SIGMA)
    descs, imgs = [], []
    for t, sigma, width in ((S, SIGMA, 1), (Ss, 300, 4)):
        info = B.plan(B.KIND_WM, t.numel(), sigma, width)
        img = torch.empty(info.out_bytes, dtype=torch.uint8, device="cuda")
        d = B.wt_seq_desc()
        d.S, d.n, d.sigma, d.sym_bytes = t.data_ptr(), t.numel(), sigma, width
        d.out, d.out_bytes = img.data_ptr(), info.out_bytes
        descs.append(d)
        imgs.append(img)
    ws = torch.empty(max(B.batch_plan(B.KIND_WM, descs), 1), dtype=torch.uint8, device="cuda")
    assert B.batch_build(B.KIND_WM, descs, ws) == B.WT_OK
    torch.cuda.synchronize()
    assert all(B.check(img) == B.WT_OK for img in imgs)
    assert torch.equal(imgs[0], single), "long sequence: batched image differs from the single build"
    assert np.array_equal(imgs[1].cpu().numpy(), oracle.build_image(oracle.KIND_WM, small, 300)), "short sequence"
    del single, imgs, ws
    torch.cuda.empty_cache()


def test_longest_sequence_huffman_shaped(seq):
    """A Huffman-shaped tree over the longest sequence (a 32-bit key per
    symbol in the workspace, 16 GiB): level 0 holds the first codeword bit of
    every symbol in input order, word for word; access, rank and select
    agree with S"""
    import torch
    S, pieces = seq
    counts = pieces.sum(axis=0).astype(np.uint64)
    codes, lens = B.huffman_codes(counts)
    img, _ = B.build(B.KIND_SHAPED, S, SIGMA, codes=codes, code_len=lens, counts=counts)
    torch.cuda.synchronize()
    assert B.check(img) == B.WT_OK
    lv = img[256:256 + 64].cpu().numpy().view(np.uint64)
    assert int(lv[0]) == N
    first = torch.tensor([(int(c) >> (int(ln) - 1)) & 1 for c, ln in zip(codes, lens)], dtype=torch.uint8,
                         device="cuda")
    off = int(lv[3])
    words = img[off:off + 8 * ((N + 63) // 64)].view(torch.int64)
    per = STEP // 64
    for a in range(0, N, STEP):
        got = packed_words(S, a, min(N, a + STEP) - a, 1, lambda x: first[x.long()])
        assert torch.equal(got, words[a // STEP * per:a // STEP * per + got.numel()]), f"level 0 from symbol {a}"
    rng = np.random.default_rng(99)
    pos = np.unique(np.concatenate([np.arange(N - 300, N), rng.integers(0, N, 4096)])).astype(np.int64)
    got = B.access(img, torch.from_numpy(pos).cuda()).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, S[torch.from_numpy(pos).cuda()].cpu().numpy()), "access"
    ip = np.concatenate([[0, N - 1, N - 2], rng.integers(0, N, 12)]).astype(np.int64)
    cs = S[torch.from_numpy(ip).cuda()].cpu().numpy().astype(np.int64)
    ranks = np.array([count_upto(S, pieces, int(c), int(i)) for c, i in zip(cs, ip)], dtype=np.int64)
    gr = B.rank(img, torch.from_numpy(cs.astype(np.int32)).cuda(), torch.from_numpy(ip).cuda()).cpu().numpy()
    assert np.array_equal(gr, ranks), "rank"
    gs = B.select(img, torch.from_numpy(cs.astype(np.int32)).cuda(), torch.from_numpy(ranks).cuda()).cpu().numpy()
    assert np.array_equal(gs, ip), "select"
    del img
    torch.cuda.empty_cache()


def test_longest_sequence_level_by_level(seq):
    """The level-by-level builder (an 8-ary tree: one level of 3-bit digits,
    21 to a word; 64 GiB of workspace) over the longest sequence: the level
    is S itself in input order, word for word; access, rank and select agree
    with S"""
    import torch
    S, pieces = seq
    img, _ = B.build(B.KIND_MULTIARY, S, SIGMA, arity_log2=3)
    torch.cuda.synchronize()
    assert B.check(img) == B.WT_OK
    lv = img[256:256 + 64].cpu().numpy().view(np.uint64)
    assert int(img[28:32].cpu().numpy().view(np.uint32)[0]) == 1 and int(lv[0]) == N
    P, step = 21, 21 << 21           # digits a word; symbols a piece (whole words)
    words = img[int(lv[3]):int(lv[3]) + 8 * ((N + P - 1) // P)].view(torch.int64)
    shifts = torch.arange(0, 3 * P, 3, device="cuda", dtype=torch.int64)
    for a in range(0, N, step):
        m = min(N, a + step) - a
        v = S[a:a + m].to(torch.int64)
        if m % P:
            v = torch.nn.functional.pad(v, (0, P - m % P))
        got = (v.view(-1, P) << shifts).sum(dim=1)
        assert torch.equal(got, words[a // P:a // P + got.numel()]), f"level from symbol {a}"
    rng = np.random.default_rng(3)
    pos = np.unique(np.concatenate([np.arange(N - 300, N), rng.integers(0, N, 4096)])).astype(np.int64)
    got = B.access(img, torch.from_numpy(pos).cuda()).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, S[torch.from_numpy(pos).cuda()].cpu().numpy()), "access"
    ip = np.concatenate([[0, N - 1, N - 2], rng.integers(0, N, 12)]).astype(np.int64)
    cs = S[torch.from_numpy(ip).cuda()].cpu().numpy().astype(np.int64)
    ranks = np.array([count_upto(S, pieces, int(c), int(i)) for c, i in zip(cs, ip)], dtype=np.int64)
    gr = B.rank(img, torch.from_numpy(cs.astype(np.int32)).cuda(), torch.from_numpy(ip).cuda()).cpu().numpy()
    assert np.array_equal(gr, ranks), "rank"
    gs = B.select(img, torch.from_numpy(cs.astype(np.int32)).cuda(), torch.from_numpy(ranks).cuda()).cpu().numpy()
    assert np.array_equal(gs, ip), "select"
    del img
    torch.cuda.empty_cache()
