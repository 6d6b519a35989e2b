"""Seeded random builds: kind, size, alphabet, symbol width, pass width and
chunk count drawn together, every image equal to the oracle's byte for byte
(combinations the targeted tests do not enumerate, e.g. a split shaped tree
under a forced pass width, or many chunks of a few tiles); and random
batches, every sequence's image equal to the oracle's; large draws (n from
2^18 to 2^23, hundreds of chunks); and draws whose n sits on a boundary of
words, superblocks, select samples, tiles or multiary (sub-)ranges, built
against the oracle and queried against brute force.  WV_RANDOM_DRAWS,
WV_RANDOM_BATCHES, WV_RANDOM_LARGE and WV_RANDOM_BOUNDARY set how many (48,
8, 2 and 16 by default); WV_RANDOM_LEVELWISE draws (8 by default) go through
the level-by-level builder; WV_RANDOM_RANGE draws (12 by default) plant one
symbol >= sigma, which every kind and the batch must report; WV_RANDOM_CODES
draws (8 by default) build shaped trees from random prefix-free codes (random
code trees up to 32 bits, not always full) and query them; WV_RANDOM_THREADS
(6 by default) draws per thread are built by four host threads at once, each
on its own stream."""
import os

import numpy as np
import pytest

from gpu_util import build_status, assert_same, gpu_image, oracle_image, shaped_codes
from paper_1610_03524_amd import binding as B

pytestmark = pytest.mark.gpu


def draw(rng):
    kind = int(rng.choice([B.KIND_WM, B.KIND_WT, B.KIND_SHAPED, B.KIND_MULTIARY]))
    n = int(2 ** rng.uniform(0, 18.2)) if rng.random() > 0.05 else 0
    sigma = max(1, int(2 ** rng.uniform(0, 20)))
    need = 1 if sigma <= 256 else (2 if sigma <= 65536 else 4)
    width = int(rng.choice([w for w in (1, 2, 4) if w >= need]))
    dt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[width]
    if kind == B.KIND_SHAPED or rng.random() < 0.3:   # skewed symbols: deep shaped trees
        S = np.minimum(rng.geometric(min(0.5, 8.0 / sigma + 1e-4), n) - 1, sigma - 1).astype(dt)
    else:
        S = rng.integers(0, sigma, n).astype(dt)
    tau = int(rng.choice([0, 0, 1, 2, 3, 5, 7, 8]))
    blocks = int(rng.choice([0, 0, 1, 2, 5, 33]))
    D = int(rng.integers(1, 5)) if kind == B.KIND_MULTIARY else 0
    return kind, S, sigma, tau, blocks, D


def check_draw(rng, seed, flags=0):
    kind, S, sigma, tau, blocks, D = draw(rng)
    tune = B.make_tuning(tau=tau, blocks=blocks, flags=flags)
    what = f"seed={seed} kind={kind} n={S.size} sigma={sigma} {S.dtype} tau={tau} blocks={blocks} D={D}"
    if kind == B.KIND_SHAPED:
        if S.size == 0:
            pytest.skip("a shaped tree needs at least one coded symbol")
        (gc, gl), (oc, ol) = shaped_codes(S, sigma)
        g = gpu_image(kind, S, sigma, codes=gc, lens=gl, tune=tune)
        o = oracle_image(kind, S, sigma, codes=oc, lens=ol)
    else:
        g = gpu_image(kind, S, sigma, D, tune=tune)
        o = oracle_image(kind, S, sigma, D)
    assert_same(g, o, what)


@pytest.mark.parametrize("seed", range(int(os.environ.get("WV_RANDOM_DRAWS", "48"))))
def test_random_build_equals_oracle(seed):
    check_draw(np.random.default_rng(5000 + seed), seed)


@pytest.mark.parametrize("seed", range(int(os.environ.get("WV_RANDOM_LEVELWISE", "8"))))
def test_random_levelwise_build_equals_oracle(seed):
    check_draw(np.random.default_rng(8000000 + seed), seed, B.FLAG_LEVELWISE)


@pytest.mark.parametrize("seed", range(int(os.environ.get("WV_RANDOM_BATCHES", "8"))))
def test_random_batch_equals_oracle(seed):
    from test_gpu_batch import run_batch
    rng = np.random.default_rng(90000 + seed)
    seqs, taus = [], []
    for _ in range(int(rng.integers(1, 40))):
        n = int(2 ** rng.uniform(0, 18)) if rng.random() > 0.05 else int(rng.integers(0, 3))
        sigma = max(1, int(2 ** rng.uniform(0, 20)))
        need = 1 if sigma <= 256 else (2 if sigma <= 65536 else 4)
        dt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[int(rng.choice([w for w in (1, 2, 4) if w >= need]))]
        if rng.random() < 0.3:
            S = np.minimum(rng.geometric(min(0.5, 4.0 / sigma + 1e-4), n) - 1, sigma - 1).astype(dt)
        else:
            S = rng.integers(0, sigma, n).astype(dt)
        seqs.append((S, sigma))
        taus.append(int(rng.choice([0, 0, 1, 2, 3, 5, 7, 8])))
    imgs = run_batch(seqs, taus=taus)
    for k, ((S, sigma), g) in enumerate(zip(seqs, imgs)):
        assert_same(g, oracle_image(B.KIND_WM, S, sigma), f"batch {seed} seq {k} n={S.size} sigma={sigma} tau={taus[k]}")


@pytest.mark.parametrize("seed", range(int(os.environ.get("WV_RANDOM_LARGE", "2"))))
def test_random_large_build_equals_oracle(seed):
    rng = np.random.default_rng(777000 + seed)
    kind = int(rng.choice([B.KIND_WM, B.KIND_WT, B.KIND_SHAPED, B.KIND_MULTIARY]))
    n = int(2 ** rng.uniform(18, 23))
    sigma = max(2, int(2 ** rng.uniform(1, 20)))
    need = 1 if sigma <= 256 else (2 if sigma <= 65536 else 4)
    dt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[int(rng.choice([w for w in (1, 2, 4) if w >= need]))]
    if kind == B.KIND_SHAPED or rng.random() < 0.4:
        S = np.minimum(rng.geometric(min(0.5, 8.0 / sigma + 1e-4), n) - 1, sigma - 1).astype(dt)
    else:
        S = rng.integers(0, sigma, n).astype(dt)
    tau = int(rng.choice([0, 0, 0, 3, 5, 7, 8]))
    blocks = int(rng.choice([0, 0, 0, 7, 100]))
    D = int(rng.integers(1, 5)) if kind == B.KIND_MULTIARY else 0
    tune = B.make_tuning(tau=tau, blocks=blocks)
    what = f"seed={seed} kind={kind} n={n} sigma={sigma} {S.dtype} tau={tau} blocks={blocks} D={D}"
    if kind == B.KIND_SHAPED:
        (gc, gl), (oc, ol) = shaped_codes(S, sigma)
        g = gpu_image(kind, S, sigma, codes=gc, lens=gl, tune=tune)
        o = oracle_image(kind, S, sigma, codes=oc, lens=ol)
    else:
        g = gpu_image(kind, S, sigma, D, tune=tune)
        o = oracle_image(kind, S, sigma, D)
    assert_same(g, o, what)


def boundary_draw(rng, sigma_lg, kinds=(B.KIND_WM, B.KIND_WT, B.KIND_SHAPED, B.KIND_MULTIARY)):
    kind = int(rng.choice(list(kinds)))
    D = int(rng.integers(1, 5)) if kind == B.KIND_MULTIARY else 0
    P = 21 if D == 3 else (64 >> (D >> 1) if D else 64)
    unit = int(rng.choice([64, 512, 4096, 8192, 8 * P, 64 * P, 256 * 64]))
    n = max(1, unit * int(rng.integers(1, 24)) + int(rng.choice([-1, 0, 0, 1])))
    sigma = max(1, int(2 ** rng.uniform(0, sigma_lg)))
    need = 1 if sigma <= 256 else (2 if sigma <= 65536 else 4)
    dt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[int(rng.choice([w for w in (1, 2, 4) if w >= need]))]
    if kind == B.KIND_SHAPED or rng.random() < 0.3:
        S = np.minimum(rng.geometric(min(0.5, 8.0 / sigma + 1e-4), n) - 1, sigma - 1).astype(dt)
    else:
        S = rng.integers(0, sigma, n).astype(dt)
    return kind, D, S, sigma, f"kind={kind} D={D} n={n} unit={unit} sigma={sigma} {S.dtype}"


@pytest.mark.parametrize("seed", range(int(os.environ.get("WV_RANDOM_BOUNDARY", "16"))))
def test_boundary_build_equals_oracle(seed):
    rng = np.random.default_rng(444000 + seed)
    kind, D, S, sigma, what = boundary_draw(rng, 20)
    tune = B.make_tuning(tau=int(rng.choice([0, 0, 2, 5, 8])), blocks=int(rng.choice([0, 0, 1, 3])))
    if kind == B.KIND_SHAPED:
        (gc, gl), (oc, ol) = shaped_codes(S, sigma)
        g = gpu_image(kind, S, sigma, codes=gc, lens=gl, tune=tune)
        o = oracle_image(kind, S, sigma, codes=oc, lens=ol)
    else:
        g = gpu_image(kind, S, sigma, D, tune=tune)
        o = oracle_image(kind, S, sigma, D)
    assert_same(g, o, f"seed={seed} {what}")


@pytest.mark.parametrize("seed", range(int(os.environ.get("WV_RANDOM_BOUNDARY", "16"))))
def test_boundary_queries_match_brute_force(seed):
    from gpu_util import to_device
    from test_gpu_queries import run_queries
    rng = np.random.default_rng(333000 + seed)
    kind, D, S, sigma, what = boundary_draw(rng, 16)
    if kind == B.KIND_SHAPED:
        (gc, gl), _ = shaped_codes(S, sigma)
        counts = B.symbol_counts(to_device(S), sigma).cpu().numpy()
        img, _ = B.build(kind, to_device(S), sigma, codes=gc, code_len=gl, counts=counts)
    else:
        img, _ = B.build(kind, to_device(S), sigma, arity_log2=D)
    run_queries(img, S, sigma, rng)


@pytest.mark.parametrize("seed", range(int(os.environ.get("WV_RANDOM_RANGE", "12"))))
def test_random_symbol_out_of_range_is_reported(seed):
    from gpu_util import to_device
    rng = np.random.default_rng(616000 + seed)
    n = int(2 ** rng.uniform(0, 20))
    sigma = max(1, int(2 ** rng.uniform(0, 16)))
    dt = np.uint8 if sigma < 256 else (np.uint16 if sigma < 65536 else np.uint32)
    S = rng.integers(0, sigma, n).astype(dt)
    bad = S.copy()
    i = int(rng.integers(0, n))
    bad[i] = int(rng.choice([sigma, min(np.iinfo(dt).max, 2 * sigma + 3), np.iinfo(dt).max]))
    what = f"seed={seed} n={n} sigma={sigma} {dt.__name__} bad S[{i}]={int(bad[i])}"
    img, _ = B.build(B.KIND_WM, to_device(bad), sigma)
    assert B.check(img) == B.WT_ERANGE, what
    for kind, D in ((B.KIND_WT, 0), (B.KIND_MULTIARY, int(rng.integers(1, 5))), (B.KIND_SHAPED, 0)):
        if kind == B.KIND_SHAPED:
            (gc, gl), _ = shaped_codes(S, sigma)
            counts = B.symbol_counts(to_device(S), sigma).cpu().numpy()
            st = build_status(kind, to_device(bad), sigma, codes=gc, code_len=gl, counts=counts)
        else:
            st = build_status(kind, to_device(bad), sigma, arity_log2=D)
        assert st == B.WT_ERANGE, f"{what} kind={kind} D={D}"
    # in a batch only the bad sequence is flagged; the others are built as alone
    seqs = [(S, sigma), (bad, sigma), (S[: n // 2 + 1].copy(), sigma)]
    imgs = run_batch_status(seqs)
    assert [st for st, _ in imgs] == [B.WT_OK, B.WT_ERANGE, B.WT_OK], what
    assert_same(imgs[0][1], oracle_image(B.KIND_WM, S, sigma), what)
    assert_same(imgs[2][1], oracle_image(B.KIND_WM, seqs[2][0], sigma), what)


def run_batch_status(seqs):
    """a batch of matrices; (status, image) per sequence"""
    import torch
    from gpu_util import to_device
    dev = [to_device(S) for S, _ in seqs]
    outs, descs = [], []
    for (S, sigma), St in zip(seqs, dev):
        info = B.plan(B.KIND_WM, S.size, sigma, S.itemsize)
        out = torch.empty(info.out_bytes, dtype=torch.uint8, device="cuda")
        d = B.wt_seq_desc()
        d.S, d.n, d.sigma, d.sym_bytes = St.data_ptr(), S.size, sigma, S.itemsize
        d.out, d.out_bytes = out.data_ptr(), info.out_bytes
        outs.append(out)
        descs.append(d)
    ws = torch.empty(max(B.batch_plan(B.KIND_WM, descs), 1), dtype=torch.uint8, device="cuda")
    assert B.batch_build(B.KIND_WM, descs, ws) == B.WT_OK
    torch.cuda.synchronize()
    return [(B.check(o), o.cpu().numpy()) for o in outs]


def random_code_tree(rng, sigma, maxlen):
    """codewords of a random binary code tree (leaves split at random, often
    along one deep path), some dropped so that the code need not be full,
    given to a random subset of the symbols"""
    leaves = [(0, 0)]
    deep = rng.random() < 0.5
    while len(leaves) < sigma:
        cand = [k for k, (c, l) in enumerate(leaves) if l < maxlen]
        if not cand:
            break
        k = cand[-1] if deep and rng.random() < 0.7 else int(rng.choice(cand))
        c, l = leaves.pop(k)
        leaves += [(2 * c, l + 1), (2 * c + 1, l + 1)]
    rng.shuffle(leaves)
    if rng.random() < 0.3 and len(leaves) > 2:
        leaves = leaves[: int(rng.integers(1, len(leaves)))]
    codes = np.zeros(sigma, np.uint64)
    lens = np.zeros(sigma, np.uint32)
    for s_, (c, l) in zip(rng.permutation(sigma)[: len(leaves)], leaves):
        codes[s_], lens[s_] = c, l
    return codes, lens


@pytest.mark.parametrize("seed", range(int(os.environ.get("WV_RANDOM_CODES", "8"))))
def test_shaped_tree_from_random_prefix_free_code(seed):
    from gpu_util import to_device
    from test_gpu_queries import run_queries
    rng = np.random.default_rng(909000 + seed)
    sigma = int(rng.integers(2, 600))
    codes, lens = random_code_tree(rng, sigma, int(rng.choice([8, 16, 24, 32])))
    if lens.max() == 0:
        pytest.skip("no codeword of positive length")
    counts = np.where(lens > 0, rng.integers(0, 400, sigma) * (rng.random(sigma) < 0.8), 0).astype(np.uint64)
    if counts.sum() == 0:
        counts[int(np.flatnonzero(lens)[0])] = 1
    S = rng.permutation(np.repeat(np.arange(sigma), counts.astype(np.int64))).astype(np.uint16)
    img, _ = B.build(B.KIND_SHAPED, to_device(S), sigma, codes=codes, code_len=lens, counts=counts)
    assert_same(img.cpu().numpy(), oracle_image(B.KIND_SHAPED, S, sigma, codes=codes, lens=lens),
                f"seed={seed} sigma={sigma} n={S.size} h={int(lens.max())}")
    run_queries(img, S, sigma, rng)


def test_concurrent_builds_from_several_threads():
    """the library's shared host state (pinned buffer pool, side stream,
    profile records) under builds of every kind from four threads, each on
    its own stream"""
    import threading
    import torch
    from gpu_util import to_device
    rounds = int(os.environ.get("WV_RANDOM_THREADS", "6"))
    results, errors = [], []

    def worker(tid):
        try:
            st = torch.cuda.Stream()
            for r in range(rounds):
                rng = np.random.default_rng(31337 * (tid + 1) + r)
                kind, S, sigma, tau, blocks, D = draw(rng)
                if S.size == 0 and kind == B.KIND_SHAPED:
                    continue
                tune = B.make_tuning(tau=tau, blocks=blocks)
                with torch.cuda.stream(st):
                    St = to_device(S)
                    if kind == B.KIND_SHAPED:
                        (gc, gl), (oc, ol) = shaped_codes(S, sigma)
                        counts = B.symbol_counts(St, sigma, stream=st).cpu().numpy().astype(np.uint64)
                        img, _ = B.build(kind, St, sigma, codes=gc, code_len=gl, counts=counts, tune=tune, stream=st)
                        want = (kind, S, sigma, 0, oc, ol)
                    else:
                        img, _ = B.build(kind, St, sigma, arity_log2=D, tune=tune, stream=st)
                        want = (kind, S, sigma, D, None, None)
                    st.synchronize()
                    results.append((img.cpu().numpy(), want, f"thread {tid} round {r} kind={kind} n={S.size}"))
        except Exception as e:   # reported after the join
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for g, (kind, S, sigma, D, oc, ol), what in results:
        o = oracle_image(kind, S, sigma, codes=oc, lens=ol) if kind == B.KIND_SHAPED else oracle_image(kind, S, sigma, D)
        assert_same(g, o, what)
