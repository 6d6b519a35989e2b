"""Pins of the CPU oracle against things other than itself (no GPU needed).

* the worked example on the sequence of Fig. 1 (values derived by hand);
* brute-force access/rank/select walked through the image, exhaustively on
  tiny inputs (a wrong bit, index or sign anywhere breaks a walk);
* closed forms: every level is a stable argsort of S by a key derived from
  the symbol (library sort, not the oracle's partition loop);
* directories against cumulative sums and ``flatnonzero``;
* Huffman codes: Kraft sum, optimal cost from an independent heap merge,
  canonical order.
"""
import heapq
import itertools
import json
import os

import numpy as np
import pytest

import dary
import oracle
from imagewalk import Image, KIND_MULTI, KIND_SHAPED, KIND_WM, KIND_WT, LEAF

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def key_bits(sigma):
    return max(1, (sigma - 1).bit_length())


def bitrev(v, nbits):
    out = np.zeros_like(v)
    for t in range(nbits):
        out |= ((v >> t) & 1) << (nbits - 1 - t)
    return out


def wm_closed_form(S, sigma):
    """level l = bit l of S stably sorted by the bit-reversed top-l prefix"""
    L = key_bits(sigma)
    x = S.astype(np.int64)
    out = []
    for l in range(L):
        pre = (x >> (L - l)) if l else np.zeros_like(x)
        order = np.argsort(bitrev(pre, l), kind="stable")
        out.append(((x[order] >> (L - 1 - l)) & 1).astype(np.uint8))
    return out


def wt_closed_form(S, sigma):
    """level l = bit l of S stably sorted by the top-l prefix"""
    L = key_bits(sigma)
    x = S.astype(np.int64)
    out = []
    for l in range(L):
        pre = (x >> (L - l)) if l else np.zeros_like(x)
        order = np.argsort(pre, kind="stable")
        out.append(((x[order] >> (L - 1 - l)) & 1).astype(np.uint8))
    return out


def multi_closed_form(S, sigma, D):
    L = key_bits(sigma)
    M = -(-L // D)
    Lb = D * M
    x = S.astype(np.int64)
    out = []
    for be in range(M):
        pre = (x >> (Lb - D * be)) if be else np.zeros_like(x)
        order = np.argsort(pre, kind="stable")
        out.append((x[order] >> (Lb - D * (be + 1))) & ((1 << D) - 1))
    return out


def brute_rank(S, c, i):
    return int(np.count_nonzero(S[:i + 1] == c))


def brute_select(S, c, k):
    pos = np.flatnonzero(S == c)
    return int(pos[k - 1]) if 1 <= k <= pos.size else None


def build(kind, S, sigma, D=1):
    if kind == KIND_SHAPED and D >= 2:
        lens = dary.huffman_lengths(oracle.symbol_counts(S, sigma), D)
        return oracle.build_image(kind, S, sigma, D, codes=dary.canonical(lens, D), lens=lens)
    if kind == KIND_SHAPED:
        codes, lens = oracle.huffman(oracle.symbol_counts(S, sigma))
        return oracle.build_image(kind, S, sigma, codes=codes, lens=lens)
    return oracle.build_image(kind, S, sigma, D)


def check_queries(img: Image, S: np.ndarray, sigma: int, all_symbols=True):
    n = S.size
    for i in range(n):
        assert img.access(i) == int(S[i]), ("access", i)
    syms = range(sigma) if all_symbols else np.unique(S)
    for c in syms:
        c = int(c)
        for i in range(n):
            assert img.rank_sym(c, i) == brute_rank(S, c, i), ("rank", c, i)
        cnt = int(np.count_nonzero(S == c))
        for k in range(1, cnt + 2):
            assert img.select_sym(c, k) == brute_select(S, c, k), ("select", c, k)


# ---------------------------------------------------------------------------
# worked example (Fig. 1 caption sequence)
# ---------------------------------------------------------------------------

def test_fig1_worked_example():
    with open(os.path.join(GOLDEN, "fig1_example.json")) as f:
        g = json.load(f)
    S = np.array(g["S"], dtype=np.uint8)
    sigma = g["sigma"]
    for kind, key in ((KIND_WT, "wt"), (KIND_WM, "wm")):
        img = Image(oracle.build_image(kind, S, sigma))
        assert img.magic == 0x54564157 and img.kind == kind and img.nlevels == g["L"]
        for l in range(g["L"]):
            bits = "".join(str(int(b)) for b in img.bits(l))
            assert bits == g[f"{key}_levels"][l]
            assert img.levels[l]["zeros"] == g[f"{key}_zeros"][l]
            assert int(img.words(l)[0]) == int(g[f"{key}_words_hex"][l], 16)
        for i, x in g["queries"]["access"]:
            assert img.access(i) == x
        for c, i, r in g["queries"]["rank"]:
            assert img.rank_sym(c, i) == r
        for c, k, p in g["queries"]["select"]:
            assert img.select_sym(c, k) == p
    # the node bitstrings of level 2 of the tree, concatenated left to right
    img = Image(oracle.build_image(KIND_WT, S, sigma))
    assert "".join(str(int(b)) for b in img.bits(2)) == "".join(g["wt_level2_nodes"])
    # final wavelet-matrix order = stable sort by the bit-reversed symbol
    order = np.argsort(bitrev(S.astype(np.int64), 3), kind="stable")
    assert S[order].tolist() == g["wm_final_order"]
    img4 = Image(oracle.build_image(KIND_MULTI, S, sigma, 2))
    assert img4.nlevels == 2
    for l in range(2):
        assert img4.digits(l).tolist() == g["multiary4_levels"][l]
    for i, x in g["queries"]["access"]:
        assert img4.access(i) == x


# ---------------------------------------------------------------------------
# brute force on every tiny input
# ---------------------------------------------------------------------------

def tiny_cases():
    for sigma, nmax in ((1, 4), (2, 6), (3, 5), (4, 4), (5, 3)):
        for n in range(0, nmax + 1):
            for t in itertools.product(range(sigma), repeat=n):
                yield sigma, np.array(t, dtype=np.uint8)


@pytest.mark.parametrize("kind,D", [(KIND_WT, 1), (KIND_WM, 1), (KIND_MULTI, 1),
                                    (KIND_MULTI, 2), (KIND_MULTI, 3), (KIND_SHAPED, 1)])
def test_exhaustive_tiny_queries(kind, D):
    for sigma, S in tiny_cases():
        if kind == KIND_SHAPED and S.size == 0:
            continue
        img = Image(build(kind, S, sigma, D))
        assert img.n == S.size and img.status == 0
        check_queries(img, S, sigma)


# ---------------------------------------------------------------------------
# closed forms on random inputs
# ---------------------------------------------------------------------------

SIZES = [0, 1, 2, 63, 64, 65, 300, 511, 512, 513]
SIGMAS = [1, 2, 3, 4, 5, 7, 8, 9, 255, 256, 257, 4096, 65536]


@pytest.mark.parametrize("sigma", SIGMAS)
def test_closed_forms_wt_wm(sigma):
    rng = np.random.default_rng(sigma)
    dt = np.uint8 if sigma <= 256 else (np.uint16 if sigma <= 65536 else np.uint32)
    for n in SIZES:
        S = rng.integers(0, sigma, n).astype(dt)
        for kind, cf in ((KIND_WT, wt_closed_form), (KIND_WM, wm_closed_form)):
            img = Image(oracle.build_image(kind, S, sigma))
            assert img.nlevels == img.key_bits == key_bits(sigma)
            for l, want in enumerate(cf(S, sigma)):
                assert np.array_equal(img.bits(l), want), (kind, n, l)
                assert img.levels[l]["n"] == n
                assert img.levels[l]["zeros"] == int(np.count_nonzero(want == 0))
                assert img.levels[l]["ones"] == int(np.count_nonzero(want))
        # both kinds share levels 0 and 1 (one node or two halves)
        a = Image(oracle.build_image(KIND_WT, S, sigma))
        b = Image(oracle.build_image(KIND_WM, S, sigma))
        for l in range(min(2, a.nlevels)):
            assert np.array_equal(a.bits(l), b.bits(l))


@pytest.mark.parametrize("D", [1, 2, 3, 4])
@pytest.mark.parametrize("sigma", [2, 5, 16, 17, 255, 4096])
def test_closed_forms_multiary(D, sigma):
    rng = np.random.default_rng(100 + D * sigma)
    for n in SIZES + [5000]:
        S = rng.integers(0, sigma, n).astype(np.uint16)
        img = Image(oracle.build_image(KIND_MULTI, S, sigma, D))
        want = multi_closed_form(S, sigma, D)
        assert img.nlevels == len(want) and img.arity_log2 == D
        for l, w in enumerate(want):
            got = img.digits(l)
            assert np.array_equal(got, w), (n, l)
            # counters against cumulative counts
            sb, blk = img.digit_counters(l)
            p = 64 // D
            d = 1 << D
            cum = np.zeros((n + 1, d), dtype=np.int64)
            for c in range(d):
                cum[1:, c] = np.cumsum(w == c)
            for k in range(sb.shape[0]):
                assert np.array_equal(sb[k].astype(np.int64), cum[min(k * 64 * p, n)])
            for bi in range(blk.shape[0]):
                t = bi * 8 * p
                base = cum[(t // (64 * p)) * 64 * p]
                assert np.array_equal(blk[bi].astype(np.int64), cum[t] - base)


def test_multiary_top_bit_matches_binary_level():
    # with L divisible by D, digit level beta's top bit is binary level beta*D
    rng = np.random.default_rng(7)
    S = rng.integers(0, 256, 3000).astype(np.uint8)
    wt = Image(oracle.build_image(KIND_WT, S, 256))
    for D in (1, 2, 4):
        mt = Image(oracle.build_image(KIND_MULTI, S, 256, D))
        for be in range(mt.nlevels):
            top = (mt.digits(be) >> (D - 1)) & 1
            assert np.array_equal(top.astype(np.uint8), wt.bits(be * D))


# ---------------------------------------------------------------------------
# directories
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [0, 1, 511, 512, 513, 4095, 4096, 4097, 20000, 70001])
def test_rank_select_directory(n):
    rng = np.random.default_rng(n)
    sigma = 2
    for p1 in (0.0, 0.03, 0.5, 1.0):
        S = (rng.random(n) < p1).astype(np.uint8)
        img = Image(oracle.build_image(KIND_WM, S, sigma))
        bits = img.bits(0)
        assert np.array_equal(bits, S)
        zp = np.concatenate([[0], np.cumsum(bits == 0)])
        d = img.rank_dir(0)
        ns = -(-n // 512)
        assert d.shape[0] == ns + 1
        for k in range(ns + 1):
            s = min(512 * k, n)
            assert int(d[k, 0]) == zp[s]
            want = 0
            if 512 * k < n:
                for j in range(1, 8):
                    want |= int(zp[min(512 * k + 64 * j, n)] - zp[512 * k]) << (9 * (j - 1))
            assert int(d[k, 1]) == want
        for i in list(range(0, n + 1, 97)) + [n]:
            assert img.rank0_via_directory(0, i) == zp[i]
        nsel = -(-n // 4096) + 1
        for which in (0, 1):
            s = img.sel(0, which)
            pos = np.flatnonzero(bits == which)[::4096]
            want = np.full(nsel, n, dtype=np.uint64)
            want[:pos.size] = pos
            assert np.array_equal(s, want)
        # second sampling level: every 512th one from the front, every 512th
        # zero from the back, n in between (at least one such entry)
        nsub = -(-n // 512) + 2
        sub = img.sub(0)
        ones, zeros = np.flatnonzero(bits == 1)[::512], np.flatnonzero(bits == 0)[::512]
        want = np.full(nsub, n, dtype=np.uint32)
        want[:ones.size] = ones
        want[nsub - zeros.size:] = zeros[::-1]
        assert ones.size + zeros.size < nsub
        assert np.array_equal(sub, want)
        # padding bits past n are zero
        w = img.words(0)
        if n % 64:
            assert int(w[-1]) >> (n % 64) == 0


# ---------------------------------------------------------------------------
# Huffman codes and shaped trees
# ---------------------------------------------------------------------------

def heap_cost(counts):
    h = [int(c) for c in counts if c > 0]
    if len(h) <= 1:
        return sum(h)
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


@pytest.mark.parametrize("seed", range(12))
def test_huffman_codes(seed):
    rng = np.random.default_rng(seed)
    sigma = int(rng.integers(1, 300))
    counts = rng.integers(0, 50, sigma).astype(np.uint64)
    if seed % 3 == 0:
        counts = (rng.geometric(0.2, sigma) - 1).astype(np.uint64)
    codes, lens = oracle.huffman(counts)
    used = counts > 0
    assert np.all((lens > 0) == used)
    k = int(used.sum())
    if k == 0:
        return
    if k == 1:
        assert lens[used].tolist() == [1]
        return
    assert sum(2.0 ** -int(l) for l in lens[used]) == pytest.approx(1.0)
    assert int((counts * lens.astype(np.uint64)).sum()) == heap_cost(counts)
    # canonical: ordered by (len, symbol) the codes increase, prefix-free
    syms = sorted(np.flatnonzero(used), key=lambda s: (int(lens[s]), int(s)))
    prev_left = -1
    for s in syms:
        left = int(codes[s]) << (64 - int(lens[s]))
        assert left > prev_left
        prev_left = left
    assert int(codes[syms[0]]) == 0


def test_huffman_tie_rule_small():
    # counts (5,1,1,2,0,7): merges {1,1}->2, then leaf 2 before node 2 -> 4,
    # then 4+5 -> 9, then 7+9: lengths 2,4,4,3,-,1 ; canonical codes
    codes, lens = oracle.huffman(np.array([5, 1, 1, 2, 0, 7], dtype=np.uint64))
    assert lens.tolist() == [2, 4, 4, 3, 0, 1]
    assert codes.tolist() == [0b10, 0b1110, 0b1111, 0b110, 0, 0b0]


def check_shaped(S, sigma, codes, lens, queries_upto=300):
    """Every level, node record and code-table entry of a shaped image against
    closed forms from the codewords (Sec. 4.3, arbitrarily-shaped trees):
    level l holds bit l of the codewords longer than l, stably sorted by their
    l-bit prefix; a node (l, P) starts after the level-l symbols whose prefix is
    smaller than P, whether or not any symbol under P occurs in S."""
    img = Image(oracle.build_image(KIND_SHAPED, S, sigma, codes=codes, lens=lens))
    h = int(lens.max())
    assert img.nlevels == h == img.key_bits
    cs = codes.astype(np.int64)[S]          # codeword of every position
    ls = lens.astype(np.int64)[S]
    for l in range(h):
        sel = np.flatnonzero(ls > l)
        pre = (cs[sel] >> (ls[sel] - l)) if l else np.zeros(sel.size, dtype=np.int64)
        order = sel[np.argsort(pre, kind="stable")]
        want = ((cs[order] >> (ls[order] - 1 - l)) & 1).astype(np.uint8)
        assert np.array_equal(img.bits(l), want)
        assert img.levels[l]["n"] == sel.size
    gc, gl = img.codes()
    assert np.array_equal(gc[lens > 0], codes[lens > 0]) and np.array_equal(gl, lens)
    # node table: every proper prefix once, ordered by (level, prefix)
    nodes = img.nodes()
    c64 = codes.astype(np.int64)
    l64 = lens.astype(np.int64)
    keys = sorted({(l, int(c64[s] >> (l64[s] - l)) if l else 0)
                   for s in np.flatnonzero(lens) for l in range(int(l64[s]))})
    assert [(nd["level"], nd["prefix"]) for nd in nodes] == keys
    keyset = set(keys)
    leaves = {(int(l64[s]), int(c64[s])): int(s) for s in np.flatnonzero(lens)}
    empty = 0
    for nd in nodes:
        l, p = nd["level"], nd["prefix"]
        sel = ls > l
        pre = (cs >> np.maximum(ls - l, 0)) if l else np.zeros_like(cs)
        members = sel & (pre == p)
        assert nd["count"] == int(members.sum())
        assert nd["start"] == int((sel & (pre < p)).sum()), (l, p)
        empty += nd["count"] == 0
        for b in (0, 1):
            ch = nd["child"][b]
            q = 2 * p + b
            if (l + 1, q) in leaves:
                assert ch == (LEAF | leaves[(l + 1, q)])
            elif (l + 1, q) in keyset:
                assert nodes[ch]["level"] == l + 1 and nodes[ch]["prefix"] == q
            else:
                assert ch == 0xFFFFFFFF
    # queries walked through the image on a prefix of S (brute force is O(n))
    m = min(S.size, queries_upto)
    if m:
        sub = S[:m]
        img2 = Image(oracle.build_image(KIND_SHAPED, sub, sigma, codes=codes, lens=lens))
        check_queries(img2, sub, sigma, all_symbols=sigma <= 64)
    return empty


@pytest.mark.parametrize("seed", range(6))
def test_shaped_closed_form_and_nodes(seed):
    rng = np.random.default_rng(50 + seed)
    sigma = [3, 17, 100, 4096, 2, 64][seed]
    n = [1, 200, 2000, 5000, 64, 777][seed]
    S = np.minimum(rng.geometric(0.05, n) - 1, sigma - 1).astype(np.uint16)
    codes, lens = oracle.huffman(oracle.symbol_counts(S, sigma))
    check_shaped(S, sigma, codes, lens)


def _code_prefix(codes, lens, s, l):
    return int(codes[s]) >> (int(lens[s]) - l) if l else 0


@pytest.mark.parametrize("seed", range(8))
def test_shaped_empty_nodes(seed):
    """Codewords given to symbols that never occur in S make empty nodes,
    and a whole absent subtree makes a chain of them; their start offsets
    (and every other record) must follow the closed form."""
    rng = np.random.default_rng(900 + seed)
    sigma = [5, 9, 16, 33, 100, 257, 4096, 12][seed]
    # every symbol gets a codeword (Huffman over counts + 1) ...
    w = rng.integers(1, 50, sigma).astype(np.uint64)
    codes, lens = oracle.huffman(w)
    assert (lens > 0).all()
    # ... but the symbols under one internal prefix, plus a few others, never
    # occur in S (full code, absent subtree and absent leaves)
    coded = np.flatnonzero(lens)
    s0 = int(rng.choice(coded))
    l0 = int(rng.integers(1, max(2, int(lens[s0]))))
    l0 = min(l0, int(lens[s0]) - 1) if lens[s0] > 1 else 0
    p0 = _code_prefix(codes, lens, s0, l0)
    absent = {int(s) for s in coded if lens[s] > l0 and _code_prefix(codes, lens, s, l0) == p0}
    absent |= {int(s) for s in rng.choice(coded, size=max(1, sigma // 5), replace=False)}
    present = np.array(sorted(set(range(sigma)) - absent), dtype=np.int64)
    if present.size == 0:
        present = np.array([int(coded[0])])
    n = int(rng.integers(1, 3000))
    S = present[rng.integers(0, present.size, n)].astype(np.uint16)
    empty = check_shaped(S, sigma, codes, lens)
    assert empty > 0


@pytest.mark.parametrize("variant", range(4))
def test_shaped_empty_nodes_incomplete_code(variant):
    """Empty nodes under a prefix code that is not full: unary-like codes with
    the deepest or a middle codeword's symbol absent."""
    sigma = 6
    # 0 -> 0, 1 -> 10, 2 -> 110, 3 -> 1110, 4 -> 11110, 5 -> 111110 (1111111 unused)
    lens = np.arange(1, sigma + 1, dtype=np.uint32)
    codes = np.array([(1 << int(l)) - 2 for l in lens], dtype=np.uint64)
    rng = np.random.default_rng(77 + variant)
    absent = [{5}, {4, 5}, {0, 5}, {1, 2, 3, 4, 5}][variant]
    present = np.array([s for s in range(sigma) if s not in absent])
    S = present[rng.integers(0, present.size, 40)].astype(np.uint8)
    empty = check_shaped(S, sigma, codes, lens)
    assert empty > 0


def test_exhaustive_tiny_queries_absent_codewords():
    """Brute force on every tiny input, with a codeword for every symbol of
    the alphabet whether or not it occurs (so most inputs have empty nodes)."""
    for sigma, S in tiny_cases():
        if S.size == 0 or sigma < 2:
            continue
        codes, lens = oracle.huffman(np.arange(1, sigma + 1, dtype=np.uint64))
        img = Image(oracle.build_image(KIND_SHAPED, S, sigma, codes=codes, lens=lens))
        assert img.n == S.size and img.status == 0
        check_queries(img, S, sigma)


def test_shaped_incomplete_code():
    # a prefix code that is not full: 0 -> "0", 1 -> "10", 2 -> "110"
    codes = np.array([0b0, 0b10, 0b110], dtype=np.uint64)
    lens = np.array([1, 2, 3], dtype=np.uint32)
    S = np.array([2, 0, 1, 1, 2, 0, 0], dtype=np.uint8)
    img = Image(oracle.build_image(KIND_SHAPED, S, 3, codes=codes, lens=lens))
    nodes = img.nodes()
    assert [(nd["level"], nd["prefix"]) for nd in nodes] == [(0, 0), (1, 1), (2, 3)]
    assert nodes[2]["child"] == (LEAF | 2, 0xFFFFFFFF)
    check_queries(img, S, 3)


# ---------------------------------------------------------------------------
# errors and layout
# ---------------------------------------------------------------------------

def test_errors():
    with pytest.raises(oracle.OracleError) as e:
        oracle.build_image(KIND_WM, np.array([0, 5, 1], dtype=np.uint8), 5)
    assert e.value.code == oracle.ERANGE
    with pytest.raises(oracle.OracleError) as e:
        oracle.build_image(KIND_WT, np.array([0], dtype=np.uint8), 0)
    assert e.value.code == oracle.EINVAL
    with pytest.raises(oracle.OracleError) as e:
        oracle.build_image(KIND_MULTI, np.array([0], dtype=np.uint8), 4, 5)
    assert e.value.code == oracle.EINVAL
    codes = np.array([0, 1, 0], dtype=np.uint64)
    lens = np.array([1, 1, 0], dtype=np.uint32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.build_image(KIND_SHAPED, np.array([0, 2], dtype=np.uint8), 3, codes=codes, lens=lens)
    assert e.value.code == oracle.ERANGE


@pytest.mark.parametrize("kind,D", [(KIND_WT, 1), (KIND_WM, 1), (KIND_MULTI, 2), (KIND_SHAPED, 1),
                                    (KIND_SHAPED, 2), (KIND_SHAPED, 4)])
def test_layout(kind, D):
    rng = np.random.default_rng(kind)
    S = rng.integers(0, 37, 1000).astype(np.uint8)
    check_layout(build(kind, S, 37, D), kind, D)


def check_layout(buf, kind, D=1):
    """every array on a 256-byte boundary, no two overlap, every byte outside
    them zero"""
    img = Image(buf)
    assert img.image_bytes == buf.size and buf.size % 256 == 0
    spans = [(0, 256 + 64 * img.nlevels)]
    for l, lv in enumerate(img.levels):
        for key in ("bits_off", "rank_off", "sel0_off", "sel1_off"):
            if lv[key]:
                assert lv[key] % 256 == 0
        m = lv["n"]
        if img.multi_levels:
            p = 64 // D
            d = 1 << D
            spans.append((lv["bits_off"], lv["bits_off"] + 8 * (-(-m // p))))
            nsb, nb = -(-m // (64 * p)), -(-m // (8 * p))
            spans.append((lv["rank_off"], lv["rank_off"] + (nsb + 1) * d * 8 + nb * d * 2))
            spans.append((lv["sel0_off"], lv["sel0_off"] + d * lv["nsel"] * 8))
        else:
            spans.append((lv["bits_off"], lv["bits_off"] + 8 * (-(-m // 64))))
            spans.append((lv["rank_off"], lv["rank_off"] + 16 * (-(-m // 512) + 1)))
            spans.append((lv["sel0_off"], lv["sel0_off"] + 8 * lv["nsel"]))
            spans.append((lv["sel1_off"], lv["sel1_off"] + 8 * lv["nsel"]))
            assert lv["sub_off"] % 256 == 0 and lv["nsub"] == -(-m // 512) + 2
            spans.append((lv["sub_off"], lv["sub_off"] + 4 * lv["nsub"]))
            assert lv["pool_off"] % 256 == 0 and lv["nslot"] == m >> 20
            spans.append((lv["pool_off"], lv["pool_off"] + 4 * 2 * lv["nslot"] * 512))
    if kind == KIND_SHAPED:
        rb = 32 if D == 1 else 24 + 4 * (1 << D)
        spans.append((img.nodes_off, img.nodes_off + rb * img.nnodes))
        spans.append((img.codes_off, img.codes_off + 16 * img.sigma))
    spans.sort()
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert a1 <= b0
    covered = np.zeros(buf.size, dtype=bool)
    for a, b in spans:
        covered[a:b] = True
    assert not buf[~covered].any(), "bytes outside every array must be zero"


LONG = 1 << 20


def select_through_structure(img, l, b, j):
    """the select of the query path: the sub-samples of ordinals 512s and
    512(s+1) bound a stretch; a stretch of 2^20 bits or more answers from its
    pool slot, any other by a search of the stretch (brute force here)"""
    lv = img.levels[l]
    sub, nsub = img.sub(l), lv["nsub"]
    s = j // 512
    p0 = int(sub[s] if b else sub[nsub - 1 - s])
    p1 = int(sub[s + 1] if b else sub[nsub - 2 - s])
    if p1 - p0 >= LONG:
        slot = (0 if b else lv["nslot"]) + (p0 >> 20)
        return int(img.pool(l)[slot * 512 + j % 512]), True
    inside = np.flatnonzero(img.bits(l)[p0:p1] == b)
    return p0 + int(inside[j - 512 * s]), False


def long_stretch_bits(case, n, rng):
    """bit strings whose 512-one (or zero) stretches include long ones: a
    dense block, a block of 512 spread over about a million bits, and a short
    tail spread to the end; complemented for zeros; or sparse at random"""
    if case == "random":
        return (rng.random(n) < 1 / 2500).astype(np.uint8)
    b = np.zeros(n, dtype=np.uint8)
    if case == "edge":
        # a stretch of exactly 2^20 bits (long), then a tail of 2^20 - 1 (not)
        b[:512] = 1
        b[np.linspace(1000, 1000 + LONG, 512, endpoint=False).astype(np.int64)] = 1
        b[1000 + LONG] = 1
        assert n == 1000 + 2 * LONG - 1
        return b
    b[:512] = 1
    b[np.linspace(1000, 1000 + 1_100_000, 512, endpoint=False).astype(np.int64)] = 1
    b[np.linspace(1_200_000, n - 1, 37).astype(np.int64)] = 1
    return b if case == "ones" else 1 - b


@pytest.mark.parametrize("case", ["ones", "zeros", "random", "edge"])
def test_long_stretches_store_every_answer(case):
    """Clark's rule for long ranges (Sec. 5.1, "Select"): selects through the
    sub-samples and the pool of stored answers equal brute force for every
    ordinal of every long stretch and for sampled others; a slot is in use
    exactly for each long stretch, its positions hold the right bit and
    increase; unused entries are n; the layout stays valid at n >= 2^20"""
    rng = np.random.default_rng({"ones": 1, "zeros": 2, "random": 3, "edge": 4}[case])
    n = 1000 + 2 * LONG - 1 if case == "edge" else (1 << 21) + 300000
    bits = long_stretch_bits(case, n, rng)
    buf = oracle.build_image(KIND_WM, bits, 2)
    check_layout(buf, KIND_WM)
    img = Image(buf)
    nslot = img.levels[0]["nslot"]
    assert nslot == n >> 20
    pool = img.pool(0).reshape(2 * nslot, 512)
    for b in (0, 1):
        pos = np.flatnonzero(bits == b)
        long_ordinals, nlong = [], 0
        for j0 in range(0, pos.size, 512):
            end = pos[j0 + 512] if j0 + 512 < pos.size else n
            if end - pos[j0] >= LONG:
                nlong += 1
                long_ordinals.extend(range(j0, min(j0 + 512, pos.size)))
        if case == ("ones" if b else "zeros"):
            assert nlong == 2   # the spread block and the tail
        if case == "random" and b == 1:
            assert nlong >= 1
        if case == "edge":
            assert nlong == b
        from_pool = 0
        for j in long_ordinals + [int(x) for x in rng.integers(0, pos.size, 300)]:
            got, stored = select_through_structure(img, 0, b, j)
            assert got == pos[j], (b, j)
            from_pool += stored
        assert from_pool >= len(long_ordinals)
        slots = pool[:nslot] if b else pool[nslot:]
        in_use = 0
        for row in slots:
            live = row[row != n].astype(np.int64)
            in_use += live.size > 0
            assert np.all(bits[live] == b) and np.all(np.diff(live) > 0)
        assert in_use == nlong


def test_matrix_walk_on_oracle_images():
    """the directory-only matrix reader of the full-size GPU tests, on oracle
    images: access equals S, rank equals counts over S"""
    from imagewalk import MatrixWalk
    rng = np.random.default_rng(9)
    for sigma, n in [(2, 1000), (300, 5000), (1 << 16, 70001)]:
        S = rng.integers(0, sigma, n).astype(np.uint32)
        img = oracle.build_image(oracle.KIND_WM, S, sigma)
        L = max(1, (sigma - 1).bit_length())
        w = MatrixWalk(img, L)
        for i in rng.integers(0, n, 200):
            assert w.access(int(i)) == int(S[i])
        for c_src, i in zip(rng.integers(0, n, 50), rng.integers(0, n, 50)):
            c = int(S[c_src])
            assert w.rank(c, int(i)) == int(np.count_nonzero(S[:i + 1] == c))


@pytest.mark.parametrize("D", [1, 2, 3, 4])
def test_multiary_select_samples(D):
    """Per-digit select samples of every multiary level (Sec. 5.2, "Select":
    a sampled structure per character): for every digit value c the position
    of its occurrences of ordinal 0, 4096, 8192, ... (numpy flatnonzero), then
    the level length as sentinel, ceil(n/4096)+1 entries per digit"""
    rng = np.random.default_rng(90 + D)
    for sigma, n in [(3, 20000), (16, 50001), (200, 9000), (1 << 12, 30000), (2, 4096), (5, 1)]:
        # skewed digits, so some values are dense and some sparse
        S = np.minimum(rng.geometric(0.2, n) - 1, sigma - 1).astype(np.uint16)
        img = Image(oracle.build_image(KIND_MULTI, S, sigma, D))
        want_digits = multi_closed_form(S, sigma, D)
        for l, lv in enumerate(img.levels):
            m = lv["n"]
            nsel = -(-m // 4096) + 1
            assert lv["nsel"] == nsel and lv["sel0_off"] % 256 == 0 and lv["sel1_off"] == 0
            dig = want_digits[l]
            tab = np.frombuffer(img.buf[lv["sel0_off"]:lv["sel0_off"] + 8 * nsel * (1 << D)].tobytes(),
                                dtype=np.uint64).reshape(1 << D, nsel)
            for c in range(1 << D):
                pos = np.flatnonzero(dig == c)[::4096]
                want = np.full(nsel, m, dtype=np.uint64)
                want[:pos.size] = pos
                assert np.array_equal(tab[c], want), (sigma, n, D, l, c)


# ---------------------------------------------------------------------------
# shaped trees over D-bit digits (Sec. 4.3: shapes carry over to multiary
# trees); pinned against closed forms and brute force, never against the
# binary shaped code path
# ---------------------------------------------------------------------------

def dary_prefix(codes, lens, syms, l, D):
    c = codes[syms].astype(np.uint64)
    sh = (D * (lens[syms].astype(np.int64) - l)).astype(np.uint64)
    return np.where(l > 0, c >> sh, np.uint64(0))


@pytest.mark.parametrize("D", [2, 3, 4])
@pytest.mark.parametrize("seed", range(6))
def test_shaped_multiary_closed_form(D, seed):
    """level l holds digit l of every symbol whose codeword is longer than l,
    stably sorted by its l-digit prefix; each node record's start and count
    are the symbols of its level under smaller prefixes and under its own; a
    child is the node of the extended prefix, else the leaf of the symbol
    whose codeword it is, else absent"""
    rng = np.random.default_rng(100 * D + seed)
    d = 1 << D
    sigma = int(rng.integers(2, 400))
    n = int(rng.integers(1, 4000))
    S = np.minimum(rng.geometric(0.02, n) - 1, sigma - 1).astype(np.uint16)
    lens = dary.random_lengths(sigma, D, rng)   # codewords for absent symbols too
    codes = dary.canonical(lens, D)
    img = Image(oracle.build_image(KIND_SHAPED, S, sigma, D, codes=codes, lens=lens))
    h = int(lens.max())
    assert img.nlevels == h and img.arity_log2 == D and img.multi_levels
    for l in range(h):
        idx = np.flatnonzero(lens[S] > l)
        pre = dary_prefix(codes, lens, S[idx], l, D)
        order = idx[np.argsort(pre, kind="stable")]
        want = (codes[S[order]] >> (np.uint64(D) * (lens[S[order]].astype(np.uint64) - np.uint64(1 + l)))) & np.uint64(d - 1)
        assert np.array_equal(img.digits(l), want.astype(np.int64)), f"level {l}"
        assert img.levels[l]["n"] == idx.size
    nodes = img.nodes()
    keys = {(nd["level"], nd["prefix"]): t for t, nd in enumerate(nodes)}
    want_keys = {(l, int(p)) for s_ in range(sigma) for l in range(int(lens[s_]))
                 for p in [int(codes[s_]) >> (D * (int(lens[s_]) - l)) if l else 0]}
    assert set(keys) == want_keys
    assert [k for k in sorted(keys)] == [(nd["level"], nd["prefix"]) for nd in nodes]
    leaf = {(int(lens[s_]), int(codes[s_])): s_ for s_ in range(sigma) if lens[s_]}
    for nd in nodes:
        l, p = nd["level"], nd["prefix"]
        idx = np.flatnonzero(lens[S] > l)
        pre = dary_prefix(codes, lens, S[idx], l, D)
        assert nd["count"] == int(np.count_nonzero(pre == p))
        assert nd["start"] == int(np.count_nonzero(pre < p))
        for c in range(d):
            q = p * d + c
            if (l + 1, q) in keys:
                assert nd["child"][c] == keys[(l + 1, q)]
            elif (l + 1, q) in leaf:
                assert nd["child"][c] == LEAF | leaf[(l + 1, q)]
            else:
                assert nd["child"][c] == 0xFFFFFFFF


@pytest.mark.parametrize("D", [2, 3])
def test_shaped_multiary_tiny_exhaustive_queries(D):
    """every sequence of length <= 4 over 4 symbols, with a d-ary Huffman code
    and with a random code that also covers absent symbols: access, rank and
    select walked through the image equal brute force"""
    rng = np.random.default_rng(D)
    sigma = 4
    for n in range(1, 5):
        for S in itertools.product(range(sigma), repeat=n):
            S = np.array(S, dtype=np.uint8)
            for variant in range(2):
                if variant == 0:
                    lens = dary.huffman_lengths(oracle.symbol_counts(S, sigma), D)
                else:
                    lens = dary.random_lengths(sigma, D, rng)
                codes = dary.canonical(lens, D)
                img = Image(oracle.build_image(KIND_SHAPED, S, sigma, D, codes=codes, lens=lens))
                check_queries(img, S, sigma, all_symbols=variant == 1)


def test_shaped_multiary_refusals():
    """a codeword of more than 32 bits is refused, and so is a symbol of S
    without a codeword"""
    S = np.array([0, 1, 2], dtype=np.uint8)
    lens = np.array([9, 1, 1], dtype=np.uint32)   # 9 digits of 4 bits
    codes = dary.canonical(lens, 4)
    with pytest.raises(oracle.OracleError) as e:
        oracle.build_image(KIND_SHAPED, S, 3, 4, codes=codes, lens=lens)
    assert e.value.code == oracle.EUNSUP
    lens = np.array([1, 1, 0], dtype=np.uint32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.build_image(KIND_SHAPED, S, 3, 2, codes=dary.canonical(lens, 2), lens=lens)
    assert e.value.code == oracle.ERANGE
