"""C-ABI checks that need no GPU: the library loads, exports every entry
point the header declares, and its host-only calls (planning, Huffman
codewords) agree with the oracle."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_1610_03524_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "wavelet.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    names = header_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(B.exported_symbols())


@pytest.mark.parametrize("kind,sigma,D", [(B.KIND_WT, 256, 0), (B.KIND_WM, 65536, 0), (B.KIND_MULTIARY, 4096, 2),
                                          (B.KIND_MULTIARY, 5, 3), (B.KIND_MULTIARY, 70000, 4), (B.KIND_WM, 1, 0),
                                          (B.KIND_WT, 3, 0), (B.KIND_WM, 2 ** 20, 0)])
@pytest.mark.parametrize("n", [0, 1, 64, 513, 4097, 100000])
def test_plan_matches_oracle_layout(kind, sigma, D, n):
    dt = np.uint8 if sigma <= 256 else (np.uint16 if sigma <= 65536 else np.uint32)
    S = np.zeros(n, dtype=dt)
    info = B.plan(kind, n, sigma, S.itemsize, B.make_shape(D) if D else None)
    img = oracle.build_image(kind, S, sigma, max(D, 1))
    assert info.out_bytes == img.size
    L = max(1, (sigma - 1).bit_length())
    assert info.nlevels == (L if kind != B.KIND_MULTIARY else -(-L // D))
    assert info.workspace_bytes > 0


def test_plan_shaped_matches_oracle():
    rng = np.random.default_rng(3)
    S = np.minimum(rng.geometric(0.05, 5000) - 1, 299).astype(np.uint16)
    counts = oracle.symbol_counts(S, 300)
    codes, lens = oracle.huffman(counts)
    info = B.plan(B.KIND_SHAPED, S.size, 300, 2, B.make_shape(0, codes, lens, counts))
    img = oracle.build_image(oracle.KIND_SHAPED, S, 300, codes=codes, lens=lens)
    assert info.out_bytes == img.size and info.nlevels == int(lens.max())


@pytest.mark.parametrize("seed", range(20))
def test_huffman_codes_equal_oracle(seed):
    rng = np.random.default_rng(seed)
    sigma = int(rng.integers(1, 5000))
    if seed % 4 == 0:
        counts = rng.integers(0, 3, sigma)
    elif seed % 4 == 1:
        counts = rng.geometric(0.01, sigma)
    else:
        counts = rng.integers(0, 10 ** int(rng.integers(1, 9)), sigma)
    codes, lens = B.huffman_codes(counts)
    ocodes, olens = oracle.huffman(counts)
    assert np.array_equal(lens, olens) and np.array_equal(codes, ocodes)


def test_plan_errors():
    with pytest.raises(B.WaveletError) as e:
        B.plan(B.KIND_WM, 10, 0, 1)
    assert e.value.code == B.WT_EINVAL
    with pytest.raises(B.WaveletError) as e:
        B.plan(B.KIND_WM, 10, 5, 3)
    assert e.value.code == B.WT_EINVAL
    with pytest.raises(B.WaveletError) as e:
        B.plan(B.KIND_MULTIARY, 10, 5, 1, B.make_shape(5))
    assert e.value.code == B.WT_EINVAL
    with pytest.raises(B.WaveletError) as e:
        B.plan(B.KIND_WM, 1 << 32, 5, 1)
    assert e.value.code == B.WT_EUNSUP
    # a symbol that occurs but has no codeword
    with pytest.raises(B.WaveletError) as e:
        B.plan(B.KIND_SHAPED, 3, 3, 1, B.make_shape(0, np.array([0, 1, 0]), np.array([1, 1, 0]),
                                                      np.array([1, 1, 1])))
    assert e.value.code == B.WT_ERANGE
    assert "out of range" in B.strerror(B.WT_ERANGE)


@pytest.mark.parametrize("codes, lens", [
    ([0, 1, 2], [1, 2, 2]),      # "0" is a prefix of "01"
    ([1, 1, 0], [2, 2, 1]),      # the same codeword twice
    ([0, 0, 3], [2, 3, 2]),      # "00" is a prefix of "000"
])
def test_plan_rejects_codes_that_are_not_prefix_free(codes, lens):
    with pytest.raises(B.WaveletError) as e:
        B.plan(B.KIND_SHAPED, 3, 3, 1, B.make_shape(0, np.array(codes), np.array(lens), np.array([1, 1, 1])))
    assert e.value.code == B.WT_EINVAL


def test_plan_counts_shaped_nodes():
    """internal nodes = distinct proper prefixes of the codewords, counted
    from the codewords in padded order"""
    rng = np.random.default_rng(3)
    for _ in range(20):
        counts = rng.integers(0, 50, int(rng.integers(2, 300)))
        counts[rng.integers(0, counts.size)] += 1
        codes, lens = B.huffman_codes(counts)
        prefixes = {(l, int(c) >> (int(k) - l)) for c, k in zip(codes, lens) for l in range(int(k))}
        img_bytes = B.plan(B.KIND_SHAPED, int(counts.sum()), counts.size, 2,
                           B.make_shape(0, codes, lens, counts)).out_bytes
        oimg = oracle.build_image(oracle.KIND_SHAPED,
                                  np.repeat(np.arange(counts.size), counts).astype(np.uint16), counts.size,
                                  codes=codes, lens=lens)
        assert img_bytes == oimg.size
        assert int(oimg[64:72].view(np.uint64)[0]) == len(prefixes)


def test_misaligned_buffers_are_rejected_before_device_work():
    """S, out and ws must be 16-byte aligned: addresses that are not are
    refused on the host, before any device call (none is made here)"""
    L = B.lib()
    big = 1 << 30
    for S, out, ws in ((0x10001, 0x20000, 0x30000), (0x10000, 0x20008, 0x30000), (0x10000, 0x20000, 0x30004)):
        for fn in (L.wm_build, L.wt_build):
            assert fn(S, 1000, 100, 1, None, None, out, big, ws, big, None) == B.WT_EINVAL
    d = B.wt_seq_desc()
    d.S, d.n, d.sigma, d.sym_bytes, d.out, d.out_bytes = 0x10002, 1000, 100, 1, 0x20000, big
    with pytest.raises(B.WaveletError) as e:
        B.batch_plan(B.KIND_WM, [d])
    assert e.value.code == B.WT_EINVAL


def expected_shape_verdict(codes, lens, counts, n):
    """the plan's verdict on a codeword set, from its stated rules: per
    symbol in order, a code longer than 32 bits is unsupported, a code with
    bits above its length is invalid, a symbol that occurs without a code is
    out of range; then the lengths must not all be 0 and the counts must add
    up to n; then no codeword may be a prefix of another (checked here pair by
    pair)"""
    for c, l, k in zip(codes, lens, counts):
        if l > 32:
            return B.WT_EUNSUP
        if l and (c >> l):
            return B.WT_EINVAL
        if k and not l:
            return B.WT_ERANGE
    if max(lens) == 0 or sum(counts) != n:
        return B.WT_EINVAL
    coded = [(c, l) for c, l in zip(codes, lens) if l]
    for i in range(len(coded)):
        for j in range(len(coded)):
            (ci, li), (cj, lj) = coded[i], coded[j]
            if i != j and li <= lj and (cj >> (lj - li)) == ci:
                return B.WT_EINVAL
    return B.WT_OK


@pytest.mark.parametrize("seed", range(400))
def test_plan_verdict_on_random_codeword_sets(seed):
    rng = np.random.default_rng(424242 + seed)
    sigma = int(rng.integers(1, 40))
    if rng.random() < 0.5:   # a valid Huffman code, perturbed
        counts = rng.integers(0, 20, sigma)
        counts[rng.integers(0, sigma)] += 1
        codes, lens = B.huffman_codes(counts)
        codes, lens = [int(c) for c in codes], [int(l) for l in lens]
        for _ in range(int(rng.integers(0, 3))):
            s = int(rng.integers(0, sigma))
            what = int(rng.integers(0, 4))
            if what == 0:
                lens[s] = int(rng.integers(0, 36))
            elif what == 1:
                codes[s] = int(rng.integers(0, 1 << 12))
            elif what == 2:
                counts[s] = int(rng.integers(0, 5))
            else:
                codes[s] ^= 1
        counts = [int(k) for k in counts]
    else:                    # arbitrary codewords
        lens = [int(rng.integers(0, 8)) if rng.random() < 0.95 else int(rng.integers(30, 36)) for _ in range(sigma)]
        codes = [int(rng.integers(0, 1 << max(l, 1))) if rng.random() < 0.9 else int(rng.integers(0, 1 << 10))
                 for l in lens]
        counts = [int(rng.integers(0, 4)) for _ in range(sigma)]
    n = sum(counts) + (int(rng.integers(-1, 2)) if rng.random() < 0.1 else 0)
    n = max(n, 0)
    want = expected_shape_verdict(codes, lens, counts, n)
    shape = B.make_shape(0, np.array(codes, dtype=np.uint64), np.array(lens), np.array(counts))
    try:
        B.plan(B.KIND_SHAPED, n, sigma, 1, shape)
        got = B.WT_OK
    except B.WaveletError as e:
        got = e.code
    assert got == want, (sigma, codes, lens, counts, n)


def test_binding_rejects_bad_arguments_before_the_library():
    """The binding refuses, with WT_EINVAL and before any pointer reaches the
    library, arguments the header does not allow: host arrays, element types
    of another width, strided views, paired arrays of different lengths, and
    host tensors (no GPU is needed: every case is refused on the host)."""
    import torch
    img = torch.zeros(4096, dtype=torch.uint8)
    pos64 = torch.zeros(8, dtype=torch.int64)
    c32 = torch.zeros(8, dtype=torch.int32)

    def refused(fn, *args, match):
        with pytest.raises(B.WaveletError) as e:
            fn(*args)
        assert e.value.code == B.WT_EINVAL and match in str(e.value), str(e.value)

    refused(B.access, img.numpy(), pos64, match="torch tensor")
    refused(B.access, img, pos64.to(torch.int32), match="dtype int32")
    refused(B.access, img, torch.zeros(16, dtype=torch.int64)[::2], match="contiguous")
    refused(B.access, img.to(torch.int64), pos64, match="dtype int64")
    refused(B.access, img, pos64, match="device tensors")
    refused(B.rank, img, c32.to(torch.int64), pos64, match="dtype int64")
    refused(B.rank, img, c32, pos64.to(torch.int32), match="dtype int32")
    refused(B.rank, img, c32[:5], pos64, match="lengths differ")
    refused(B.rank, img, c32, pos64, match="device tensors")
    refused(B.select, img, c32, pos64[:3], match="lengths differ")
    refused(B.select, img, c32, pos64.float(), match="dtype float32")
    refused(B.select, img, c32, pos64, match="device tensors")
    S = torch.zeros(100, dtype=torch.int32)
    ws = torch.zeros(1 << 16, dtype=torch.uint8)
    refused(B.build_into, B.KIND_WM, S.to(torch.int64), 100, img, ws, match="dtype int64")
    refused(B.build_into, B.KIND_WM, S[::2], 100, img, ws, match="contiguous")
    refused(B.build_into, B.KIND_WM, S, 100, img.to(torch.int32), ws, match="dtype int32")
    refused(B.build_into, B.KIND_WM, S, 100, img, ws, match="device tensors")
    refused(B.symbol_counts, S.double(), 100, match="dtype float64")
    refused(B.check, img, match="device tensors")
    refused(B.image_bytes, img[::2], match="contiguous")
    refused(B.make_desc, S, 100, img, match="device tensors")
    refused(B.batch_build, B.KIND_WM, [], ws.to(torch.int16), match="dtype int16")


def test_no_alloc_build_refuses_sizes_beyond_its_scratch():
    """wm_build_noalloc refuses, on the host and before any device call (no
    GPU is needed here), a build whose workspace exceeds the library's scratch
    array, and invalid arguments as wm_build does"""
    L = B.lib()
    assert L.wm_build_noalloc(0x10000, 1 << 28, 1 << 16, 4, None, 0x20000, 1 << 31, None) == B.WT_ENOSPC
    assert L.wm_build_noalloc(0x10000, 1000, 0, 4, None, 0x20000, 1 << 20, None) == B.WT_EINVAL
    assert L.wm_build_noalloc(0x10000, 1000, 100, 3, None, 0x20000, 1 << 20, None) == B.WT_EINVAL


def test_device_huffman_refuses_on_the_host():
    """wt_huffman_codes_dev checks its arguments before launching (no GPU
    needed): sigma above its one-workgroup limit, sigma 0, null pointers"""
    L = B.lib()
    p = 0x10000
    assert L.wt_huffman_codes_dev(p, 4097, p, p, p, None) == B.WT_EUNSUP
    assert L.wt_huffman_codes_dev(p, 0, p, p, p, None) == B.WT_EINVAL
    assert L.wt_huffman_codes_dev(None, 10, p, p, p, None) == B.WT_EINVAL
    assert L.wt_huffman_codes_dev(p, 10, p, p, None, None) == B.WT_EINVAL


def test_queries_refuse_batches_beyond_one_launch():
    """access / rank / select run one thread a query in one launch: a batch
    needing 2^31 workgroups or more is refused before any device call (no GPU
    needed), an empty one is a no-op, null arrays are argument errors"""
    L = B.lib()
    p, big = 0x10000, (1 << 31) * 256
    assert L.wt_access(p, p, p, big, None) == B.WT_EUNSUP
    assert L.wt_rank(p, p, p, p, big, None) == B.WT_EUNSUP
    assert L.wt_select(p, p, p, p, big, None) == B.WT_EUNSUP
    assert L.wt_access(p, None, None, 0, None) == B.WT_OK
    assert L.wt_rank(p, None, p, p, 5, None) == B.WT_EINVAL
    assert L.wt_select(None, p, p, p, 5, None) == B.WT_EINVAL


def test_chunk_geometry_near_2_to_the_32():
    """Every pass's chunks (read from the plan trace): C a multiple of the
    8192-key tile that fits 32 bits, K chunks covering n without an empty one
    -- also for one requested chunk or one huge tile count over a sequence
    within a tile of 2^32, where a single chunk would not fit 32 bits"""
    import re
    import subprocess
    import sys
    cases = [((1 << 32) - 1, "blocks=1"), ((1 << 32) - 1, "tile=1 << 20"), ((1 << 32) - 8192, "blocks=1"),
             ((1 << 32) - 8193, "blocks=1"), ((1 << 32) - 1, ""), ((1 << 32) - 1, "blocks=3"),
             ((1 << 31) + 1, "blocks=1"), (8193, "blocks=1")]
    code = "from paper_1610_03524_amd import binding as B\n" + "".join(
        f"B.plan(B.KIND_WM, {n}, 4, 1, tune=B.make_tuning({t}))\n" for n, t in cases)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       env={**os.environ, "WT_TRACE": "1"}, timeout=120)
    assert r.returncode == 0, r.stderr
    got = [(int(k), int(c)) for k, c in re.findall(r"chunks K=(\d+) of C=(\d+) keys", r.stderr)]
    assert len(got) == len(cases)
    for (n, t), (K, C) in zip(cases, got):
        assert C % 8192 == 0 and 0 < C <= (1 << 32) - 8192, (n, t, K, C)
        assert K * C >= n and (K - 1) * C < n, (n, t, K, C)


def test_trace_logs_plans_only_when_asked():
    """WT_TRACE=1 logs every plan (path, passes, chunks, level offsets) and
    batch plan on stderr; without it the library prints nothing"""
    import subprocess
    import sys
    code = ("from paper_1610_03524_amd import binding as B\n"
            "B.plan(B.KIND_WM, 1000000, 300, 2)\n"
            "d = B.wt_seq_desc(); d.S = 256; d.n = 100000; d.sigma = 1000; d.sym_bytes = 4\n"
            "d.out = 256; d.out_bytes = 1 << 30\n"
            "B.batch_plan(B.KIND_WM, [d])\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, WT_TRACE="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    lines = [l for l in r.stderr.splitlines() if l.startswith("[wt] ")]
    assert any("plan matrix n=1000000 sigma=300" in l for l in lines), r.stderr
    assert any("passes: tau=" in l and "chunks K=" in l for l in lines), r.stderr
    assert sum("  level " in l for l in lines) == 9, r.stderr
    assert any(l.startswith("[wt] batch plan: 1 sequences") for l in lines), r.stderr
    env.pop("WT_TRACE")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "[wt]" not in r.stderr


@pytest.mark.parametrize("D", [2, 3, 4])
def test_plan_of_shaped_multiary_trees(D):
    """wt_plan over codewords of D-bit digits: level sizes from the counts,
    the oracle's image size; refusals for a prefix, a codeword wider than its
    length, more than 32 bits, and a symbol of S without a codeword"""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import dary
    rng = np.random.default_rng(D)
    sigma = 300
    S = np.minimum(rng.geometric(0.02, 20000) - 1, sigma - 1).astype(np.uint16)
    counts = np.bincount(S, minlength=sigma).astype(np.uint64)
    lens = dary.huffman_lengths(counts, D)
    codes = dary.canonical(lens, D)
    info = B.plan(B.KIND_SHAPED, S.size, sigma, 2, B.make_shape(D, codes, lens, counts))
    assert info.nlevels == int(lens.max()) and info.arity_log2 == D and info.key_bits == D * int(lens.max())
    for l in range(info.nlevels):
        assert info.level_n[l] == int(counts[lens > l].sum())
    assert info.out_bytes == oracle.build_image(oracle.KIND_SHAPED, S, sigma, D, codes=codes, lens=lens).size

    def verdict(c, ln, cnt=counts):
        try:
            B.plan(B.KIND_SHAPED, int(cnt.sum()), sigma, 2, B.make_shape(D, c, ln, cnt))
            return B.WT_OK
        except B.WaveletError as e:
            return e.code
    a, b = [int(x) for x in np.flatnonzero(lens)[:2]]
    bad = codes.copy()
    bad[b] = codes[a] << np.uint64(D)   # a's codeword extended: a is a prefix of b
    ln = lens.copy()
    ln[b] = lens[a] + 1
    assert verdict(bad, ln) == B.WT_EINVAL
    wide = codes.copy()
    wide[a] |= np.uint64(1) << np.uint64(D * int(lens[a]))
    assert verdict(wide, lens) == B.WT_EINVAL
    long_ = lens.copy()
    long_[a] = 32 // D + 1
    assert verdict(codes, long_) == B.WT_EUNSUP
    none = lens.copy()
    none[int(np.flatnonzero(counts)[0])] = 0
    assert verdict(codes, none) == B.WT_ERANGE


def test_shaped_digit_trees_plan_their_path():
    """shaped trees over 2- and 4-bit digits are planned as matrix passes over
    padded codewords, split at 16 key bits when longer codewords are rare;
    3-bit digits level by level (WT_TRACE shows the plan)"""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, 'tests')\n"
            "import numpy as np, dary\n"
            "from paper_1610_03524_amd import binding as B\n"
            "for D, sigma in [(2, 4096), (4, 300), (3, 300)]:\n"
            "    rng = np.random.default_rng(7 * D + sigma)\n"
            "    S = np.minimum(rng.geometric(0.01, 200003) - 1, sigma - 1)\n"
            "    counts = np.bincount(S, minlength=sigma).astype(np.uint64)\n"
            "    lens = dary.huffman_lengths(counts, D)\n"
            "    B.plan(B.KIND_SHAPED, S.size, sigma, 2, B.make_shape(D, dary.canonical(lens, D), lens, counts))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, WT_TRACE="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    plans = [l for l in r.stderr.splitlines() if l.startswith("[wt] plan shaped")]
    assert len(plans) == 3, r.stderr
    assert "path=matrix passes" in plans[0] and "path=matrix passes" in plans[1], plans
    assert "path=level by level" in plans[2], plans
    split = [l for l in r.stderr.splitlines() if "split at 16 key bits" in l]
    assert len(split) == 1, r.stderr   # the 4-ary code of sigma 4096 is longer than 16 bits, rarely


def test_plan_reports_the_split_of_shaped_digit_trees():
    """wt_plan_info.split_bits / split_long: 16 key bits and the long-code
    symbols for a 4-ary Huffman shape whose long codewords are rare"""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import dary
    rng = np.random.default_rng(11)
    sigma = 4096
    S = np.minimum(rng.geometric(0.01, 200003) - 1, sigma - 1)
    counts = np.bincount(S, minlength=sigma).astype(np.uint64)
    lens = dary.huffman_lengths(counts, 2)
    info = B.plan(B.KIND_SHAPED, S.size, sigma, 2, B.make_shape(2, dary.canonical(lens, 2), lens, counts))
    assert info.key_bits == 2 * int(lens.max()) > 16
    assert info.split_bits == 16
    assert info.split_long == int(counts[lens > 8].sum()) > 0


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more, it says so and exits with
    status 2 before touching a device"""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for n in (2, 8):
        r = subprocess.run([sys.executable, "bench.py", "--gpus", str(n)], cwd=root, capture_output=True,
                           text=True, timeout=120)
        assert r.returncode == 2 and "one GPU only" in (r.stdout + r.stderr), (n, r.returncode, r.stdout, r.stderr)
