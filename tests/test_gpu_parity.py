"""GPU parity: every image the HIP library builds equals the oracle's image
byte for byte (integer work, tolerance 0), over sizes that span many tiles
and ragged tails, edge alphabets and degenerate sequences."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same, gpu_image, oracle_image, shaped_codes, to_device
from paper_1610_03524_amd import binding as B

pytestmark = pytest.mark.gpu

EDGE_N = [0, 1, 63, 64, 65, 511, 512, 513, 4095, 4096, 4097, 70001]
SIGMAS = [1, 2, 3, 4, 5, 8, 255, 256, 257, 4096, 65536, 65537, 1 << 20]


def dtype_for(sigma):
    return np.uint8 if sigma <= 256 else (np.uint16 if sigma <= 65536 else np.uint32)


def patterns(n, sigma, rng):
    dt = dtype_for(sigma)
    yield "uniform", rng.integers(0, sigma, n).astype(dt)
    if n > 1:
        yield "equal", np.full(n, sigma - 1, dtype=dt)
        yield "sorted", np.sort(rng.integers(0, sigma, n)).astype(dt)
        yield "reverse", np.sort(rng.integers(0, sigma, n))[::-1].astype(dt).copy()
        yield "alternating", (np.arange(n) % min(sigma, 2) * (sigma - 1)).astype(dt)
        rare = np.zeros(n, dtype=dt)
        rare[n // 2] = sigma - 1
        yield "one_rare", rare


shaped_inputs = shaped_codes


@pytest.mark.parametrize("kind", [B.KIND_WM, B.KIND_WT])
@pytest.mark.parametrize("sigma", SIGMAS)
def test_binary_parity(kind, sigma):
    rng = np.random.default_rng(sigma * 7 + kind)
    for n in EDGE_N:
        for name, S in patterns(n, sigma, rng):
            g = gpu_image(kind, S, sigma)
            o = oracle_image(kind, S, sigma)
            assert_same(g, o, f"kind={kind} sigma={sigma} n={n} {name}")


@pytest.mark.parametrize("D", [1, 2, 3, 4])
@pytest.mark.parametrize("sigma", [2, 5, 16, 17, 256, 4096, 65536])
def test_multiary_parity(D, sigma):
    rng = np.random.default_rng(1000 + D * sigma)
    for n in [0, 1, 31, 32, 33, 2047, 2048, 2049, 70001]:
        for name, S in patterns(n, sigma, rng):
            g = gpu_image(B.KIND_MULTIARY, S, sigma, D)
            o = oracle_image(B.KIND_MULTIARY, S, sigma, D)
            assert_same(g, o, f"D={D} sigma={sigma} n={n} {name}")


@pytest.mark.parametrize("sigma", [2, 3, 100, 4096])
def test_shaped_parity(sigma):
    rng = np.random.default_rng(77 + sigma)
    for n in [1, 2, 64, 513, 4097, 70001]:
        for p in (0.5, 0.05, 0.005):
            S = np.minimum(rng.geometric(p, n) - 1, sigma - 1).astype(dtype_for(sigma))
            (gc, gl), (oc, ol) = shaped_inputs(S, sigma)
            g = gpu_image(B.KIND_SHAPED, S, sigma, codes=gc, lens=gl)
            o = oracle_image(B.KIND_SHAPED, S, sigma, codes=oc, lens=ol)
            assert_same(g, o, f"shaped sigma={sigma} n={n} p={p}")


@pytest.mark.parametrize("kind", [B.KIND_WM, B.KIND_WT])
def test_levelwise_equals_default(kind):
    rng = np.random.default_rng(5)
    S = rng.integers(0, 1000, 200003).astype(np.uint16)
    a = gpu_image(kind, S, 1000)
    b = gpu_image(kind, S, 1000, tune=B.make_tuning(flags=B.FLAG_LEVELWISE))
    assert_same(a, b, "levelwise vs default")


def test_symbol_out_of_range_sets_status():
    """a symbol >= sigma is found on the device: every stream-ordered build
    returns WT_OK and wt_check reports WT_ERANGE; the level-by-level tree path,
    which reads the counts back, returns it directly"""
    import torch
    S = to_device(np.array([0, 1, 7, 2], dtype=np.uint8))
    for kind, D in ((B.KIND_WM, 0), (B.KIND_WT, 0), (B.KIND_MULTIARY, 2), (B.KIND_MULTIARY, 1)):
        img, _ = B.build(kind, S, 5, arity_log2=D)
        assert B.check(img) == B.WT_ERANGE, (kind, D)
    with pytest.raises(B.WaveletError) as e:
        B.build(B.KIND_MULTIARY, S, 5, arity_log2=3)
    assert e.value.code == B.WT_ERANGE
    torch.cuda.synchronize()


def test_shaped_counts_that_differ_from_the_shape_are_reported():
    """the shape's counts fix the level sizes; a sequence whose counts differ
    is found on the device and wt_check returns WT_EINVAL (the image is then
    unspecified, but the build stays in bounds)"""
    import torch
    rng = np.random.default_rng(8)
    S = rng.integers(0, 40, 5000).astype(np.uint8)
    counts = oracle.symbol_counts(S, 40)
    codes, lens = oracle.huffman(counts)
    T = S.copy()
    T[17] = (T[17] + 1) % 40               # same length, one count moved
    img, _ = B.build(B.KIND_SHAPED, to_device(T), 40, codes=codes, code_len=lens, counts=counts)
    assert B.check(img) == B.WT_EINVAL
    img, _ = B.build(B.KIND_SHAPED, to_device(S), 40, codes=codes, code_len=lens, counts=counts)
    assert B.check(img) == B.WT_OK
    assert_same(img.cpu().numpy(), oracle.build_image(oracle.KIND_SHAPED, S, 40, codes=codes, lens=lens), "shaped")
    torch.cuda.synchronize()


def test_buffer_too_small():
    import torch
    S = to_device(np.arange(100, dtype=np.uint8))
    info = B.plan(B.KIND_WM, 100, 100, 1)
    out = torch.empty(info.out_bytes - 1, dtype=torch.uint8, device="cuda")
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device="cuda")
    assert B.build_into(B.KIND_WM, S, 100, out, ws) == B.WT_ENOSPC
    out = torch.empty(info.out_bytes, dtype=torch.uint8, device="cuda")
    ws = torch.empty(info.workspace_bytes - 1, dtype=torch.uint8, device="cuda")
    assert B.build_into(B.KIND_WM, S, 100, out, ws) == B.WT_ENOSPC


@pytest.mark.parametrize("tau", [0, 1, 2, 3, 5, 7, 8])
@pytest.mark.parametrize("blocks", [0, 1, 3, 7])
def test_wm_passes_any_tau_and_chunking(tau, blocks):
    """the matrix does not depend on the pass width or on how the sequence is
    cut into chunks and tiles (many tiles per chunk, ragged last tile)"""
    from paper_1610_03524_amd import inputs
    S = inputs.c2_zipf(n=(1 << 18) + 4097, sigma=1 << 16, seed=11)
    o = oracle_image(B.KIND_WM, S, 1 << 16)
    g = gpu_image(B.KIND_WM, S, 1 << 16, tune=B.make_tuning(tau=tau, blocks=blocks))
    assert_same(g, o, f"tau={tau} blocks={blocks}")


@pytest.mark.parametrize("sigma,dt", [(256, np.uint8), (5, np.uint8), (1 << 20, np.uint32), (3000, np.uint16)])
def test_wm_passes_widths(sigma, dt):
    rng = np.random.default_rng(sigma)
    S = rng.integers(0, sigma, 300001).astype(dt)
    o = oracle_image(B.KIND_WM, S, sigma)
    for blocks in (0, 2):
        g = gpu_image(B.KIND_WM, S, sigma, tune=B.make_tuning(blocks=blocks))
        assert_same(g, o, f"sigma={sigma} blocks={blocks}")
    # narrow passes: byte keys in LDS with remaining bits written for the
    # next pass, from symbols of every width
    for tau in (2, 3):
        g = gpu_image(B.KIND_WM, S, sigma, tune=B.make_tuning(tau=tau))
        assert_same(g, o, f"sigma={sigma} tau={tau}")


def fibonacci_sequence(nsym, rng):
    """symbol s appears F(s + 1) times (F(1) = F(2) = 1), shuffled: its
    Huffman tree is a path, so the codes reach nsym - 1 bits"""
    f = [1, 1]
    while len(f) < nsym:
        f.append(f[-1] + f[-2])
    S = np.repeat(np.arange(nsym, dtype=np.uint8), f[:nsym])
    rng.shuffle(S)
    return S


@pytest.mark.parametrize("nsym", [20, 30, 32, 33])
def test_shaped_long_codes(nsym):
    """code lengths up to 31 bits (gathered from matrix levels over padded
    codes, most runs of the deep levels being leaves) and 32 bits (the
    one-level-per-pass builder)"""
    S = fibonacci_sequence(nsym, np.random.default_rng(nsym))
    (gc, gl), (oc, ol) = shaped_inputs(S, nsym)
    assert int(gl.max()) == nsym - 1
    g = gpu_image(B.KIND_SHAPED, S, nsym, codes=gc, lens=gl)
    o = oracle_image(B.KIND_SHAPED, S, nsym, codes=oc, lens=ol)
    assert_same(g, o, f"shaped fibonacci nsym={nsym}")


@pytest.mark.parametrize("kind", [B.KIND_WT, B.KIND_SHAPED])
def test_trees_many_chunks(kind):
    """7M symbols, 17 key bits: three passes, every chunk two tiles long"""
    rng = np.random.default_rng(17)
    sigma, n = 65537, 7_000_003
    if kind == B.KIND_WT:
        S = rng.integers(0, sigma, n).astype(np.uint32)
        g = gpu_image(kind, S, sigma)
        o = oracle_image(kind, S, sigma)
    else:
        S = np.minimum(rng.geometric(0.0005, n) - 1, sigma - 1).astype(np.uint32)
        (gc, gl), (oc, ol) = shaped_inputs(S, sigma)
        g = gpu_image(kind, S, sigma, codes=gc, lens=gl)
        o = oracle_image(kind, S, sigma, codes=oc, lens=ol)
    assert_same(g, o, f"kind={kind} n={n}")


def split_case(counts, long_len, rng):
    """a shuffled sequence over four symbols with codes 0, 10, 110 0..0 and
    111 1..1 (the last two long_len bits long)"""
    codes = np.array([0, 0b10, 0b110 << (long_len - 3), (1 << long_len) - 1], dtype=np.uint64)
    lens = np.array([1, 2, long_len, long_len], dtype=np.uint32)
    S = np.repeat(np.arange(4, dtype=np.uint8), counts)
    rng.shuffle(S)
    return S, codes, lens


@pytest.mark.parametrize("name,counts", [
    ("split, few long", [70001, 30000, 5, 3]),       # deep levels from the small second matrix
    ("split, no long", [50000, 20001, 0, 0]),        # long codes that never occur
    ("no split, many long", [4000, 3000, 2500, 1501]),
    ("two symbols", [1, 0, 1, 0]),                   # too few for a split
])
@pytest.mark.parametrize("long_len", [17, 20, 31])
@pytest.mark.parametrize("dt", [np.uint8, np.uint16, np.uint32])
def test_shaped_split_at_16_bits(name, counts, long_len, dt):
    """shaped trees deeper than 16 levels: levels above 16 from a matrix over
    16-bit key prefixes of every symbol, the deeper ones from a matrix over the
    long-code symbols alone (when they are at most 1/8 of the sequence); every
    symbol width (16-byte loads of 16, 8 or 4 symbols, ragged last block)"""
    S, codes, lens = split_case(counts, long_len, np.random.default_rng(long_len + sum(counts)))
    S = S.astype(dt)
    o = oracle_image(B.KIND_SHAPED, S, 4, codes=codes, lens=lens)
    for tune in (None, B.make_tuning(tau=3, blocks=2)):
        g = gpu_image(B.KIND_SHAPED, S, 4, codes=codes, lens=lens, tune=tune)
        assert_same(g, o, f"{name} long_len={long_len} tune={tune is not None}")


DD_CASES = [(1, 1, 0), (2, 1000, 0), (3, 8191, 3), (5, 8192, 7), (8, 8193, 2), (17, 65537, 5), (100, 300001, 40),
            (255, 1 << 20, 128), (256, (1 << 20) + 12345, 0), (256, 5 * 8192 * 3 + 1, 15), (7, 3 * 8192, 3)]


@pytest.mark.parametrize("sigma,n,blocks", DD_CASES)
def test_balanced_tree_by_domain_decomposition(sigma, n, blocks):
    """Balanced trees over at most 8 key bits are built in one pass straight
    into tree order (Sec. 4.2): the K chunks of the pass are built alone and
    their runs of every node placed by prefix sums over the per-chunk counts,
    the words shared by two chunks OR-ed.  Every chunk count (blocks = 0:
    automatic) gives the oracle's image, and so does the matrix-and-gather
    path forced with a narrower pass."""
    import torch
    rng = np.random.default_rng(sigma * 7919 + n)
    S = rng.integers(0, sigma, n).astype(np.uint8 if sigma <= 256 else np.uint16)
    want = oracle_image(B.KIND_WT, S, sigma)
    tune = B.make_tuning(blocks=blocks)
    info = B.plan(B.KIND_WT, n, sigma, S.itemsize, tune=tune)
    L = max(1, (sigma - 1).bit_length())
    assert info.tau == L   # one pass covers every level
    assert_same(gpu_image(B.KIND_WT, S, sigma, tune=tune), want, f"direct sigma={sigma} n={n} blocks={blocks}")
    if L >= 3:
        narrow = B.make_tuning(tau=L - 1, blocks=blocks)
        assert B.plan(B.KIND_WT, n, sigma, S.itemsize, tune=narrow).tau == L - 1
        assert_same(gpu_image(B.KIND_WT, S, sigma, tune=narrow), want, f"matrix path sigma={sigma} n={n}")
    torch.cuda.synchronize()
