"""Builds are stream-ordered: a wavelet-matrix build is kernel launches
only, tree builds add no host wait (runs derived on the device, or a shaped
tree's tables from its shape, uploaded from pinned buffers), and a batched
build returns without waiting.  So a caller can capture any of them into a
HIP graph and replay it.  Every replay must write the oracle's image, after
eager work has overwritten the images and the workspace in between."""
import numpy as np
import pytest

import dary
from gpu_util import assert_same, oracle_image, to_device
from paper_1610_03524_amd import binding as B

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,sigma,dt", [((1 << 18) + 4097, 1 << 16, np.uint32), (300001, 256, np.uint8),
                                        ((1 << 20) + 3, 1000, np.uint16)])
def test_wm_build_replayed_from_a_graph(n, sigma, dt):
    import torch
    rng = np.random.default_rng(n + sigma)
    S = rng.integers(0, sigma, n).astype(dt)
    St = to_device(S)
    info = B.plan(B.KIND_WM, n, sigma, S.itemsize)
    out = torch.empty(info.out_bytes, dtype=torch.uint8, device="cuda")
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device="cuda")
    assert B.build_into(B.KIND_WM, St, sigma, out, ws) == B.WT_OK
    torch.cuda.synchronize()
    eager = out.cpu().numpy()
    assert_same(eager, oracle_image(B.KIND_WM, S, sigma), f"eager n={n} sigma={sigma}")

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rc = B.build_into(B.KIND_WM, St, sigma, out, ws, stream=s)
    assert rc == B.WT_OK
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(0xA5)        # eager work between replays over the image and the workspace
        ws.fill_(0x5A + rep)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), f"replay {rep}: n={n} sigma={sigma}"
        assert B.check(out) == B.WT_OK


def _replay_checks(g, outs, ws, wants, what):
    """replay a captured build three times, eager work overwriting every image
    and the workspace in between; every replay equals the oracle"""
    import torch
    for rep in range(3):
        for o in outs:
            o.fill_(0xA5)
        ws.fill_(0x5A + rep)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, (o, w) in enumerate(zip(outs, wants)):
            assert_same(o.cpu().numpy(), w, f"{what} replay {rep} image {k}")
            assert B.check(o) == B.WT_OK


TREE_CASES = [
    ("balanced u8", B.KIND_WT, 0, 300001, 256, np.uint8),
    ("balanced u16", B.KIND_WT, 0, (1 << 19) + 77, 3000, np.uint16),
    ("binary multiary", B.KIND_MULTIARY, 1, 200003, 700, np.uint16),
    ("4-ary", B.KIND_MULTIARY, 2, (1 << 19) + 5, 4096, np.uint16),
    ("16-ary", B.KIND_MULTIARY, 4, 100001, 70000, np.uint32),
    ("huffman", B.KIND_SHAPED, 0, 400009, 4096, np.uint16),
    ("huffman, levels of 2^20 bits", B.KIND_SHAPED, 0, (1 << 21) + 9, 4096, np.uint16),
    ("4-ary huffman", B.KIND_SHAPED, 2, 400009, 4096, np.uint16),
    ("16-ary huffman", B.KIND_SHAPED, 4, 300007, 70000, np.uint32),
]


@pytest.mark.parametrize("name,kind,D,n,sigma,dt", TREE_CASES, ids=[c[0] for c in TREE_CASES])
def test_tree_build_replayed_from_a_graph(name, kind, D, n, sigma, dt):
    """tree builds are stream-ordered too (balanced and multiary trees derive
    their runs on the device; a shaped tree's tables come from its shape), so
    wt_build and multiary_build can be captured and replayed"""
    import torch
    import oracle
    rng = np.random.default_rng(n ^ sigma)
    if kind == B.KIND_SHAPED:
        S = np.minimum(rng.geometric(0.01, n) - 1, sigma - 1).astype(dt)
    else:
        S = rng.integers(0, sigma, n).astype(dt)
    St = to_device(S)
    codes = lens = counts = None
    if kind == B.KIND_SHAPED:
        counts = oracle.symbol_counts(S, sigma)
        if D >= 2:   # d-ary Huffman codewords over D-bit digits
            lens = dary.huffman_lengths(counts, D)
            codes = dary.canonical(lens, D)
        else:
            codes, lens = B.huffman_codes(counts)
        want = oracle.build_image(oracle.KIND_SHAPED, S, sigma, max(D, 1), codes=codes, lens=lens)
    else:
        want = oracle_image(kind, S, sigma, D)
    shape = B.make_shape(D, codes, lens, counts) if (D or codes is not None) else None
    info = B.plan(kind, n, sigma, S.itemsize, shape)
    out = torch.empty(info.out_bytes, dtype=torch.uint8, device="cuda")
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device="cuda")
    assert B.build_into(kind, St, sigma, out, ws, shape) == B.WT_OK
    torch.cuda.synchronize()
    assert_same(out.cpu().numpy(), want, f"eager {name}")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        rc = B.build_into(kind, St, sigma, out, ws, shape, stream=s)
    assert rc == B.WT_OK
    torch.cuda.synchronize()
    _replay_checks(g, [out], ws, [want], name)


def test_batch_build_replayed_from_a_graph():
    """a batched build returns without waiting (its staged descriptors retire
    with the stream; under capture they are kept for the graph), so it can be
    captured and replayed"""
    import torch
    rng = np.random.default_rng(2024)
    seqs = []
    for k in range(24):
        n = int(2 ** rng.uniform(4, 17))
        sigma = max(2, int(2 ** rng.uniform(1, 20)))
        seqs.append((rng.integers(0, sigma, n).astype(np.uint32), sigma))
    dev = [to_device(S) for S, _ in seqs]
    outs = [torch.empty(B.plan(B.KIND_WM, S.size, sg, 4).out_bytes, dtype=torch.uint8, device="cuda")
            for S, sg in seqs]
    descs = [B.make_desc(St, sg, o) for St, (_, sg), o in zip(dev, seqs, outs)]
    ws = torch.empty(max(B.batch_plan(B.KIND_WM, descs), 1), dtype=torch.uint8, device="cuda")
    wants = [oracle_image(B.KIND_WM, S, sg) for S, sg in seqs]
    assert B.batch_build(B.KIND_WM, descs, ws) == B.WT_OK
    torch.cuda.synchronize()
    for k, (o, w) in enumerate(zip(outs, wants)):
        assert_same(o.cpu().numpy(), w, f"eager batch image {k}")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        rc = B.batch_build(B.KIND_WM, descs, ws, stream=s)
    assert rc == B.WT_OK
    torch.cuda.synchronize()
    _replay_checks(g, outs, ws, wants, "batch")
