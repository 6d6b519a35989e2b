"""Parity at the full sizes of the benchmark configurations, in the launch
configuration bench.py times (default tuning; the tuned pass width for the
batch).  Where the oracle finishes in seconds (C1, C3, sampled C4 sequences)
the images are compared with the oracle's byte for byte; the 2^28-symbol
matrix (C2) is compared array by array with digests of the oracle's image,
computed once by a committed script that runs the oracle alone."""
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
    """C2: 2^28 uint32 Zipf symbols, sigma 2^16, in the launch configuration
    the benchmark times.  The whole image is compared with the oracle's
    through SHA-256 digests of every array (tests/golden/c2_image.json,
    written by tests/golden/make_c2_image.py from the oracle alone); the input
    drawn on the device is first checked against the digest of the host
    draw the oracle built from."""
    import hashlib
    import json
    import os
    import torch
    from imagewalk import array_digests
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_image.json")) as f:
        golden = json.load(f)
    n, sigma = golden["n"], golden["sigma"]
    S = inputs.c2_zipf(n=n, sigma=sigma, seed=golden["seed"], device="cuda")
    Sh = S.cpu().numpy().view(np.uint32)
    assert hashlib.sha256(Sh.tobytes()).hexdigest() == golden["input_sha256"], "device draw differs from the host draw"
    info = B.plan(B.KIND_WM, n, sigma, 4)
    assert info.out_bytes == golden["image_bytes"]
    out = torch.empty(info.out_bytes, dtype=torch.uint8, device="cuda")
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device="cuda")
    assert B.build_into(B.KIND_WM, S, sigma, out, ws) == B.WT_OK
    torch.cuda.synchronize()
    assert B.check(out) == B.WT_OK
    img = out.cpu().numpy()
    del out, ws
    got = array_digests(img)
    want = golden["digests"]
    assert list(got) == list(want)
    bad = [k for k in want if k != "image" and got[k] != want[k]]
    assert not bad, f"{len(bad)} arrays differ from the oracle's, first: {bad[0]}"
    assert got["image"] == want["image"]
    # a few queries walked through the image against S itself
    walk = MatrixWalk(img, info.nlevels)
    rng = np.random.default_rng(28)
    for i in rng.integers(0, n, 64):
        assert walk.access(int(i)) == int(Sh[i]), f"access({i})"


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
