"""Builds from several host threads at once, each on its own stream.

The library's host state (pinned staging pool, event pool, profile records,
the per-device second stream of split shaped trees) is shared by every
caller.  Four threads build, over and over and at the same time, a wavelet
matrix, a balanced tree, a split Huffman-shaped tree (its long-code matrix
on the shared second stream) and a batch; every image must equal the
oracle's."""
import threading

import numpy as np
import pytest

import oracle
from gpu_util import shaped_codes, to_device
from paper_1610_03524_amd import binding as B

pytestmark = pytest.mark.gpu

ROUNDS = 12


def fibonacci_sequence(nsym, rng):
    """symbol s appears F(s + 1) times, shuffled: Huffman codes reach nsym - 1
    bits, and the long ones are rare (a tree split at 16 bits)"""
    f = [1, 1]
    while len(f) < nsym:
        f.append(f[-1] + f[-2])
    S = np.repeat(np.arange(nsym, dtype=np.uint8), f[:nsym])
    rng.shuffle(S)
    return S


def test_builds_from_several_threads_at_once():
    import torch
    rng = np.random.default_rng(2024)
    wm_S, wm_sigma = rng.integers(0, 1000, 300001).astype(np.uint16), 1000
    wt_S, wt_sigma = rng.integers(0, 70000, 200003).astype(np.uint32), 70000
    sh_S = fibonacci_sequence(24, rng)
    (gc, gl), (oc, ol) = shaped_codes(sh_S, 24)
    sh_counts = B.symbol_counts(to_device(sh_S), 24).cpu().numpy()
    batch = [(rng.integers(0, s, n).astype(np.uint32), s) for n, s in ((5000, 7), (90001, 300), (1, 2), (40000, 65537))]
    want = {
        "wm": oracle.build_image(oracle.KIND_WM, wm_S, wm_sigma),
        "wt": oracle.build_image(oracle.KIND_WT, wt_S, wt_sigma),
        "shaped": oracle.build_image(oracle.KIND_SHAPED, sh_S, 24, codes=oc, lens=ol),
        "batch": [oracle.build_image(oracle.KIND_WM, S, s) for S, s in batch],
    }
    plan = B.plan(B.KIND_SHAPED, sh_S.size, 24, 1, shape=B.make_shape(codes=gc, code_len=gl, counts=sh_counts))
    assert plan.split_bits, "the shaped input must take the split path (a second matrix on the shared stream)"
    got = {k: [] for k in want}
    errors = []
    start = threading.Barrier(4)

    def worker(name):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                if name == "batch":
                    dev = [to_device(S) for S, _ in batch]
                else:
                    dev = to_device({"wm": wm_S, "wt": wt_S, "shaped": sh_S}[name])
                start.wait()
                for _ in range(ROUNDS):
                    if name == "wm":
                        img, _ = B.build(B.KIND_WM, dev, wm_sigma, stream=st)
                    elif name == "wt":
                        img, _ = B.build(B.KIND_WT, dev, wt_sigma, stream=st)
                    elif name == "shaped":
                        img, _ = B.build(B.KIND_SHAPED, dev, 24, codes=gc, code_len=gl, counts=sh_counts,
                                         stream=st)
                    else:
                        descs, img = [], []
                        for t, (_, s) in zip(dev, batch):
                            info = B.plan(B.KIND_WM, t.numel(), s, 4)
                            o = torch.empty(info.out_bytes, dtype=torch.uint8, device="cuda")
                            d = B.wt_seq_desc()
                            d.S, d.n, d.sigma, d.sym_bytes = t.data_ptr(), t.numel(), s, 4
                            d.out, d.out_bytes = o.data_ptr(), info.out_bytes
                            descs.append(d)
                            img.append(o)
                        ws = torch.empty(max(B.batch_plan(B.KIND_WM, descs), 1), dtype=torch.uint8,
                                         device="cuda")
                        assert B.batch_build(B.KIND_WM, descs, ws, stream=st) == B.WT_OK
                    st.synchronize()
                    got[name].append([i.cpu().numpy() for i in img] if name == "batch" else img.cpu().numpy())
        except Exception as e:   # reported after the join
            errors.append((name, repr(e)))

    threads = [threading.Thread(target=worker, args=(k,)) for k in ("wm", "wt", "shaped", "batch")]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads), "a build thread did not finish"
    assert not errors, errors
    for name, imgs in got.items():
        assert len(imgs) == ROUNDS, name
        for r, img in enumerate(imgs):
            if name == "batch":
                for k, (g, w) in enumerate(zip(img, want[name])):
                    assert np.array_equal(g, w), f"batch round {r} sequence {k}"
            else:
                assert np.array_equal(img, want[name]), f"{name} round {r}"
