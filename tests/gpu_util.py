"""Helpers of the GPU tests: run a build through the C-ABI binding and
compare its image with the oracle's byte by byte."""
from __future__ import annotations

import numpy as np

import oracle
from imagewalk import Image
from paper_1610_03524_amd import binding as B

DEV = "cuda"


def to_device(S: np.ndarray):
    import torch
    view = {np.uint8: np.uint8, np.uint16: np.int16, np.uint32: np.int32}[S.dtype.type]
    return torch.from_numpy(np.ascontiguousarray(S).view(view)).to(DEV)


def gpu_image(kind, S: np.ndarray, sigma: int, D: int = 0, tune=None, codes=None, lens=None) -> np.ndarray:
    import torch
    St = to_device(S)
    counts = None
    if kind == B.KIND_SHAPED:
        counts = oracle_free_counts(St, sigma)
    img, _ = B.build(kind, St, sigma, arity_log2=D, codes=codes, code_len=lens, counts=counts, tune=tune)
    torch.cuda.synchronize()
    assert B.check(img) == B.WT_OK
    return img.cpu().numpy()


def oracle_free_counts(St, sigma):
    """symbol counts from the library (device histogram)"""
    return B.symbol_counts(St, sigma).cpu().numpy().astype(np.uint64)


def oracle_image(kind, S, sigma, D=0, codes=None, lens=None) -> np.ndarray:
    return oracle.build_image(kind, S, sigma, max(D, 1), codes=codes, lens=lens)


def describe_diff(a: np.ndarray, b: np.ndarray) -> str:
    """where two images first differ (level and array), for failure messages"""
    if a.size != b.size:
        return f"sizes differ: {a.size} vs {b.size}"
    idx = np.flatnonzero(a != b)
    if idx.size == 0:
        return "equal"
    off = int(idx[0])
    img = Image(b)
    where = "header"
    for l, lv in enumerate(img.levels):
        for key in ("bits_off", "rank_off", "sel0_off", "sel1_off"):
            if lv[key] and lv[key] <= off:
                where = f"level {l} {key[:-4]} (+{off - lv[key]})"
    if img.nodes_off and off >= img.nodes_off:
        where = "nodes" if off < img.codes_off else "codes"
    return f"{idx.size} bytes differ, first at {off}: {where}; gpu={a[off]} oracle={b[off]}"


def assert_same(gpu: np.ndarray, ora: np.ndarray, what=""):
    assert gpu.size == ora.size and np.array_equal(gpu, ora), f"{what}: {describe_diff(gpu, ora)}"


def shaped_codes(S, sigma):
    """codewords for the GPU build from the library (device counts + host
    Huffman), and for the oracle from the oracle's own counts and Huffman."""
    counts = B.symbol_counts(to_device(S), sigma).cpu().numpy().astype(np.uint64)
    gcodes, glens = B.huffman_codes(counts)
    ocodes, olens = oracle.huffman(oracle.symbol_counts(S, sigma))
    return (gcodes, glens), (ocodes, olens)
