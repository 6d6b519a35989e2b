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
        for key in ("bits_off", "rank_off", "sel0_off", "sel1_off", "sub_off", "pool_off"):
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


def brute_queries(S: np.ndarray, args):
    """access / rank / select of one mixed batch answered on S itself, by the
    definitions of Sec. 2 (rank inclusive, select 1-based), in the element
    types the binding returns (access int32 view of u32, rank and select
    int64 views of u64)"""
    pos, rc, ri, sc, sk = (np.asarray(a.cpu().numpy(), dtype=np.int64) for a in args)
    n = S.size
    x = S.astype(np.int64)
    acc = np.where(pos < n, x[np.minimum(pos, max(n - 1, 0))] if n else 0, 0xFFFFFFFF)
    acc = acc.astype(np.uint32).view(np.int32)
    order = np.argsort(x, kind="stable")          # positions grouped by symbol, increasing
    key = x[order] * (n + 1) + order
    sym = x[order]

    def first(c):
        return np.searchsorted(sym, c, side="left")

    def count(c):
        return np.searchsorted(sym, c, side="right") - first(c)

    rnk = np.searchsorted(key, rc * (n + 1) + ri, side="right") - first(rc)
    rnk = np.where(ri < n, rnk, -1).astype(np.int64)
    cnt = count(sc)
    ok = (sk >= 1) & (sk <= cnt)
    sel = np.where(ok, order[np.minimum(first(sc) + sk - 1, max(n - 1, 0))] if n else 0, -1).astype(np.int64)
    return acc, rnk, sel


def build_status(kind, St, sigma, **kw):
    """status a build reports for a device sequence: the launch's return code
    when it refuses, else what wt_check reads from the image (a symbol >= sigma
    or counts that differ from the shape's are found on the device)"""
    import torch
    try:
        img, _ = B.build(kind, St, sigma, **kw)
    except B.WaveletError as e:
        torch.cuda.synchronize()
        return e.code
    return B.check(img)
