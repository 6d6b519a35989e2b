"""Prefix-free codes over D-bit digits for shaped multiary trees (test and
bench input preparation, not the method): canonical codes from lengths that
satisfy Kraft's inequality, random lengths, and d-ary Huffman lengths."""
import heapq

import numpy as np


def canonical(lens: np.ndarray, D: int) -> np.ndarray:
    """canonical codewords for digit lengths (0 = no codeword): in (length,
    symbol) order, each code is the previous one plus one, shifted by the
    digits its length adds"""
    d = 1 << D
    order = sorted((int(l), s) for s, l in enumerate(lens) if l)
    codes = np.zeros(len(lens), dtype=np.uint64)
    code, prev = 0, None
    for l, s in order:
        if prev is not None:
            code = (code + 1) * d ** (l - prev)
        assert code < d ** l, "lengths violate Kraft's inequality"
        codes[s] = code
        prev = l
    return codes


def random_lengths(sigma: int, D: int, rng, present=None, max_bits: int = 32) -> np.ndarray:
    """random digit lengths with sum d^-len <= 1: every symbol (or those in
    `present`) gets ceil(log_d k) digits, then random symbols get longer"""
    d = 1 << D
    syms = list(range(sigma)) if present is None else sorted(present)
    k = len(syms)
    base = 1
    while d ** base < k:
        base += 1
    lens = np.zeros(sigma, dtype=np.uint32)
    lens[syms] = base
    cap = max_bits // D
    for s in rng.choice(syms, size=min(k, 1 + k // 2), replace=False):
        lens[s] = min(cap, base + int(rng.integers(0, 4)))
    return lens


def huffman_lengths(counts: np.ndarray, D: int) -> np.ndarray:
    """d-ary Huffman code lengths (in digits): zero-weight dummies make the
    leaf count 1 mod (d-1), then the d lightest subtrees merge, ties by order
    of creation; absent symbols get length 0, a single present one length 1"""
    d = 1 << D
    present = [s for s in range(len(counts)) if counts[s]]
    lens = np.zeros(len(counts), dtype=np.uint32)
    if len(present) == 1:
        lens[present[0]] = 1
        return lens
    heap = [(int(counts[s]), t, [s]) for t, s in enumerate(present)]
    t = len(heap)
    while (len(heap) - 1) % (d - 1):
        heap.append((0, t, []))
        t += 1
    heapq.heapify(heap)
    while len(heap) > 1:
        w, members = 0, []
        for _ in range(min(d, len(heap))):
            a, _, m = heapq.heappop(heap)
            w += a
            members += m
        for s in members:
            lens[s] += 1
        heapq.heappush(heap, (w, t, members))
        t += 1
    return lens
