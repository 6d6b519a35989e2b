"""Test-side reader of canonical wavelet images, with query walkers.

This module is part of the test suite only.  It decodes an image (the byte
layout the oracle and the GPU library both emit), and answers access / rank /
select by walking the levels the way the queries on these structures are
defined (the pointerless traversals that Sec. 2 says replace the topology
pointers).  Tests compare these walks with brute force on S, which pins the
*meaning* of an image independently of how it was built.
"""
from __future__ import annotations

import numpy as np

MAGIC = 0x54564157
KIND_WT, KIND_WM, KIND_SHAPED, KIND_MULTI = 1, 2, 3, 4
LEAF = 0x80000000
NO_CHILD = 0xFFFFFFFF


def _u64(buf, off, count=1):
    return np.frombuffer(buf[off:off + 8 * count].tobytes(), dtype=np.uint64)


class Image:
    def __init__(self, buf: np.ndarray):
        self.buf = np.asarray(buf, dtype=np.uint8)
        b = self.buf
        h32 = np.frombuffer(b[:40].tobytes(), dtype=np.uint32)
        self.magic, self.version, self.kind, self.arity_log2 = (int(v) for v in h32[:4])
        self.n = int(_u64(b, 16)[0])
        self.sigma = int(h32[6])
        self.nlevels = int(h32[7])
        self.key_bits = int(h32[8])
        self.status = int(h32[9])
        self.image_bytes = int(_u64(b, 40)[0])
        self.levels_off = int(_u64(b, 48)[0])
        self.nodes_off = int(_u64(b, 56)[0])
        self.nnodes = int(_u64(b, 64)[0])
        self.codes_off = int(_u64(b, 72)[0])
        self.ncoded = int(_u64(b, 80)[0])
        # digit levels: multiary trees, and shaped trees of D-bit digits
        self.multi_levels = self.kind == 4 or (self.kind == 3 and self.arity_log2 >= 2)
        self.levels = []
        for l in range(self.nlevels):
            e = _u64(b, self.levels_off + 64 * l, 8)
            lv = dict(n=int(e[0]), zeros=int(e[1]), ones=int(e[2]), bits_off=int(e[3]), rank_off=int(e[4]),
                      sel0_off=int(e[5]), sel1_off=int(e[6]), nsel=int(e[7]), sub_off=0, nsub=0,
                      pool_off=0, nslot=0)
            if not self.multi_levels:
                # binary: the select sub-samples follow sel1, the pool of
                # stored answers follows them (neither is in the record)
                lv["sub_off"] = (lv["sel1_off"] + 8 * lv["nsel"] + 255) // 256 * 256
                lv["nsub"] = -(-lv["n"] // 512) + 2
                lv["pool_off"] = (lv["sub_off"] + 4 * lv["nsub"] + 255) // 256 * 256
                lv["nslot"] = lv["n"] >> 20
            self.levels.append(lv)
        self._bits = {}
        self._zpre = {}

    # ---- binary levels ---------------------------------------------------
    def words(self, l: int) -> np.ndarray:
        lv = self.levels[l]
        nw = (lv["n"] + 63) // 64
        return _u64(self.buf, lv["bits_off"], nw)

    def bits(self, l: int) -> np.ndarray:
        if l not in self._bits:
            lv = self.levels[l]
            raw = self.buf[lv["bits_off"]:lv["bits_off"] + (lv["n"] + 7) // 8]
            self._bits[l] = np.unpackbits(raw, bitorder="little")[:lv["n"]]
        return self._bits[l]

    def _zeros_prefix(self, l: int) -> np.ndarray:
        if l not in self._zpre:
            z = np.zeros(self.levels[l]["n"] + 1, dtype=np.int64)
            z[1:] = np.cumsum(self.bits(l) == 0)
            self._zpre[l] = z
        return self._zpre[l]

    def rank_dir(self, l: int) -> np.ndarray:
        lv = self.levels[l]
        ns = (lv["n"] + 511) // 512
        return _u64(self.buf, lv["rank_off"], 2 * (ns + 1)).reshape(ns + 1, 2)

    def sel(self, l: int, which: int) -> np.ndarray:
        lv = self.levels[l]
        off = lv["sel1_off"] if which else lv["sel0_off"]
        return _u64(self.buf, off, lv["nsel"])

    def sub(self, l: int) -> np.ndarray:
        """select sub-samples: ones' positions of ordinal 512j at j, zeros'
        at nsub-1-j, unused entries n"""
        lv = self.levels[l]
        return np.frombuffer(self.buf[lv["sub_off"]:lv["sub_off"] + 4 * lv["nsub"]].tobytes(), dtype=np.uint32)

    def pool(self, l: int) -> np.ndarray:
        """stored answers of the long sub-ranges: 2 * nslot slots of 512
        positions, the ones' slots first"""
        lv = self.levels[l]
        size = 4 * 2 * lv["nslot"] * 512
        return np.frombuffer(self.buf[lv["pool_off"]:lv["pool_off"] + size].tobytes(), dtype=np.uint32)

    def rank0_via_directory(self, l: int, i: int) -> int:
        """zeros in [0, i) using only the directory and one word."""
        d = self.rank_dir(l)
        k, q = divmod(i, 512)
        r = int(d[k, 0])
        if q >= 64:
            r += (int(d[k, 1]) >> (9 * (q // 64 - 1))) & 511
        t = q % 64
        if t:
            w = int(self.words(l)[i // 64])
            r += t - bin(w & ((1 << t) - 1)).count("1")
        return r

    def rank(self, l: int, b: int, i: int) -> int:
        """number of b-bits in [0, i) on binary level l"""
        z = int(self._zeros_prefix(l)[i])
        return z if b == 0 else i - z

    def select(self, l: int, b: int, j: int) -> int:
        """position of the b-bit with 0-based ordinal j on level l"""
        pos = np.flatnonzero(self.bits(l) == b)
        return int(pos[j])

    # ---- multiary levels ---------------------------------------------------
    def digits(self, l: int) -> np.ndarray:
        D = self.arity_log2
        p = 64 // D
        lv = self.levels[l]
        nw = (lv["n"] + p - 1) // p
        w = _u64(self.buf, lv["bits_off"], nw)
        t = np.arange(lv["n"], dtype=np.uint64)
        return ((w[t // p] >> (np.uint64(D) * (t % p))) & np.uint64((1 << D) - 1)).astype(np.int64)

    def digit_counters(self, l: int):
        D = self.arity_log2
        p, d = 64 // D, 1 << D
        m = self.levels[l]["n"]
        sbd, bd = 64 * p, 8 * p
        nsb, nb = -(-m // sbd), -(-m // bd)
        off = self.levels[l]["rank_off"]
        sb = _u64(self.buf, off, (nsb + 1) * d).reshape(nsb + 1, d)
        o2 = off + (nsb + 1) * d * 8
        blk = np.frombuffer(self.buf[o2:o2 + nb * d * 2].tobytes(), dtype=np.uint16).reshape(nb, d)
        return sb, blk

    def mrank(self, l: int, c: int, i: int) -> int:
        return int(np.count_nonzero(self.digits(l)[:i] == c))

    # ---- shaped trees ------------------------------------------------------
    def nodes(self):
        """node records: binary {u64 start, u64 count, u32 child[2], u32 level,
        u32 prefix}; D-bit digits {u64 start, u64 count, u32 level, u32 prefix,
        u32 child[2^D]}"""
        if getattr(self, "_nodes", None) is not None:
            return self._nodes
        out = []
        D = self.arity_log2 if self.multi_levels else 1
        d = 1 << D
        rb = 32 if D == 1 else 24 + 4 * d
        for t in range(self.nnodes):
            o = self.nodes_off + rb * t
            st, cnt = (int(v) for v in _u64(self.buf, o, 2))
            w = [int(v) for v in np.frombuffer(self.buf[o + 16:o + rb].tobytes(), dtype=np.uint32)]
            if D == 1:
                out.append(dict(start=st, count=cnt, child=(w[0], w[1]), level=w[2], prefix=w[3]))
            else:
                out.append(dict(start=st, count=cnt, child=tuple(w[2:2 + d]), level=w[0], prefix=w[1]))
        self._nodes = out
        return out

    # ---- levels of either form (bits, or D-bit digits) ---------------------
    def sym_at(self, l: int, p: int) -> int:
        return int(self.digits(l)[p]) if self.multi_levels else int(self.bits(l)[p])

    def rank_any(self, l: int, g: int, i: int) -> int:
        """occurrences of bit / digit g in [0, i) of level l"""
        return self.mrank(l, g, i) if self.multi_levels else self.rank(l, g, i)

    def select_any(self, l: int, g: int, j: int) -> int:
        if self.multi_levels:
            return int(np.flatnonzero(self.digits(l) == g)[j])
        return self.select(l, g, j)

    def code_digit(self, c: int, t: int) -> int:
        """digit t (from the top) of c's codeword"""
        codes, lens = self.codes()
        D = self.arity_log2 if self.multi_levels else 1
        return int((int(codes[c]) >> (D * (int(lens[c]) - 1 - t))) & ((1 << D) - 1))

    def codes(self):
        if getattr(self, "_codes", None) is not None:
            return self._codes
        c = np.zeros(self.sigma, dtype=np.uint64)
        ln = np.zeros(self.sigma, dtype=np.uint32)
        for s in range(self.sigma):
            o = self.codes_off + 16 * s
            c[s] = _u64(self.buf, o)[0]
            ln[s] = np.frombuffer(self.buf[o + 8:o + 12].tobytes(), dtype=np.uint32)[0]
        self._codes = (c, ln)
        return self._codes

    # ---- queries -----------------------------------------------------------
    def access(self, i: int) -> int:
        if self.kind == KIND_WM:
            x = 0
            for l in range(self.nlevels):
                b = int(self.bits(l)[i])
                x = (x << 1) | b
                i = self.rank(l, b, i) + (self.levels[l]["zeros"] if b else 0)
            return x
        if self.kind == KIND_WT:
            s, e, x = 0, self.n, 0
            for l in range(self.nlevels):
                b = int(self.bits(l)[i])
                x = (x << 1) | b
                zs, zi, ze = self.rank(l, 0, s), self.rank(l, 0, i), self.rank(l, 0, e)
                if b == 0:
                    i, e = s + (zi - zs), s + (ze - zs)
                else:
                    i = s + (ze - zs) + (i - s) - (zi - zs)
                    s = s + (ze - zs)
            return x
        if self.kind == KIND_MULTI:
            d = 1 << self.arity_log2
            s, e, x = 0, self.n, 0
            for l in range(self.nlevels):
                g = int(self.digits(l)[i])
                x = (x << self.arity_log2) | g
                below = sum(self.mrank(l, c, e) - self.mrank(l, c, s) for c in range(g))
                ns = s + below
                i, e = ns + self.mrank(l, g, i) - self.mrank(l, g, s), ns + self.mrank(l, g, e) - self.mrank(l, g, s)
                s = ns
                assert d > g
            return x
        if self.kind == KIND_SHAPED:
            nodes = self.nodes()
            v, rel = 0, i
            while True:
                nd = nodes[v]
                l, st = nd["level"], nd["start"]
                b = self.sym_at(l, st + rel)
                rel = self.rank_any(l, b, st + rel) - self.rank_any(l, b, st)
                ch = nd["child"][b]
                if ch & LEAF:
                    return ch & ~LEAF
                v = ch
        raise ValueError("kind")

    def rank_sym(self, c: int, i: int) -> int:
        """occurrences of c in positions 0..i (inclusive)"""
        if self.kind in (KIND_WM, KIND_WT):
            L = self.nlevels
            if c >= (1 << L):
                return 0
            if self.kind == KIND_WM:
                s, e = 0, i + 1
                for l in range(L):
                    b = (c >> (L - 1 - l)) & 1
                    z = self.levels[l]["zeros"] if b else 0
                    s, e = self.rank(l, b, s) + z, self.rank(l, b, e) + z
                return e - s
            s, p, e = 0, i + 1, self.n
            for l in range(L):
                b = (c >> (L - 1 - l)) & 1
                zs, zp, ze = self.rank(l, 0, s), self.rank(l, 0, p), self.rank(l, 0, e)
                if b == 0:
                    p, e = s + (zp - zs), s + (ze - zs)
                else:
                    p = s + (ze - zs) + (p - s) - (zp - zs)
                    s = s + (ze - zs)
            return p - s
        if self.kind == KIND_MULTI:
            D, M = self.arity_log2, self.nlevels
            s, p, e = 0, i + 1, self.n
            for l in range(M):
                g = (c >> (D * (M - 1 - l))) & ((1 << D) - 1)
                below = sum(self.mrank(l, cc, e) - self.mrank(l, cc, s) for cc in range(g))
                ns = s + below
                p = ns + self.mrank(l, g, p) - self.mrank(l, g, s)
                e = ns + self.mrank(l, g, e) - self.mrank(l, g, s)
                s = ns
            return p - s
        if self.kind == KIND_SHAPED:
            codes, lens = self.codes()
            if lens[c] == 0:
                return 0
            nodes = self.nodes()
            v, rel = 0, i + 1
            for t in range(int(lens[c])):
                nd = nodes[v]
                l, st = nd["level"], nd["start"]
                b = self.code_digit(c, t)
                rel = self.rank_any(l, b, st + rel) - self.rank_any(l, b, st)
                v = nd["child"][b]
            return rel
        raise ValueError("kind")

    def select_sym(self, c: int, k: int):
        """position of the k-th occurrence of c (k >= 1), None if absent"""
        if k < 1:
            return None
        total = self.rank_sym(c, self.n - 1) if self.n else 0
        if k > total:
            return None
        if self.kind == KIND_WM:
            L = self.nlevels
            s = 0
            for l in range(L):
                b = (c >> (L - 1 - l)) & 1
                s = self.rank(l, b, s) + (self.levels[l]["zeros"] if b else 0)
            p = s + k - 1
            for l in range(L - 1, -1, -1):
                b = (c >> (L - 1 - l)) & 1
                p = self.select(l, b, p - (self.levels[l]["zeros"] if b else 0))
            return p
        if self.kind == KIND_WT:
            L = self.nlevels
            starts = []
            s, e = 0, self.n
            for l in range(L):
                starts.append(s)
                b = (c >> (L - 1 - l)) & 1
                zs, ze = self.rank(l, 0, s), self.rank(l, 0, e)
                if b == 0:
                    e = s + (ze - zs)
                else:
                    s = s + (ze - zs)
            p = s + k - 1
            child_start = s
            for l in range(L - 1, -1, -1):
                b = (c >> (L - 1 - l)) & 1
                st = starts[l]
                p = self.select(l, b, self.rank(l, b, st) + (p - child_start))
                child_start = st
            return p
        if self.kind == KIND_SHAPED:
            codes, lens = self.codes()
            nodes = self.nodes()
            path = []
            v = 0
            for t in range(int(lens[c])):
                path.append(v)
                v = nodes[v]["child"][self.code_digit(c, t)]
            rel = k - 1
            for t in range(int(lens[c]) - 1, -1, -1):
                nd = nodes[path[t]]
                l, st = nd["level"], nd["start"]
                b = self.code_digit(c, t)
                rel = self.select_any(l, b, self.rank_any(l, b, st) + rel) - st
            return rel
        if self.kind == KIND_MULTI:
            lo, hi = 0, self.n - 1
            while lo < hi:
                mid = (lo + hi) // 2
                if self.rank_sym(c, mid) >= k:
                    hi = mid
                else:
                    lo = mid + 1
            return lo
        raise ValueError("kind")


class MatrixWalk:
    """Wavelet-matrix queries through the rank directories alone, for images
    too large to expand (a zero at position i of level l moves to rank0(i),
    a one to Z_l + rank1(i))."""

    def __init__(self, img, nlevels):
        self.img, self.L = img, nlevels
        self.lv = [self.level(l) for l in range(nlevels)]

    def level(self, l):
        """(n, zeros, ones, bits_off, rank_off, sel0_off, sel1_off, nsel)"""
        d = self.img[256 + 64 * l:256 + 64 * (l + 1)].view(np.uint64)
        return [int(x) for x in d[:8]]

    def words(self, l):
        n, off = self.lv[l][0], self.lv[l][3]
        return self.img[off:off + 8 * ((n + 63) // 64)].view(np.uint64)

    def rank0(self, l, i):
        """zeros in [0, i) of level l"""
        roff = self.lv[l][4]
        k, q = divmod(i, 512)
        d = self.img[roff + 16 * k:roff + 16 * k + 16].view(np.uint64)
        r = int(d[0])
        if q >= 64:
            r += (int(d[1]) >> (9 * (q // 64 - 1))) & 511
        t = q % 64
        if t:
            w = int(self.words(l)[i // 64])
            r += t - bin(w & ((1 << t) - 1)).count("1")
        return r

    def bit(self, l, i):
        return (int(self.words(l)[i // 64]) >> (i % 64)) & 1

    def access(self, i):
        x = 0
        for l in range(self.L):
            b = self.bit(l, i)
            x = (x << 1) | b
            r0 = self.rank0(l, i)
            i = self.lv[l][1] + (i - r0) if b else r0
        return x

    def rank(self, c, i):
        """occurrences of c in positions 0..i"""
        s, e = 0, i + 1
        for l in range(self.L):
            if (c >> (self.L - 1 - l)) & 1:
                z = self.lv[l][1]
                s, e = z + s - self.rank0(l, s), z + e - self.rank0(l, e)
            else:
                s, e = self.rank0(l, s), self.rank0(l, e)
        return e - s


def array_digests(buf: np.ndarray) -> dict:
    """SHA-256 of the whole image and of every array in it (header with the
    level descriptors, then per level its bits, rank directory and select
    samples, or a multiary level's digits and counters), keyed by name in
    image order; used to compare images too large to keep two copies of"""
    import hashlib
    b = np.ascontiguousarray(np.asarray(buf, dtype=np.uint8))
    img = Image(b)
    out = {"image": hashlib.sha256(b.tobytes()).hexdigest()}
    head = img.levels_off + 64 * img.nlevels
    out["header"] = hashlib.sha256(b[:head].tobytes()).hexdigest()
    for l, lv in enumerate(img.levels):
        m = lv["n"]
        spans = [("bits", lv["bits_off"], 8 * (-(-m // 64))),
                 ("rank", lv["rank_off"], 16 * (-(-m // 512) + 1)),
                 ("sel0", lv["sel0_off"], 8 * lv["nsel"]),
                 ("sel1", lv["sel1_off"], 8 * lv["nsel"])]
        if lv["sub_off"]:
            spans.append(("sub", lv["sub_off"], 4 * lv["nsub"]))
        if lv["nslot"]:
            spans.append(("pool", lv["pool_off"], 4 * 2 * lv["nslot"] * 512))
        for name, off, size in spans:
            if off:
                out[f"level{l}.{name}"] = hashlib.sha256(b[off:off + size].tobytes()).hexdigest()
    return out
