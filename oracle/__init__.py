"""CPU oracle for the wavelet tree / wavelet matrix builders.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never loads it, and it shares no code with the GPU path.

The oracle is a plain level-by-level C builder (``wavelet_oracle.c``) that
follows the paper's definitions:

* balanced binary wavelet tree -- Sec. 2 (recursive definition of the tree);
* wavelet matrix -- Sec. 4.3, paragraph "Wavelet matrix";
* arbitrary-shaped (Huffman-shaped) tree from codewords -- Sec. 4.3,
  paragraph "Arbitrarily-shaped binary trees";
* balanced multiary tree, degree d = 2^D -- Sec. 4.3, paragraph "Multiary";
* binary rank (rank of 0, ranges/sub-ranges) and sampled select -- Sec. 5.1;
* multiary per-digit rank counters -- Sec. 5.2, "Rank";
* canonical Huffman codewords for the Huffman-shaped tree.

It returns the canonical byte image of each structure; parity with the GPU
library is byte equality of images.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wavelet_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

KIND_WT = 1
KIND_WM = 2
KIND_SHAPED = 3
KIND_MULTI = 4

OK = 0
EINVAL = -1
ERANGE = -2
ENOMEM = -3
EUNSUP = -5


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}")
        self.code = code


def build_library() -> str:
    """Compile the oracle with gcc (plain -O2, single-threaded)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           "-o", _SO, _SRC]
    subprocess.run(cmd, check=True)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build_library()
    lib = ctypes.CDLL(_SO)
    lib.oracle_build.restype = ctypes.c_int
    lib.oracle_build.argtypes = [
        ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
        ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.POINTER(ctypes.POINTER(ctypes.c_uint8)), ctypes.POINTER(ctypes.c_uint64)]
    lib.oracle_free.restype = None
    lib.oracle_free.argtypes = [ctypes.c_void_p]
    lib.oracle_huffman.restype = ctypes.c_int
    lib.oracle_huffman.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                   ctypes.c_void_p]
    _lib = lib
    return lib


def build_image(kind: int, S: np.ndarray, sigma: int, arity_log2: int = 1,
                codes: np.ndarray | None = None, lens: np.ndarray | None = None) -> np.ndarray:
    """Build a structure over S and return its canonical image (uint8 array)."""
    lib = _load()
    S = np.ascontiguousarray(S)
    if S.dtype not in (np.uint8, np.uint16, np.uint32):
        raise TypeError("S must be uint8, uint16 or uint32")
    cp = lp = None
    if kind == KIND_SHAPED:
        codes = np.ascontiguousarray(codes, dtype=np.uint64)
        lens = np.ascontiguousarray(lens, dtype=np.uint32)
        cp, lp = codes.ctypes.data, lens.ctypes.data
    img = ctypes.POINTER(ctypes.c_uint8)()
    nbytes = ctypes.c_uint64(0)
    rc = lib.oracle_build(kind, S.ctypes.data if S.size else None, S.dtype.itemsize,
                          S.size, sigma, arity_log2, cp, lp,
                          ctypes.byref(img), ctypes.byref(nbytes))
    if rc != OK:
        raise OracleError(rc)
    try:
        out = np.ctypeslib.as_array(img, shape=(nbytes.value,)).copy()
    finally:
        lib.oracle_free(img)
    return out


def huffman(counts: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Canonical Huffman codewords (codes, lens) for per-symbol counts."""
    lib = _load()
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    sigma = counts.size
    codes = np.zeros(sigma, dtype=np.uint64)
    lens = np.zeros(sigma, dtype=np.uint32)
    rc = lib.oracle_huffman(counts.ctypes.data, sigma, codes.ctypes.data, lens.ctypes.data)
    if rc != OK:
        raise OracleError(rc)
    return codes, lens


def symbol_counts(S: np.ndarray, sigma: int) -> np.ndarray:
    """Occurrences of every symbol (plain definition, a library bincount)."""
    return np.bincount(np.asarray(S, dtype=np.int64), minlength=sigma).astype(np.uint64)
