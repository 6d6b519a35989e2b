"""ctypes binding of libwavelet (the C-ABI of include/wavelet.h).

Argument marshalling only: every step of a build or query runs in the HIP
library.  PyTorch supplies device memory and the stream.  Importing this
module does not load the library; the first call does, and raises if the
library was not built (there is no other implementation to fall back to).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwavelet.so")

WT_OK, WT_EINVAL, WT_ERANGE, WT_ENOSPC, WT_EHIP, WT_EUNSUP = 0, -1, -2, -3, -4, -5
KIND_WT, KIND_WM, KIND_SHAPED, KIND_MULTIARY = 1, 2, 3, 4
FLAG_LEVELWISE = 1
FLAG_PROFILE = 2
U32_MAX = 0xFFFFFFFF
U64_MAX = 0xFFFFFFFFFFFFFFFF

c_u32, c_u64, c_vp, c_int = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int


class wt_shape(ctypes.Structure):
    _fields_ = [("arity_log2", c_u32), ("reserved", c_u32), ("codes", c_vp),
                ("code_len", c_vp), ("counts", c_vp)]


class wt_tuning(ctypes.Structure):
    _fields_ = [("tau", c_u32), ("tile", c_u32), ("blocks", c_u32), ("flags", c_u32)]


class wt_plan_info(ctypes.Structure):
    _fields_ = [("kind", c_u32), ("nlevels", c_u32), ("key_bits", c_u32), ("arity_log2", c_u32),
                ("n", c_u64), ("sigma", c_u32), ("tau", c_u32), ("out_bytes", c_u64),
                ("workspace_bytes", c_u64), ("level_n", c_u64 * 32), ("split_bits", c_u32),
                ("reserved0", c_u32), ("split_long", c_u64)]


class wt_seq_desc(ctypes.Structure):
    _fields_ = [("S", c_vp), ("n", c_u64), ("sigma", c_u32), ("sym_bytes", c_u32),
                ("out", c_vp), ("out_bytes", c_u64), ("tau", c_u32), ("reserved", c_u32)]


class wt_profile_entry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", c_u64), ("ms", ctypes.c_double)]


class WaveletError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


_lib = None

_SIGS = {
    "wt_plan": (c_int, [c_int, c_u64, c_u32, c_u32, c_vp, c_vp, c_vp]),
    "wt_build": (c_int, [c_vp, c_u64, c_u32, c_u32, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp,
                         ctypes.c_size_t, c_vp]),
    "wm_build": (c_int, [c_vp, c_u64, c_u32, c_u32, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp,
                         ctypes.c_size_t, c_vp]),
    "multiary_build": (c_int, [c_vp, c_u64, c_u32, c_u32, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp,
                               ctypes.c_size_t, c_vp]),
    "wm_build_noalloc": (c_int, [c_vp, c_u64, c_u32, c_u32, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "wt_check": (c_int, [c_vp, c_vp]),
    "wt_access": (c_int, [c_vp, c_vp, c_vp, c_u64, c_vp]),
    "wt_rank": (c_int, [c_vp, c_vp, c_vp, c_vp, c_u64, c_vp]),
    "wt_select": (c_int, [c_vp, c_vp, c_vp, c_vp, c_u64, c_vp]),
    "wt_symbol_counts": (c_int, [c_vp, c_u64, c_u32, c_u32, c_vp, c_vp]),
    "wt_huffman_codes": (c_int, [c_vp, c_u32, c_vp, c_vp]),
    "wt_huffman_codes_dev": (c_int, [c_vp, c_u32, c_vp, c_vp, c_vp, c_vp]),
    "wt_batch_plan": (c_int, [c_int, c_vp, c_u32, c_vp, c_vp]),
    "wt_batch_build": (c_int, [c_int, c_vp, c_u32, c_vp, ctypes.c_size_t, c_vp, c_vp]),
    "wt_image_bytes": (c_int, [c_vp, c_vp, c_vp]),
    "wt_profile_read": (c_int, [c_vp, c_u32, c_vp]),
    "wt_strerror": (ctypes.c_char_p, [c_int]),
}


def lib():
    """Load libwavelet.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1610_03524_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols() -> list[str]:
    return list(_SIGS)


def strerror(code: int) -> str:
    try:
        return lib().wt_strerror(code).decode()
    except Exception:  # library missing: still format the error
        return f"status {code}"


def _check(rc: int, what: str):
    if rc != WT_OK:
        raise WaveletError(rc, what)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


# element types the header declares for every device argument (signedness is
# not checked: tests and callers view unsigned data through torch's signed
# types of the same width)
_SYM_DTYPES = ("uint8", "int8", "int16", "uint16", "int32", "uint32")
_U64 = ("int64", "uint64")
_U32 = ("int32", "uint32")
_U8 = ("uint8", "int8")


def _arg(t, name: str, dtypes, what: str):
    """Reject, before any pointer reaches the library, an argument that is not a
    contiguous device tensor of one of the element types the header declares
    (a host array or a strided view would be read as device memory of another
    shape).  Raises WaveletError(WT_EINVAL)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise WaveletError(WT_EINVAL, f"{what}: {name} must be a torch tensor, got {type(t).__name__}")
    dt = str(t.dtype).replace("torch.", "")
    if dt not in dtypes:
        raise WaveletError(WT_EINVAL, f"{what}: {name} has dtype {dt}, expected one of {', '.join(dtypes)}")
    if not t.is_contiguous():
        raise WaveletError(WT_EINVAL, f"{what}: {name} must be contiguous")
    return t


def _same_len(what: str, **named):
    sizes = {k: v.numel() for k, v in named.items()}
    if len(set(sizes.values())) > 1:
        raise WaveletError(WT_EINVAL, f"{what}: lengths differ: {sizes}")


def _on_device(what: str, *ts):
    """every tensor in device memory, all on one device (checked after the
    element types and lengths)"""
    for t in ts:
        if t.device.type != "cuda":
            raise WaveletError(WT_EINVAL, f"{what}: arguments must be device tensors, got {t.device}")
    devs = {str(t.device) for t in ts}
    if len(devs) > 1:
        raise WaveletError(WT_EINVAL, f"{what}: arguments on different devices: {sorted(devs)}")


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _sym_bytes(S) -> int:
    return S.element_size()


def make_shape(arity_log2: int = 0, codes=None, code_len=None, counts=None):
    """Build a wt_shape; keeps the numpy arrays alive on the returned object."""
    sh = wt_shape()
    sh.arity_log2 = arity_log2
    keep = []
    if codes is not None:
        codes = np.ascontiguousarray(codes, dtype=np.uint64)
        code_len = np.ascontiguousarray(code_len, dtype=np.uint32)
        counts = np.ascontiguousarray(counts, dtype=np.uint64)
        keep = [codes, code_len, counts]
        sh.codes, sh.code_len, sh.counts = codes.ctypes.data, code_len.ctypes.data, counts.ctypes.data
    sh._keep = keep
    return sh


def make_tuning(tau: int = 0, tile: int = 0, blocks: int = 0, flags: int = 0):
    t = wt_tuning()
    t.tau, t.tile, t.blocks, t.flags = tau, tile, blocks, flags
    return t


def plan(kind: int, n: int, sigma: int, sym_bytes: int, shape=None, tune=None) -> wt_plan_info:
    info = wt_plan_info()
    rc = lib().wt_plan(kind, n, sigma, sym_bytes, ctypes.byref(shape) if shape else None,
                       ctypes.byref(tune) if tune else None, ctypes.byref(info))
    _check(rc, "wt_plan")
    return info


def _build_fn(kind: int):
    L = lib()
    return {KIND_WT: L.wt_build, KIND_SHAPED: L.wt_build, KIND_WM: L.wm_build,
            KIND_MULTIARY: L.multiary_build}[kind]


def build_into(kind: int, S, sigma: int, out, ws, shape=None, tune=None, stream=None) -> int:
    """Call wt_build / wm_build / multiary_build on caller-owned buffers."""
    _arg(S, "S", _SYM_DTYPES, "build")
    _arg(out, "out", _U8, "build")
    _arg(ws, "ws", _U8, "build")
    _on_device("build", S, out, ws)
    fn = _build_fn(kind)
    return fn(_ptr(S), S.numel(), sigma, _sym_bytes(S), ctypes.byref(shape) if shape else None,
              ctypes.byref(tune) if tune else None, _ptr(out), out.numel(), _ptr(ws), ws.numel(),
              _stream(stream))


def build(kind: int, S, sigma: int, arity_log2: int = 0, codes=None, code_len=None, counts=None,
          tune=None, stream=None):
    """Plan, allocate and build; returns (image tensor on S's device, plan info)."""
    import torch
    shape = make_shape(arity_log2, codes, code_len, counts) if (arity_log2 or codes is not None) else None
    info = plan(kind, S.numel(), sigma, _sym_bytes(S), shape, tune)
    out = torch.empty(info.out_bytes, dtype=torch.uint8, device=S.device)
    ws = torch.empty(max(info.workspace_bytes, 1), dtype=torch.uint8, device=S.device)
    _check(build_into(kind, S, sigma, out, ws, shape, tune, stream), "build")
    return out, info


def check(image, stream=None) -> int:
    _arg(image, "image", _U8, "wt_check")
    _on_device("wt_check", image)
    return lib().wt_check(_ptr(image), _stream(stream))


def access(image, pos, stream=None):
    import torch
    _arg(image, "image", _U8, "wt_access")
    _arg(pos, "pos", _U64, "wt_access")
    _on_device("wt_access", image, pos)
    res = torch.empty(pos.numel(), dtype=torch.int32, device=pos.device)
    _check(lib().wt_access(_ptr(image), _ptr(pos), _ptr(res), pos.numel(), _stream(stream)), "wt_access")
    return res


def rank(image, c, i, stream=None):
    import torch
    _arg(image, "image", _U8, "wt_rank")
    _arg(c, "c", _U32, "wt_rank")
    _arg(i, "i", _U64, "wt_rank")
    _same_len("wt_rank", c=c, i=i)
    _on_device("wt_rank", image, c, i)
    res = torch.empty(i.numel(), dtype=torch.int64, device=i.device)
    _check(lib().wt_rank(_ptr(image), _ptr(c), _ptr(i), _ptr(res), i.numel(), _stream(stream)), "wt_rank")
    return res


def select(image, c, k, stream=None):
    import torch
    _arg(image, "image", _U8, "wt_select")
    _arg(c, "c", _U32, "wt_select")
    _arg(k, "k", _U64, "wt_select")
    _same_len("wt_select", c=c, k=k)
    _on_device("wt_select", image, c, k)
    res = torch.empty(k.numel(), dtype=torch.int64, device=k.device)
    _check(lib().wt_select(_ptr(image), _ptr(c), _ptr(k), _ptr(res), k.numel(), _stream(stream)), "wt_select")
    return res


def symbol_counts(S, sigma: int, stream=None):
    import torch
    _arg(S, "S", _SYM_DTYPES, "wt_symbol_counts")
    _on_device("wt_symbol_counts", S)
    counts = torch.empty(sigma, dtype=torch.int64, device=S.device)
    _check(lib().wt_symbol_counts(_ptr(S), S.numel(), _sym_bytes(S), sigma, _ptr(counts), _stream(stream)),
           "wt_symbol_counts")
    return counts


def huffman_codes(counts: np.ndarray):
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    codes = np.zeros(counts.size, dtype=np.uint64)
    lens = np.zeros(counts.size, dtype=np.uint32)
    _check(lib().wt_huffman_codes(counts.ctypes.data, counts.size, codes.ctypes.data, lens.ctypes.data),
           "wt_huffman_codes")
    return codes, lens


def huffman_codes_dev(counts, stream=None):
    """canonical Huffman codewords computed on the device from device counts
    (int64 tensor of sigma); returns (codes int64, lengths int32, status int32)
    device tensors, not synchronized"""
    import torch
    _arg(counts, "counts", _U64, "wt_huffman_codes_dev")
    _on_device("wt_huffman_codes_dev", counts)
    sigma = counts.numel()
    codes = torch.empty(sigma, dtype=torch.int64, device=counts.device)
    lens = torch.empty(sigma, dtype=torch.int32, device=counts.device)
    status = torch.empty(1, dtype=torch.int32, device=counts.device)
    _check(lib().wt_huffman_codes_dev(_ptr(counts), sigma, _ptr(codes), _ptr(lens), _ptr(status), _stream(stream)),
           "wt_huffman_codes_dev")
    return codes, lens, status


def image_bytes(image, stream=None) -> int:
    _arg(image, "image", _U8, "wt_image_bytes")
    _on_device("wt_image_bytes", image)
    b = ctypes.c_uint64(0)
    _check(lib().wt_image_bytes(_ptr(image), ctypes.byref(b), _stream(stream)), "wt_image_bytes")
    return b.value


def profile_read(cap: int = 64) -> dict:
    """{kernel name: (launches, total ms)} of profiled builds since the last read"""
    arr = (wt_profile_entry * cap)()
    cnt = ctypes.c_uint32(0)
    _check(lib().wt_profile_read(arr, cap, ctypes.byref(cnt)), "wt_profile_read")
    return {arr[i].name.decode(): (arr[i].launches, arr[i].ms) for i in range(min(cap, cnt.value))}


def make_desc(S, sigma: int, out, tau: int = 0) -> wt_seq_desc:
    """One batch descriptor over a device sequence and its image buffer,
    checked like the arguments of a single build."""
    _arg(S, "S", _SYM_DTYPES, "wt_seq_desc")
    _arg(out, "out", _U8, "wt_seq_desc")
    _on_device("wt_seq_desc", S, out)
    d = wt_seq_desc()
    d.S, d.n, d.sigma, d.sym_bytes = S.data_ptr(), S.numel(), sigma, S.element_size()
    d.out, d.out_bytes, d.tau = out.data_ptr(), out.numel(), tau
    return d


def desc_array(descs):
    """descs as the C array the batch calls take (a ctypes array is used as is,
    so a caller that builds several batches of the same sequences marshals once)"""
    if isinstance(descs, ctypes.Array):
        return descs
    return (wt_seq_desc * len(descs))(*descs)


def batch_plan(kind: int, descs, tune=None) -> int:
    arr = desc_array(descs)
    ws = ctypes.c_uint64(0)
    _check(lib().wt_batch_plan(kind, arr, len(descs), ctypes.byref(tune) if tune else None, ctypes.byref(ws)),
           "wt_batch_plan")
    return ws.value


def batch_build(kind: int, descs, ws, tune=None, stream=None) -> int:
    _arg(ws, "ws", _U8, "wt_batch_build")
    _on_device("wt_batch_build", ws)
    arr = desc_array(descs)
    return lib().wt_batch_build(kind, arr, len(descs), _ptr(ws), ws.numel(),
                                ctypes.byref(tune) if tune else None, _stream(stream))
