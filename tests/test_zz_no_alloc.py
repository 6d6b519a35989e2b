"""The allocation-free matrix build (wm_build_noalloc): through the C-ABI, two
calls in a row on one GPU, the second with a smaller input, each image equal
byte for byte to wm_build's on the same input (and to the oracle's); a size
beyond the library's scratch array is refused before any device work."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import assert_same, to_device
from paper_1610_03524_amd import binding as B


def _noalloc(St, sigma, out, tune=None, stream=None):
    return B.lib().wm_build_noalloc(St.data_ptr(), St.numel(), sigma, St.element_size(),
                                    ctypes.byref(tune) if tune else None, out.data_ptr(), out.numel(),
                                    B._stream(stream))


@pytest.mark.gpu
def test_no_alloc_build_equals_wm_build_twice():
    import torch
    rng = np.random.default_rng(4242)
    cases = [((1 << 21) + 12345, 70000, np.uint32, 0),    # 17 key bits: three passes, 16-bit payload
             (50001, 300, np.uint16, 0),                  # smaller, narrower, different sigma
             (777, 5, np.uint8, 2)]                       # tiny, forced pass width
    for n, sigma, dt, tau in cases:
        S = rng.integers(0, sigma, n).astype(dt)
        St = to_device(S)
        tune = B.make_tuning(tau=tau) if tau else None
        ref, info = B.build(B.KIND_WM, St, sigma, tune=tune)
        out = torch.full((info.out_bytes,), 0xA5, dtype=torch.uint8, device="cuda")
        assert _noalloc(St, sigma, out, tune) == B.WT_OK
        torch.cuda.synchronize()
        assert B.check(out) == B.WT_OK
        got = out.cpu().numpy()
        assert_same(got, ref.cpu().numpy(), f"noalloc vs wm_build n={n} sigma={sigma}")
        assert_same(got, oracle.build_image(oracle.KIND_WM, S, sigma), f"noalloc vs oracle n={n}")


@pytest.mark.gpu
def test_no_alloc_refuses_oversized_builds():
    import torch
    St = torch.zeros(16, dtype=torch.int32, device="cuda")
    out = torch.zeros(256, dtype=torch.uint8, device="cuda")
    info = B.plan(B.KIND_WM, 1 << 28, 1 << 16, 4)
    assert info.workspace_bytes > (64 << 20)
    rc = B.lib().wm_build_noalloc(St.data_ptr(), 1 << 28, 1 << 16, 4, None, out.data_ptr(), out.numel(),
                                  B._stream(None))
    assert rc == B.WT_ENOSPC
