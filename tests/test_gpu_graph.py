"""A wavelet-matrix build is stream-ordered device work only (kernel
launches: no host synchronization, copy or memset), so a caller can capture
it into a HIP graph and replay it.  Every replay must write the image the
eager build writes, after eager work has overwritten the image and the
workspace in between."""
import numpy as np
import pytest

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
