"""Serving: every build and query result in the continuous-batching mix is
identical to the same request run alone -- the oracle's image and the
brute-force answers on S -- and a request that cannot be served fails alone;
admission respects the budget."""
import os
import threading
import time

import numpy as np
import pytest

import oracle
from gpu_util import brute_queries, to_device
from paper_1610_03524_amd import binding as B
from paper_1610_03524_amd import serve

pytestmark = pytest.mark.gpu


def pool(k=24, seed=9):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        n = int(2 ** rng.uniform(6, 17))
        sigma = max(2, int(2 ** rng.uniform(1, 20)))
        out.append((rng.integers(0, sigma, n).astype(np.uint32), sigma))
    return out


def alone(host, batches):
    """what every request returns when run alone, from the definitions: the
    oracle's image of each sequence and brute-force answers on S"""
    imgs = [oracle.build_image(oracle.KIND_WM, S, sigma) for S, sigma in host]
    res = [brute_queries(host[t][0], args) for t, args in batches]
    return imgs, res


@pytest.mark.parametrize("mode", ["continuous", "plain"])
def test_results_same_alone_and_in_the_mix(mode):
    import torch
    host = pool()
    rng = np.random.default_rng(1)
    batches = [(t, serve.make_query_batch(host[t][0], 3000, rng)) for t in range(len(host)) for _ in range(2)]
    want_imgs, want_q = alone(host, batches)
    dev = [(to_device(S), sigma) for S, sigma in host]
    srv = serve.WaveletServer(dev, hbm_budget=1 << 34, ws_bytes=1 << 28, mode=mode)
    srv.start()
    # builds arrive in bursts, every structure is built twice, queries are
    # submitted as soon as their target is resident (so they overlap builds)
    qreqs = []
    pending = list(range(len(batches)))
    for rep in range(2):
        for i in range(len(host)):
            srv.submit_build(i)
            if i % 5 == 0:
                time.sleep(0.001)
            ready = [b for b in pending if srv.is_resident(batches[b][0])]
            for b in ready[:2]:
                qreqs.append((b, srv.submit_query(batches[b][0], batches[b][1])))
                pending.remove(b)
    deadline = time.time() + 60
    while pending and time.time() < deadline:
        for b in [b for b in pending if srv.is_resident(batches[b][0])]:
            qreqs.append((b, srv.submit_query(batches[b][0], batches[b][1])))
            pending.remove(b)
        time.sleep(0.002)
    while any(not r.done for r in srv.all_reqs) and time.time() < deadline:
        time.sleep(0.005)
    srv.close()
    torch.cuda.synchronize()
    assert not pending
    for r in srv.all_reqs:
        assert r.done and r.error == 0, (r.kind, r.seq, r.error)
    for i in range(len(host)):
        got = srv.resident[i].image.cpu().numpy()
        assert np.array_equal(got, want_imgs[i]), f"image {i}"
    for b, r in qreqs:
        for g, w in zip(r.result, want_q[b]):
            assert np.array_equal(g.cpu().numpy(), w), f"query batch {b}"
    if mode == "continuous":
        assert max(srv.batches) > 1   # builds were batched


def test_workspace_that_fits_the_batch_but_not_a_single_build():
    """Admission counts a sequence's batched workspace; its single build can
    need a little more.  With a workspace of exactly the batched figure a
    lone request is built as a batch of one (continuous mode) and equals the
    oracle's image; the plain queue, which builds one by one, refuses it."""
    import torch
    rng = np.random.default_rng(77)
    S, sigma = rng.integers(0, 5209, 2611909).astype(np.uint32), 5209
    dev = [(to_device(S), sigma)]
    probe = serve.WaveletServer(dev, hbm_budget=1 << 34, ws_bytes=1 << 20)
    _, batch_ws, single_ws, _ = probe._costs(0)
    del probe
    assert single_ws > batch_ws   # the case this test is about
    want = oracle.build_image(oracle.KIND_WM, S, sigma)
    for mode, code in (("continuous", 0), ("plain", B.WT_ENOSPC)):
        srv = serve.WaveletServer(dev, hbm_budget=1 << 34, ws_bytes=batch_ws, mode=mode)
        srv.start()
        r = srv.submit_build(0)
        deadline = time.time() + 60
        while not r.done and time.time() < deadline:
            time.sleep(0.002)
        srv.close()
        torch.cuda.synchronize()
        assert r.done and r.error == code, (mode, r.error)
        if code == 0:
            assert np.array_equal(srv.resident[0].image.cpu().numpy(), want)


def test_budget_admission_and_eviction():
    import torch
    host = pool(12, seed=3)
    dev = [(to_device(S), sigma) for S, sigma in host]
    sizes = [B.plan(B.KIND_WM, S.size, sigma, 4).out_bytes for S, sigma in host]
    budget = sorted(sizes)[-3] + sorted(sizes)[-4]   # two mid-size images fit
    srv = serve.WaveletServer(dev, hbm_budget=budget, ws_bytes=1 << 28)
    srv.start()
    reqs = [srv.submit_build(i) for i in range(len(host))]
    deadline = time.time() + 60
    while any(not r.done for r in reqs) and time.time() < deadline:
        time.sleep(0.005)
    srv.close()
    assert srv.used <= budget
    for r, sz in zip(reqs, sizes):
        if sz > budget:
            assert r.error == B.WT_ENOSPC
        else:
            assert r.error == 0
    # whatever stayed resident is exactly the image built alone
    want, _ = alone(host, [])
    for i, st in srv.resident.items():
        assert np.array_equal(st.image.cpu().numpy(), want[i])
    torch.cuda.synchronize()


@pytest.mark.parametrize("seed", range(int(os.environ.get("WV_RANDOM_SERVE", "4"))))
@pytest.mark.parametrize("mode", ["continuous", "plain"])
def test_random_mix_same_as_alone(seed, mode):
    """random pools, query batch sizes, repeats and burst timing; every image
    and every query result equal to the request run alone"""
    import torch
    rng = np.random.default_rng(12345 + seed)
    host = pool(int(rng.integers(4, 40)), seed=1000 + seed)
    nb = int(rng.integers(1, 4))
    batches = [(t, serve.make_query_batch(host[t][0], int(rng.integers(1, 4000)), rng))
               for t in range(len(host)) for _ in range(nb)]
    want_imgs, want_q = alone(host, batches)
    dev = [(to_device(S), sigma) for S, sigma in host]
    srv = serve.WaveletServer(dev, hbm_budget=1 << 34, ws_bytes=1 << 28, mode=mode)
    srv.start()
    qreqs, pending = [], list(range(len(batches)))
    burst = int(rng.integers(1, 9))
    pause = float(rng.choice([0.0, 0.0005, 0.002]))
    for _ in range(int(rng.integers(1, 4))):
        for i in rng.permutation(len(host)):
            srv.submit_build(int(i))
            if i % burst == 0 and pause:
                time.sleep(pause)
            for b in [b for b in pending if srv.is_resident(batches[b][0])][:3]:
                qreqs.append((b, srv.submit_query(batches[b][0], batches[b][1])))
                pending.remove(b)
    deadline = time.time() + 60
    while pending and time.time() < deadline:
        for b in [b for b in pending if srv.is_resident(batches[b][0])]:
            qreqs.append((b, srv.submit_query(batches[b][0], batches[b][1])))
            pending.remove(b)
        time.sleep(0.001)
    while any(not r.done for r in srv.all_reqs) and time.time() < deadline:
        time.sleep(0.002)
    srv.close()
    torch.cuda.synchronize()
    assert not pending
    for r in srv.all_reqs:
        assert r.done and r.error == 0, (r.kind, r.seq, r.error)
    for i in range(len(host)):
        assert np.array_equal(srv.resident[i].image.cpu().numpy(), want_imgs[i]), f"image {i}"
    for b, r in qreqs:
        for g, w in zip(r.result, want_q[b]):
            assert np.array_equal(g.cpu().numpy(), w), f"query batch {b}"


@pytest.mark.parametrize("seed", range(int(os.environ.get("WV_RANDOM_EVICT", "4"))))
@pytest.mark.parametrize("mode", ["continuous", "plain"])
def test_random_mix_under_a_small_budget(seed, mode):
    """budgets of one to four images: structures are evicted and rebuilt
    while queries run; a query either finds its structure (results as alone)
    or reports WT_EINVAL, resident images are as alone, usage stays within
    the budget"""
    import torch
    rng = np.random.default_rng(777777 + seed)
    host = pool(int(rng.integers(6, 30)), seed=5000 + seed)
    sizes = [B.plan(B.KIND_WM, S.size, sigma, 4).out_bytes for S, sigma in host]
    budget = int(max(sizes) * rng.uniform(1.0, 4.0)) + 4096
    batches = [(t, serve.make_query_batch(host[t][0], int(rng.integers(1, 2000)), rng)) for t in range(len(host))]
    want_imgs, want_q = alone(host, batches)
    dev = [(to_device(S), sigma) for S, sigma in host]
    srv = serve.WaveletServer(dev, hbm_budget=budget, ws_bytes=1 << 28, mode=mode)
    srv.start()
    qreqs = []
    for _ in range(2):
        for i in rng.permutation(len(host)):
            srv.submit_build(int(i))
            if rng.random() < 0.3:
                time.sleep(0.0005)
            for b in range(len(batches)):
                if rng.random() < 0.1 and srv.is_resident(batches[b][0]):
                    qreqs.append((b, srv.submit_query(batches[b][0], batches[b][1])))
    deadline = time.time() + 60
    while any(not r.done for r in srv.all_reqs) and time.time() < deadline:
        time.sleep(0.002)
    srv.close()
    torch.cuda.synchronize()
    assert all(r.done for r in srv.all_reqs)
    assert srv.used <= budget
    for b, r in qreqs:
        if r.error == B.WT_EINVAL:
            continue
        assert r.error == 0
        for g, w in zip(r.result, want_q[b]):
            assert np.array_equal(g.cpu().numpy(), w), f"query batch {b}"
    for i, st in list(srv.resident.items()):
        assert np.array_equal(st.image.cpu().numpy(), want_imgs[i]), f"image {i}"


@pytest.mark.parametrize("mode", ["continuous", "plain"])
def test_bad_requests_fail_alone(mode):
    """a sequence the library refuses (sigma = 0) and one holding a symbol >=
    sigma, in a mix of good ones: the two fail with their own codes (WT_EINVAL
    at admission, WT_ERANGE from the image status) and are never resident;
    every other build equals the oracle and every query brute force, and the
    workers keep serving after them"""
    import torch
    host = pool(10, seed=21)
    bad_sigma = len(host)
    S0 = host[0][0].copy()
    host.append((S0, 0))                       # refused by the plan
    rng = np.random.default_rng(5)
    S1 = rng.integers(0, 300, 5000).astype(np.uint32)
    S1[1234] = 300                             # one symbol == sigma
    host.append((S1, 300))
    bad_range = len(host) - 1
    good = [i for i in range(len(host)) if i not in (bad_sigma, bad_range)]
    batches = [(t, serve.make_query_batch(host[t][0], 1500, rng)) for t in good]
    want_imgs = {i: oracle.build_image(oracle.KIND_WM, *host[i]) for i in good}
    want_q = [brute_queries(host[t][0], args) for t, args in batches]
    dev = [(to_device(S), sigma) for S, sigma in host]
    srv = serve.WaveletServer(dev, hbm_budget=1 << 34, ws_bytes=1 << 28, mode=mode)
    srv.start()
    order = [bad_sigma] + good[:4] + [bad_range] + good[4:] + [bad_sigma, bad_range]
    reqs = {}
    for i in order:
        reqs.setdefault(i, []).append(srv.submit_build(i))
    deadline = time.time() + 60
    while any(not r.done for r in srv.all_reqs) and time.time() < deadline:
        time.sleep(0.002)
    qreqs = [(b, srv.submit_query(t, args)) for b, (t, args) in enumerate(batches)]
    while any(not r.done for r in srv.all_reqs) and time.time() < deadline:
        time.sleep(0.002)
    srv.close()
    torch.cuda.synchronize()
    assert all(r.done for r in srv.all_reqs)
    assert all(r.error == B.WT_EINVAL for r in reqs[bad_sigma])
    assert all(r.error == B.WT_ERANGE for r in reqs[bad_range])
    assert bad_sigma not in srv.resident and bad_range not in srv.resident
    for i in good:
        assert all(r.error == 0 for r in reqs[i]), i
        assert np.array_equal(srv.resident[i].image.cpu().numpy(), want_imgs[i]), f"image {i}"
    for b, r in qreqs:
        assert r.error == 0
        for g, w in zip(r.result, want_q[b]):
            assert np.array_equal(g.cpu().numpy(), w), f"query batch {b}"
    # a query on a structure that was never built fails alone as well
    srv2 = serve.WaveletServer(dev, hbm_budget=1 << 34, ws_bytes=1 << 28, mode=mode)
    srv2.start()
    q = srv2.submit_query(bad_range, batches[0][1])
    ok = srv2.submit_build(good[0])
    while not (q.done and ok.done) and time.time() < deadline:
        time.sleep(0.002)
    srv2.close()
    assert q.error == B.WT_EINVAL and ok.error == 0
