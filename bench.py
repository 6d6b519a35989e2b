#!/usr/bin/env python3
"""Benchmark: wavelet-matrix construction on one MI355X.

Default workload: n = 2^28 uint32 symbols, sigma = 2^16, Zipf(s=1.1) over a
seed-permuted alphabet (16 levels, rank directory and sampled select on every
level).  One step = one complete wm_build (every level bitvector, every rank
directory, every select sample, the image header) from the input already in
HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --workload c1|c3h|c3m|c4|c5  (the other configurations)
    python bench.py --copy-calibration           (1 GiB copy for PMC scaling)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "build GB/s of input (symbol-levels/sec) and % HBM roofline; batched vs plain"


def algorithmic_bytes(info, n, sym_bytes):
    """compulsory bytes of one build: read S once, write every output array
    once (level bits, rank directory, select samples, header)"""
    return n * sym_bytes + info.out_bytes


def symbol_levels(info):
    return sum(int(info.level_n[l]) for l in range(info.nlevels))


KERNEL_TIMING = ("HIP events recorded around every launch on the build stream, in a second loop of the "
                 "same builds right after the timed one (the events add gaps between launches, not kernel time, "
                 "so the headline loop runs without them)")


def profiled_kernels(B, build_profiled, steps, stream):
    """{kernel: (launches, ms)} over `steps` builds run with WT_FLAG_PROFILE"""
    import torch
    build_profiled()
    torch.cuda.synchronize()
    B.profile_read()
    for _ in range(steps):
        build_profiled()
    torch.cuda.synchronize()
    return B.profile_read()


def time_builds(build_once, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        build_once()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        build_once()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps   # ms per step


def cpu_baseline_wm(S_dev, sigma, target_s=15.0):
    """the oracle (single-threaded C, -O2) on a prefix of the same input"""
    import oracle
    n_total = S_dev.numel()
    n_s = min(n_total, 1 << 22)
    S = S_dev[:n_s].cpu().numpy().view(np.uint32)
    t = time.perf_counter()
    oracle.build_image(oracle.KIND_WM, S, sigma)
    dt = time.perf_counter() - t
    # grow the sample towards ~target_s seconds of oracle work
    if dt < target_s / 4 and n_s < n_total:
        n_s = int(min(n_total, n_s * max(1.0, target_s / max(dt, 1e-3))))
        n_s = max(1 << 22, n_s & ~0xFFFF)
        S = S_dev[:n_s].cpu().numpy().view(np.uint32)
        t = time.perf_counter()
        oracle.build_image(oracle.KIND_WM, S, sigma)
        dt = time.perf_counter() - t
    return {"value": round(n_s * 4 / dt / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_s} symbols of the same input, full wavelet matrix with directories, "
                      f"{dt:.1f} s single-threaded", **host_cpu()}


def device_copy_gbps(reps=10):
    """bytes read + written per second by a plain 1 GiB device-to-device copy:
    the bandwidth ceiling measured on this machine, beside the nominal peak"""
    import torch
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2 * (1 << 30) * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return round(gbps, 1)


def per_build_times(build_once, stream, reps=20):
    """every build timed alone with events, 512 MiB written between builds so
    that no input or output is left in the L2 or MALL; median, p10, p90"""
    import torch
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    ms = []
    for r in range(reps):
        flush.fill_(r & 0xFF)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        build_once()
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    del flush
    q = np.percentile(ms, [50, 10, 90])
    return {"reps": reps, "median_ms": round(float(q[0]), 4), "p10_ms": round(float(q[1]), 4),
            "p90_ms": round(float(q[2]), 4), "flush": "512 MiB written before every build"}


def cpu_baseline_oracle(kind, S, sigma, D=0, codes=None, lens=None, target_s=10.0):
    """the oracle (single-threaded C, -O2) on a prefix of S grown towards
    ~target_s seconds (the whole input built again and again when it takes
    less); GB/s of input"""
    import oracle
    n_s = min(S.size, 1 << 18)
    while True:
        t = time.perf_counter()
        oracle.build_image(kind, S[:n_s], sigma, max(D, 1), codes=codes, lens=lens)
        dt = time.perf_counter() - t
        if dt >= target_s / 4 or n_s >= S.size:
            break
        n_s = int(min(S.size, n_s * max(2.0, target_s / max(dt, 1e-3))))
    builds = 1
    while dt < target_s / 4:   # the whole input is short: repeat it
        t = time.perf_counter()
        oracle.build_image(kind, S[:n_s], sigma, max(D, 1), codes=codes, lens=lens)
        dt += time.perf_counter() - t
        builds += 1
    what = f"first {n_s} symbols of the same input" if n_s < S.size else f"the whole input ({n_s} symbols)"
    rep_ = f", built {builds} times" if builds > 1 else ""
    return {"value": round(builds * n_s * S.itemsize / dt / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{what}{rep_}, {dt:.1f} s single-threaded", **host_cpu()}


def pass_alg_bytes(info, n, sym_bytes):
    """algorithmic (compulsory) bytes of every launch of the partition pass
    kernel: the first pass reads S once, and every pass writes the bits of its
    levels once.  The compacted remaining keys one pass writes and the next
    reads are intermediate traffic: they appear in the measured traffic (and
    so in the amplification), never here."""
    L, tau = info.nlevels, info.tau
    per = []
    for l0 in range(0, L, tau):
        t = min(tau, L - l0)
        per.append((n * sym_bytes if l0 == 0 else 0) + t * ((n + 63) // 64) * 8)
    return per


def pass_payload_bytes(info, n):
    """bytes of compacted remaining keys the passes write and read back (not
    algorithmic; reported beside the roofline only)"""
    L, tau = info.nlevels, info.tau
    width = lambda bits: 1 if bits <= 8 else (2 if bits <= 16 else 4)
    total = 0
    for l0 in range(0, L, tau):
        rem = L - l0 - min(tau, L - l0)
        if rem:
            total += 2 * n * width(rem)
    return total


def host_cpu():
    """the host CPU model (lscpu / cpuinfo), the cores this process may run on
    and the worker threads a pool uses here (the CPU share the box gives one
    GPU caps it: OMP_NUM_THREADS)"""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return {"cpu_model": model, "nproc": nproc, "pool_threads": min(nproc, share) if share > 0 else nproc}


# the sources the pass kernel is compiled from
PASS_SOURCES = ["paper_1610_03524_amd/csrc/wv_common.h", "paper_1610_03524_amd/csrc/wv_wm_core.h",
                "paper_1610_03524_amd/csrc/wv_wm_passes.hip"]


def pass_source_digest():
    import hashlib
    h = hashlib.sha256()
    for rel in PASS_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_from_profile():
    """HBM bytes per launch of the pass kernel measured with rocprofv3 PMC
    counters (FETCH_SIZE, WRITE_SIZE), scaled by the same counters' reading
    for a plain copy; null when the kernel's sources changed since"""
    path = os.path.join(ROOT, "profiles", "wm_pass_c2_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sha256") != pass_source_digest():
        return None
    return rec.get("bytes_per_launch")


def copy_calibration(steps):
    """a plain 1 GiB device copy, for scaling the PMC byte counters"""
    import torch
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(steps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "launches": steps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--workload", default="c2", choices=["c2", "c1", "c3h", "c3m", "c3hm", "c4", "c5"])
    ap.add_argument("--horizon", type=float, default=2.0,
                    help="c5: seconds of arrivals per rate, at least enough for --min-builds builds")
    ap.add_argument("--min-builds", type=int, default=3000,
                    help="c5: arrivals per rate at least (so that a p99 rests on 30 samples or more)")
    ap.add_argument("--modes", default="continuous,plain", help="c5: serving modes, run in this order per rate")
    ap.add_argument("--rates", default="100,300,1000,3000,10000,20000,50000", help="c5: build arrival rates /s")
    ap.add_argument("--limit", type=int, default=8192, help="c4: number of sequences")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU form of this "
              "build is a design, not an implementation", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.steps)
        return
    if args.workload in ("c1", "c3h", "c3m", "c3hm"):
        bench_tree(args)
        return
    if args.workload == "c4":
        bench_batch(args)
        return
    if args.workload == "c5":
        bench_serve(args)
        return

    import torch
    from paper_1610_03524_amd import binding as B
    from paper_1610_03524_amd import inputs, tune as T

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    sigma = 1 << 16
    n = 1 << 28
    S = inputs.c2_zipf(n=n, sigma=sigma, seed=2, device=dev)
    torch.cuda.synchronize()
    tau, tile = T.choose_tuning(n, sigma)   # the tuner's choice for this shape (0 = automatic)
    tune = B.make_tuning(tau=tau, tile=tile)
    prof_tune = B.make_tuning(tau=tau, tile=tile, flags=B.FLAG_PROFILE)
    info = B.plan(B.KIND_WM, n, sigma, 4, tune=tune)
    out = torch.empty(info.out_bytes, dtype=torch.uint8, device=dev)
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device=dev)

    def build_with(tn):
        rc = B.build_into(B.KIND_WM, S, sigma, out, ws, tune=tn, stream=stream)
        if rc != 0:
            raise RuntimeError(f"wm_build failed: {B.strerror(rc)}")

    ms = time_builds(lambda: build_with(tune), args.steps, args.warmup, stream)
    assert B.check(out, stream) == B.WT_OK
    prof = profiled_kernels(B, lambda: build_with(prof_tune), args.steps, stream)
    t = ms / 1e3
    per_build = per_build_times(lambda: build_with(tune), stream)
    copy_gbps = device_copy_gbps()

    # dominant kernel: the partition pass, timed live with HIP events
    launches, pass_ms = prof["wm_pass"]
    per_launch_ms = pass_ms / launches
    alg_per_launch = sum(pass_alg_bytes(info, n, 4)) / info_passes(info)
    achieved = alg_per_launch / (per_launch_ms / 1e3) / 1e9
    payload_per_launch = pass_payload_bytes(info, n) / info_passes(info)
    balg = algorithmic_bytes(info, n, 4)
    traffic = traffic_from_profile()
    line = {
        "metric": METRIC,
        "value": round(n * 4 / t / 1e9, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "C2 wavelet matrix: n=2^28 uint32, sigma=2^16, Zipf(s=1.1) over a permuted "
                               "alphabet, 16 levels + rank directory + select samples",
                   "n": n, "sigma": sigma, "levels": info.nlevels, "tau": info.tau,
                   "tiles_per_chunk": tile or "automatic"},
        "symbol_levels_per_s": round(symbol_levels(info) / t, 1),
        "roofline": {"bound": "hbm", "kernel": "wm_pass", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic, "alg_bytes_per_launch": int(alg_per_launch),
                     "alg_bytes_rule": "first pass reads S once; every pass writes its levels' bits once",
                     "amplification": round(traffic / alg_per_launch, 3) if traffic else None,
                     "payload_bytes_per_launch": int(payload_per_launch),
                     "avg_launch_ms": round(per_launch_ms, 4),
                     "frac_of_device_copy": round(achieved / copy_gbps, 4)},
        "build_roofline": {"alg_bytes": balg, "achieved": round(balg / t / 1e9, 2),
                           "frac": round(balg / t / 1e9 / HBM_PEAK_GBPS, 4),
                           "frac_of_device_copy": round(balg / t / 1e9 / copy_gbps, 4)},
        "device_copy_GBps": copy_gbps,
        "per_build": per_build,
        "kernel_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in sorted(prof.items())},
        "kernel_timing": KERNEL_TIMING,
    }
    line["queries"] = query_rates(out, S, n, sigma, info.nlevels, stream)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_wm(S, sigma)
    print(json.dumps(line), flush=True)


def query_rates(img, S, n, sigma, levels, stream, m=1 << 22, reps=5):
    """Batched access / rank / select on the built matrix, outside the timed
    build step: m queries per kind from the same input (uniform positions,
    symbols drawn from S, select ranks uniform in [1, occurrences]).  Each
    query reads, per level, a bit word and a directory entry: two 64-byte
    lines of random access, the algorithmic bytes of the line rate below
    (select reads more: it searches the level's select samples).  An image
    smaller than the 256 MiB last-level cache is served from cache, so no
    HBM fraction is given for it."""
    import torch
    from paper_1610_03524_amd import binding as B
    dev = S.device
    g = torch.Generator(device=dev)
    g.manual_seed(10)
    pos = torch.randint(0, n, (m,), device=dev, generator=g, dtype=torch.int64)
    Sl = S.to(torch.int64) & ((1 << (8 * S.element_size())) - 1)   # stored unsigned
    c = Sl[torch.randint(0, n, (m,), device=dev, generator=g, dtype=torch.int64)].to(torch.int32)
    counts = torch.bincount(Sl, minlength=sigma)
    k = (torch.rand(m, device=dev, generator=g) * counts[c.long()]).long() + 1
    got = B.access(img, pos[:1 << 16], stream).to(torch.int64)
    assert torch.equal(got, Sl[pos[:1 << 16]]), "access differs from S"
    kinds = {"access": lambda: B.access(img, pos, stream), "rank": lambda: B.rank(img, c, pos, stream),
             "select": lambda: B.select(img, c, k, stream)}
    out = {"queries_per_batch": m, "levels": levels, "image_bytes": img.numel()}
    cached = img.numel() < (256 << 20)
    for name, fn in kinds.items():
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        lines = m * levels * 2 * 64
        out[name] = {"queries_per_s": round(m / dt, 1), "ms_per_batch": round(dt * 1e3, 3),
                     "line_GBps": round(lines / dt / 1e9, 1)}
        if cached:
            out[name]["cache_resident"] = True
        else:
            out[name]["frac"] = round(lines / dt / 1e9 / HBM_PEAK_GBPS, 4)
    return out


def info_passes(info):
    return -(-info.nlevels // info.tau)


def dary_huffman_codes(counts, D):
    """the shape of a Huffman-shaped d-ary tree (its input, prepared on the
    host): d-ary Huffman code lengths in digits (zero-weight dummies bring the
    leaf count to 1 mod d-1, the d lightest subtrees merge, ties by creation
    order) and canonical codewords in (length, symbol) order"""
    import heapq
    d = 1 << D
    present = [s for s in range(len(counts)) if counts[s]]
    lens = np.zeros(len(counts), dtype=np.uint32)
    if len(present) == 1:
        lens[present[0]] = 1
    else:
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
            lens[members] += 1
            heapq.heappush(heap, (w, t, members))
            t += 1
    codes = np.zeros(len(counts), dtype=np.uint64)
    code, prev = 0, None
    for l, s in sorted((int(l), s) for s, l in enumerate(lens) if l):
        if prev is not None:
            code = (code + 1) * d ** (l - prev)
        codes[s] = code
        prev = l
    return codes, lens


def tree_kernel_bytes(name, info, sym_bytes, kind):
    """compulsory bytes of all launches of one kernel in one tree build, or
    None for a kernel without a stated figure.  The tree is gathered from the
    levels of a wavelet matrix over its keys (the symbols, or the codewords
    padded to the longest code for the shaped tree)."""
    n = int(info.n)
    K = int(info.key_bits)
    D = int(info.arity_log2) if (kind == 4 or (kind == 3 and int(info.arity_log2) >= 2)) else 1
    key_w = 4 if kind == 3 else sym_bytes
    tree_bits = sum(int(info.level_n[l]) * D for l in range(info.nlevels))
    # the matrix whose passes are timed as "wm_pass" / "wm_hist": (symbols,
    # key bits, key width, pass width).  A shaped tree split at h1 bits builds
    # it over the top h1 code bits of every symbol (16-bit keys); its second
    # matrix, over the whole codes of the long-code symbols, runs on a side
    # stream and is timed as one entry ("side_matrix")
    h1 = int(info.split_bits)
    mats = [(n, h1, 2, int(info.tau))] if h1 else [(n, K, key_w, int(info.tau))]
    if name == "wm_pass":
        # the same rule as the matrix build: the first pass reads its keys
        # once and every pass writes its levels' bits once (the matrix levels
        # carry exactly the tree's bits, in another order of runs); the
        # compacted keys between passes are intermediate
        total = 0
        for m, L, in_w, tau in mats:
            for l0 in range(0, L, tau):
                t = min(tau, L - l0)
                total += (m * in_w if l0 == 0 else 0) + t * ((m + 63) // 64) * 8
        return total
    if name == "wm_hist":            # histograms read S (first pass) once
        return sum(m * w for m, L, w, tau in mats)
    if name == "tree_perm":          # write the tree levels once (reading the matrix runs is intermediate)
        return tree_bits // 8
    if name == "tree_digits":        # write one digit level per digit level (its matrix reads are intermediate)
        return info.nlevels * (n * D // 8)
    if name == "tree_keys":          # read S once (the codes it writes are intermediate)
        return n * sym_bytes
    if name == "lw_emit":            # level by level: level 0 reads S, every level's digits written once
        return n * sym_bytes + sum((int(info.level_n[l]) * D + 63) // 64 * 8 for l in range(info.nlevels))
    return None


def bench_tree(args):
    """C1 (balanced tree, 2^20 uint8, sigma 256), C3 Huffman-shaped (2^26
    uint16, sigma 4096, geometric 0.01) or C3 4-ary tree"""
    import torch
    from paper_1610_03524_amd import binding as B
    from paper_1610_03524_amd import inputs
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if args.workload == "c1":
        Sn = inputs.c1_uniform()
        sigma, kind, D, name = 256, B.KIND_WT, 0, "C1 balanced wavelet tree: n=2^20 uint8, sigma=256, uniform"
        St = torch.from_numpy(Sn).to(dev)
    else:
        Sn = inputs.c3_geometric()
        sigma = 4096
        St = torch.from_numpy(Sn.view(np.int16)).to(dev)
        if args.workload == "c3h":
            kind, D, name = B.KIND_SHAPED, 0, "C3 Huffman-shaped wavelet tree: n=2^26 uint16, sigma=4096, geometric(0.01)"
        elif args.workload == "c3hm":
            kind, D, name = (B.KIND_SHAPED, 2, "C3 Huffman-shaped 4-ary wavelet tree: n=2^26 uint16, sigma=4096, "
                                               "geometric(0.01), 4-ary Huffman codewords")
        else:
            kind, D, name = B.KIND_MULTIARY, 2, "C3 4-ary wavelet tree: n=2^26 uint16, sigma=4096, geometric(0.01)"
    n, sym = Sn.size, Sn.itemsize
    codes = lens = counts = None
    if kind == B.KIND_SHAPED:
        counts = B.symbol_counts(St, sigma).cpu().numpy().astype(np.uint64)
        codes, lens = B.huffman_codes(counts) if D < 2 else dary_huffman_codes(counts, D)
    tune = B.make_tuning()
    prof_tune = B.make_tuning(flags=B.FLAG_PROFILE)
    shape = B.make_shape(D, codes, lens, counts) if (D or codes is not None) else None
    info = B.plan(kind, n, sigma, sym, shape, tune)
    out = torch.empty(info.out_bytes, dtype=torch.uint8, device=dev)
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device=dev)

    def build_with(tn):
        rc = B.build_into(kind, St, sigma, out, ws, shape, tn, stream)
        if rc != 0:
            raise RuntimeError(B.strerror(rc))

    for _ in range(args.warmup):
        build_with(tune)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        build_with(tune)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    assert B.check(out, stream) == B.WT_OK
    prof = profiled_kernels(B, lambda: build_with(prof_tune), args.steps, stream)
    dom = max((k for k in prof if tree_kernel_bytes(k, info, sym, kind) is not None), key=lambda k: prof[k][1])
    dom_ms = prof[dom][1] / prof[dom][0]
    dom_bytes = tree_kernel_bytes(dom, info, sym, kind) / (prof[dom][0] / args.steps)
    balg = algorithmic_bytes(info, n, sym)
    t = ms / 1e3
    line = {
        "metric": METRIC, "value": round(n * sym / t / 1e9, 3), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u16" if sym == 2 else "u8", "data": "synthetic",
        "config": {"workload": name, "n": n, "sigma": sigma, "levels": info.nlevels,
                   "path": {"c1": "one pass of the matrix passes straight into tree order (domain decomposition)",
                            "c3h": "wavelet-matrix passes over the padded codewords (split at 16 bits), runs moved "
                                   "to tree order",
                            "c3m": "wavelet-matrix passes over the keys, 2-bit digits assembled, runs moved to "
                                   "tree order",
                            "c3hm": "level by level over the 2-bit digits of the codewords"}[args.workload]},
        "symbol_levels_per_s": round(symbol_levels(info) / t, 1),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(dom_bytes / (dom_ms / 1e3) / 1e9, 2),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(dom_bytes / (dom_ms / 1e3) / 1e9 / HBM_PEAK_GBPS, 4), "traffic": None,
                     "alg_bytes_per_launch": int(dom_bytes), "avg_launch_ms": round(dom_ms, 4)},
        "build_roofline": {"alg_bytes": balg, "achieved": round(balg / t / 1e9, 2),
                           "frac": round(balg / t / 1e9 / HBM_PEAK_GBPS, 4)},
        "kernel_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in sorted(prof.items())},
        "kernel_timing": KERNEL_TIMING,
    }
    line["queries"] = query_rates(out, St, n, sigma, info.nlevels, stream, m=1 << 20)
    if not args.no_cpu_baseline:
        import oracle
        okind = {B.KIND_WT: oracle.KIND_WT, B.KIND_SHAPED: oracle.KIND_SHAPED, B.KIND_MULTIARY: oracle.KIND_MULTI}[kind]
        line["cpu_baseline"] = cpu_baseline_oracle(okind, Sn, sigma, D, codes, lens)
    print(json.dumps(line), flush=True)


def bench_batch(args):
    """C4: wavelet matrices of 8192 uint32 sequences (n log-uniform in
    [2^10, 2^22], sigma log-uniform in [4, 2^20]); one batched build against a
    loop of per-sequence wm_build calls on one stream"""
    import torch
    from paper_1610_03524_amd import binding as B
    from paper_1610_03524_amd import inputs, tune as T
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    ns, sig, children = inputs.c4_sizes()
    k = min(args.limit, len(ns))
    ns, sig = ns[:k], sig[:k]
    # one buffer, every sequence starting on a 16-byte boundary (the library's
    # alignment rule for S)
    offs = np.concatenate([[0], np.cumsum((ns + 3) // 4 * 4)])
    total = int(ns.sum())   # symbols (the padding is not input)
    t_gen = time.perf_counter()
    big = torch.empty(int(offs[-1]), dtype=torch.int32, device=dev)
    for i in range(k):
        S = inputs.c4_sequence(int(ns[i]), int(sig[i]), children[i])
        big[int(offs[i]):int(offs[i]) + S.size].copy_(torch.from_numpy(S.view(np.int32)), non_blocking=False)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    infos = [B.plan(B.KIND_WM, int(ns[i]), int(sig[i]), 4) for i in range(k)]
    out_off = np.concatenate([[0], np.cumsum([(inf.out_bytes + 255) // 256 * 256 for inf in infos])])
    images = torch.empty(int(out_off[-1]), dtype=torch.uint8, device=dev)
    descs = []
    for i in range(k):
        d = B.wt_seq_desc()
        d.S = big.data_ptr() + 4 * int(offs[i])
        d.n, d.sigma, d.sym_bytes = int(ns[i]), int(sig[i]), 4
        d.out, d.out_bytes = images.data_ptr() + int(out_off[i]), infos[i].out_bytes
        d.tau = T.choose_tau(int(ns[i]), int(sig[i]))
        descs.append(d)
    descs = B.desc_array(descs)   # marshalled once, outside the timed calls
    batch_tile = T.choose_batch_tile()
    batch_tune = B.make_tuning(tile=batch_tile)
    need = B.batch_plan(B.KIND_WM, descs, batch_tune)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    single_ws = torch.empty(max(inf.workspace_bytes for inf in infos), dtype=torch.uint8, device=dev)

    def batched():
        rc = B.batch_build(B.KIND_WM, descs, ws, batch_tune, stream=stream)
        if rc != 0:
            raise RuntimeError(B.strerror(rc))

    lib = B.lib()

    tunings = [B.make_tuning(tau=d.tau) for d in descs]
    import ctypes

    def plain():
        for d, tn in zip(descs, tunings):
            rc = lib.wm_build(d.S, d.n, d.sigma, 4, None, ctypes.byref(tn), d.out, d.out_bytes,
                              single_ws.data_ptr(), single_ws.numel(), B._stream(stream))
            if rc != 0:
                raise RuntimeError(B.strerror(rc))

    # the same loop spread round-robin over 4 streams, one workspace each
    streams = [torch.cuda.Stream() for _ in range(4)]
    ws4 = [torch.empty_like(single_ws) for _ in streams]

    def plain4():
        for q, (d, tn) in enumerate(zip(descs, tunings)):
            st, w = streams[q % 4], ws4[q % 4]
            rc = lib.wm_build(d.S, d.n, d.sigma, 4, None, ctypes.byref(tn), d.out, d.out_bytes,
                              w.data_ptr(), w.numel(), B._stream(st))
            if rc != 0:
                raise RuntimeError(B.strerror(rc))

    res, spread = {}, {}
    reps = max(5, args.steps // 4)
    for name, fn in (("batched", batched), ("plain", plain), ("plain_4_streams", plain4)):
        fn()
        torch.cuda.synchronize()
        each = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            each.append(time.perf_counter() - t0)
        res[name] = float(np.median(each))
        spread[name] = [round(float(v), 4) for v in np.percentile(each, [10, 90])]
    # kernel launches of one batch, from the library's own per-kernel counters
    B.profile_read()
    rc = B.batch_build(B.KIND_WM, descs, ws, B.make_tuning(tile=batch_tile, flags=B.FLAG_PROFILE), stream=stream)
    if rc != 0:
        raise RuntimeError(B.strerror(rc))
    torch.cuda.synchronize()
    launches = {name: int(v[0]) for name, v in sorted(B.profile_read().items())}
    # the same batch captured once in a HIP graph and replayed: one graph
    # launch per batch, and the images equal the eager ones
    batched()
    torch.cuda.synchronize()
    eager_images = images.clone()
    gs = torch.cuda.Stream()
    gs.wait_stream(stream)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gs, capture_error_mode="relaxed"):
        rc = B.batch_build(B.KIND_WM, descs, ws, batch_tune, stream=gs)
    if rc != 0:
        raise RuntimeError(B.strerror(rc))
    images.fill_(0xA5)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    if not torch.equal(images, eager_images):
        raise RuntimeError("graph-replayed batch differs from the eager batch")
    del eager_images
    each = []
    for _ in range(reps):
        t0 = time.perf_counter()
        graph.replay()
        torch.cuda.synchronize()
        each.append(time.perf_counter() - t0)
    res["graph"] = float(np.median(each))
    spread["graph"] = [round(float(v), 4) for v in np.percentile(each, [10, 90])]
    balg = sum(4 * int(ns[i]) + infos[i].out_bytes for i in range(k))
    tb, tp, t4, tg = res["batched"], res["plain"], res["plain_4_streams"], res["graph"]
    line = {
        "metric": METRIC, "value": round(total * 4 / tb / 1e9, 3), "unit": "GB/s", "n_gpus": 1,
        "steps": reps, "warmup": 1, "ms_per_step": round(tb * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"C4 batched wavelet matrices: {k} uint32 sequences, n log-uniform [2^10, 2^22], "
                               f"sigma log-uniform [4, 2^20]", "symbols": total},
        "batched": {"s": round(tb, 4), "p10_p90_s": spread["batched"], "builds_per_s": round(k / tb, 1),
                    "input_GBps": round(total * 4 / tb / 1e9, 2),
                    "build_roofline_frac": round(balg / tb / 1e9 / HBM_PEAK_GBPS, 4),
                    "tiles_per_chunk": batch_tile or "automatic",
                    "kernel_launches": sum(launches.values()), "launches_by_kernel": launches},
        "batched_graph_replay": {"s": round(tg, 4), "p10_p90_s": spread["graph"], "builds_per_s": round(k / tg, 1),
                                 "input_GBps": round(total * 4 / tg / 1e9, 2), "graph_launches": 1,
                                 "images_equal_eager": True},
        "plain": {"s": round(tp, 4), "p10_p90_s": spread["plain"], "builds_per_s": round(k / tp, 1),
                  "input_GBps": round(total * 4 / tp / 1e9, 2)},
        "plain_4_streams": {"s": round(t4, 4), "p10_p90_s": spread["plain_4_streams"],
                            "builds_per_s": round(k / t4, 1), "input_GBps": round(total * 4 / t4 / 1e9, 2)},
        "timing": f"median of {reps} timed repetitions of each form after one untimed one",
        "speedup_batched_vs_plain": round(tp / tb, 3),
        "speedup_batched_vs_plain_4_streams": round(t4 / tb, 3),
        "input_generation_s": round(t_gen, 1),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_batch(ns, sig, children)
    print(json.dumps(line), flush=True)


def cpu_baseline_batch(ns, sig, children, target_s=10.0):
    """the oracle over the first C4 sequences on a pool of host threads (one
    sequence per task; the C library releases the interpreter while it runs),
    one per core this process may use up to the machine's CPU share, and
    single-threaded on the same sample; GB/s of input"""
    import concurrent.futures as cf
    import oracle
    from paper_1610_03524_amd import inputs
    cpu = host_cpu()
    threads = cpu["pool_threads"]
    seqs, total = [], 0
    for i in range(len(ns)):
        seqs.append((inputs.c4_sequence(int(ns[i]), int(sig[i]), children[i]), int(sig[i])))
        total += int(ns[i])
        if total >= 1 << 26:
            break
    nbytes = sum(S.size * 4 for S, _ in seqs)
    t = time.perf_counter()
    for S, sg in seqs:
        oracle.build_image(oracle.KIND_WM, S, sg)
    t1 = time.perf_counter() - t
    t = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda a: oracle.build_image(oracle.KIND_WM, *a), seqs))
    tp = time.perf_counter() - t
    return {"value": round(nbytes / tp / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "single_thread_GBps": round(nbytes / t1 / 1e9, 4),
            "sample": f"first {len(seqs)} C4 sequences ({nbytes // 4} symbols): {tp:.1f} s on {threads} "
                      f"threads, {t1:.1f} s on one", **cpu}



def bench_serve(args):
    """C5: Poisson build requests (the C4 size mix) and query batches of 2^16
    mixed access/rank/select on resident structures; continuous batching
    against a plain one-request-at-a-time queue; p50/p99 latency and
    throughput per arrival rate"""
    import threading
    import torch
    from paper_1610_03524_amd import inputs, serve, tune as T
    P = min(args.limit, 512)
    ns, sig, children = inputs.c4_sizes()
    host = [(inputs.c4_sequence(int(ns[i]), int(sig[i]), children[i]), int(sig[i])) for i in range(P)]
    dev = [(torch.from_numpy(S.view(np.int32)).cuda(), sg) for S, sg in host]
    rng = np.random.default_rng(5)
    qb = [serve.make_query_batch(S, 1 << 16, rng) for S, _ in host]
    torch.cuda.synchronize()
    rows = []
    # warm-up of both modes (first launches of the single and the batched
    # build, allocator, streams), not recorded
    rates = [("warmup", 20000.0, 0.25)] + [("run", float(r), max(args.horizon, args.min_builds / float(r)))
                                         for r in args.rates.split(",")]
    for tag, rate, horizon in rates:
        bt, ids, qt = inputs.c5_requests(rate, horizon, seed=5, count=P)
        events = sorted([(t, "b", int(i)) for t, i in zip(bt, ids)] + [(t, "q", -1) for t in qt])
        for mode in args.modes.split(","):
            srv = serve.WaveletServer(dev, hbm_budget=64 << 30, ws_bytes=4 << 30, mode=mode, tau_of=T.choose_tau,
                                      batch_tile=T.choose_batch_tile())
            srv.start()
            pick = np.random.default_rng(int(rate))
            t0 = time.perf_counter()
            skipped = 0
            for t, kind, i in events:
                dt = t0 + t - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                if kind == "b":
                    srv.submit_build(i)
                else:
                    res = srv.resident_ids()
                    if not res:
                        skipped += 1
                        continue
                    tgt = res[pick.integers(0, len(res))]
                    srv.submit_query(tgt, qb[tgt])
            deadline = time.perf_counter() + 60
            while any(not r.done for r in srv.all_reqs) and time.perf_counter() < deadline:
                time.sleep(0.002)
            t_end = time.perf_counter()
            srv.close()
            bl, ql = srv.latencies("build"), srv.latencies("query")
            unfinished = sum(1 for r in srv.all_reqs if not r.done)
            if tag == "warmup":
                del srv
                continue
            rows.append({"rate": rate, "mode": mode, "horizon_s": round(horizon, 2), "builds": int(len(bl)),
                         "query_batches": int(len(ql)),
                         "build_p50_ms": serve.percentile_ms(bl, 50), "build_p99_ms": serve.percentile_ms(bl, 99),
                         "query_p50_ms": serve.percentile_ms(ql, 50), "query_p99_ms": serve.percentile_ms(ql, 99),
                         "builds_per_s": round(len(bl) / (t_end - t0), 1),
                         "queries_per_s": round(len(ql) * (1 << 16) / (t_end - t0), 1),
                         "mean_batch": round(float(np.mean(srv.batches)), 2) if srv.batches else None,
                         "unfinished": unfinished, "queries_skipped_no_structure": skipped})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
            del srv
            torch.cuda.empty_cache()
    print(json.dumps({
        "metric": "serving p50/p99 latency and throughput (continuous batching vs plain queue)",
        "workload": f"C5: Poisson builds from the C4 mix over a pool of {P} sequences, query batches of 2^16 "
                    f"mixed access/rank/select at max(10, rate/10)/s, max({args.horizon} s, {args.min_builds} "
                    f"arrivals) per rate, HBM budget 64 GiB",
        "n_gpus": 1, "data": "synthetic", "rows": rows}), flush=True)


if __name__ == "__main__":
    main()
