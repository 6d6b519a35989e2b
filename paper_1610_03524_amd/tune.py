"""Autotuner of the pass width tau for wavelet-matrix builds.

The image does not depend on tau (tested), so tau is a pure speed choice.  For
a bucket (L = key bits, lg = ceil(log2 n)) the tuner times wm_build for every
candidate tau on a uniform synthetic sequence of that shape and keeps the
fastest; the winners are cached in ``tune_cache.json`` next to this file,
keyed by the GPU architecture.  ``choose_tau`` reads the cache (0 = let the
library decide when a bucket has no entry).

    python -m paper_1610_03524_amd.tune [--max-lg 22]
"""
from __future__ import annotations

import argparse
import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache.json")
ARCH = "gfx950"

_cache = None


def bucket(n: int, sigma: int) -> str:
    L = max(1, (sigma - 1).bit_length())
    lg = max(0, math.ceil(math.log2(max(n, 1))))
    return f"{ARCH}:L{L}:n{lg}"


def load_cache() -> dict:
    global _cache
    if _cache is None:
        _cache = {}
        if os.path.exists(CACHE):
            with open(CACHE) as f:
                _cache = json.load(f)
    return _cache


def choose_tau(n: int, sigma: int) -> int:
    return int(load_cache().get(bucket(n, sigma), {}).get("tau", 0))


def time_tau(n: int, sigma: int, tau: int, reps: int = 5) -> float:
    import torch
    from . import binding as B
    S = torch.randint(0, sigma, (n,), dtype=torch.int32, device="cuda")
    tune = B.make_tuning(tau=tau)
    info = B.plan(B.KIND_WM, n, sigma, 4, tune=tune)
    out = torch.empty(info.out_bytes, dtype=torch.uint8, device="cuda")
    ws = torch.empty(max(info.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    for _ in range(2):
        B.build_into(B.KIND_WM, S, sigma, out, ws, tune=tune)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        B.build_into(B.KIND_WM, S, sigma, out, ws, tune=tune)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(min_L=2, max_L=20, min_lg=10, max_lg=22, step_lg=2, out=CACHE) -> dict:
    cache = dict(load_cache())
    for L in range(min_L, max_L + 1, 2):
        for lg in range(min_lg, max_lg + 1, step_lg):
            n, sigma = 1 << lg, 1 << L
            cands = sorted({t for t in (2, 3, 4, 5, 6, 7, 8) if t <= L} | {min(8, L)})
            times = {t: time_tau(n, sigma, t) for t in cands}
            best = min(times, key=times.get)
            cache[bucket(n, sigma)] = {"tau": best, "ms": round(times[best], 4),
                                       "tried": {str(k): round(v, 4) for k, v in times.items()}}
            print(f"L={L} n=2^{lg}: tau={best} ({times[best]:.3f} ms)", flush=True)
    with open(out, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return cache


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-lg", type=int, default=22)
    ap.add_argument("--max-L", type=int, default=20)
    ap.add_argument("--out", default=CACHE)
    args = ap.parse_args()
    tune(max_lg=args.max_lg, max_L=args.max_L, out=args.out)
