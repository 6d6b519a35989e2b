"""Autotuner of the pass width tau and of the chunk size of wavelet-matrix builds.

Neither changes the image (tested), so both are pure speed choices.  For a
bucket (L = key bits, lg = ceil(log2 n)) the tuner times wm_build on a uniform
synthetic sequence of that shape: every candidate tau with the automatic
chunking first, then, with the fastest tau, every candidate chunk size in tiles
of 8192 keys (the ``tile`` field of wt_tuning; 0 = one chunk per resident
workgroup).  Batched builds get one chunk size for the whole batch, timed on
the first sequences of the batched configuration's size mix.  The winners are
cached in ``tune_cache.json`` next to this file, keyed by the GPU
architecture; ``choose_tuning`` and ``choose_batch_tile`` read the cache (0 =
let the library decide when there is no entry).

    python -m paper_1610_03524_amd.tune [--max-lg 28] [--batch-limit 2048]
"""
from __future__ import annotations

import argparse
import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache.json")
ARCH = "gfx950"
TILE_KEYS = 8192
TAU_CANDIDATES = (2, 3, 4, 5, 6, 7, 8)
TILE_CANDIDATES = (0, 1, 2, 4, 8, 16, 32, 64)

_cache = None


def bucket(n: int, sigma: int) -> str:
    L = max(1, (sigma - 1).bit_length())
    lg = max(0, math.ceil(math.log2(max(n, 1))))
    return f"{ARCH}:L{L}:n{lg}"


def batch_key() -> str:
    return f"{ARCH}:batch"


def load_cache() -> dict:
    global _cache
    if _cache is None:
        _cache = {}
        if os.path.exists(CACHE):
            with open(CACHE) as f:
                _cache = json.load(f)
    return _cache


def choose_tuning(n: int, sigma: int) -> tuple[int, int]:
    """(tau, tiles per chunk) of the bucket of (n, sigma); 0 = automatic"""
    e = load_cache().get(bucket(n, sigma), {})
    return int(e.get("tau", 0)), int(e.get("tile", 0))


def choose_tau(n: int, sigma: int) -> int:
    return choose_tuning(n, sigma)[0]


def choose_batch_tile() -> int:
    return int(load_cache().get(batch_key(), {}).get("tile", 0))


def _median_ms(run, reps: int) -> float:
    import torch
    for _ in range(2):
        run()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        run()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def time_build(S, sigma: int, tau: int, tile: int, reps: int = 5) -> float:
    import torch
    from . import binding as B
    tune = B.make_tuning(tau=tau, tile=tile)
    info = B.plan(B.KIND_WM, S.numel(), sigma, 4, tune=tune)
    out = torch.empty(info.out_bytes, dtype=torch.uint8, device="cuda")
    ws = torch.empty(max(info.workspace_bytes, 1), dtype=torch.uint8, device="cuda")

    def run():
        rc = B.build_into(B.KIND_WM, S, sigma, out, ws, tune=tune)
        if rc:
            raise RuntimeError(B.strerror(rc))
    return _median_ms(run, reps)


def tile_candidates(n: int) -> list[int]:
    """chunk sizes giving distinct chunk counts (0 = automatic first)"""
    tiles = max(1, -(-n // TILE_KEYS))
    seen, out = set(), [0]
    for t in TILE_CANDIDATES[1:]:
        if t > tiles:
            break
        k = -(-tiles // t)
        if k not in seen:
            seen.add(k)
            out.append(t)
    return out


def tune(min_L=2, max_L=20, min_lg=10, max_lg=28, step_lg=2, out=CACHE) -> dict:
    import torch
    cache = dict(load_cache())
    for L in range(min_L, max_L + 1, 2):
        for lg in range(min_lg, max_lg + 1, step_lg):
            n, sigma = 1 << lg, 1 << L
            S = torch.randint(0, sigma, (n,), dtype=torch.int32, device="cuda")
            taus = sorted({t for t in TAU_CANDIDATES if t <= L} | {min(8, L)})
            tt = {t: time_build(S, sigma, t, 0) for t in taus}
            tau = min(tt, key=tt.get)
            tl = {t: (tt[tau] if t == 0 else time_build(S, sigma, tau, t)) for t in tile_candidates(n)}
            tile = min(tl, key=tl.get)
            cache[bucket(n, sigma)] = {"tau": tau, "tile": tile, "ms": round(tl[tile], 4),
                                       "tried_tau": {str(k): round(v, 4) for k, v in tt.items()},
                                       "tried_tile": {str(k): round(v, 4) for k, v in tl.items()}}
            print(f"L={L} n=2^{lg}: tau={tau} tile={tile} ({tl[tile]:.3f} ms)", flush=True)
            del S
    with open(out, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return cache


def tune_batch(limit: int = 2048, out=CACHE) -> dict:
    """one chunk size for batched builds, timed on the first `limit`
    sequences of the batched configuration (per-sequence tau from the cache)"""
    import numpy as np
    import torch
    from . import binding as B
    from . import inputs
    ns, sig, children = inputs.c4_sizes()
    ns, sig = ns[:limit], sig[:limit]
    offs = np.concatenate([[0], np.cumsum((ns + 3) // 4 * 4)])
    big = torch.empty(int(offs[-1]), dtype=torch.int32, device="cuda")
    for i in range(len(ns)):
        S = inputs.c4_sequence(int(ns[i]), int(sig[i]), children[i])
        big[int(offs[i]):int(offs[i]) + S.size].copy_(torch.from_numpy(S.view(np.int32)))
    infos = [B.plan(B.KIND_WM, int(ns[i]), int(sig[i]), 4) for i in range(len(ns))]
    out_off = np.concatenate([[0], np.cumsum([(f.out_bytes + 255) // 256 * 256 for f in infos])])
    images = torch.empty(int(out_off[-1]), dtype=torch.uint8, device="cuda")
    descs = []
    for i in range(len(ns)):
        d = B.wt_seq_desc()
        d.S, d.n, d.sigma, d.sym_bytes = big.data_ptr() + 4 * int(offs[i]), int(ns[i]), int(sig[i]), 4
        d.out, d.out_bytes = images.data_ptr() + int(out_off[i]), infos[i].out_bytes
        d.tau = choose_tau(int(ns[i]), int(sig[i]))
        descs.append(d)
    descs = B.desc_array(descs)
    times = {}
    for tile in TILE_CANDIDATES:
        tune_ = B.make_tuning(tile=tile)
        ws = torch.empty(max(B.batch_plan(B.KIND_WM, descs, tune_), 1), dtype=torch.uint8, device="cuda")

        def run():
            rc = B.batch_build(B.KIND_WM, descs, ws, tune_)
            if rc:
                raise RuntimeError(B.strerror(rc))
        times[tile] = _median_ms(run, 5)
        print(f"batch of {len(ns)}: tile={tile} {times[tile]:.3f} ms", flush=True)
        del ws
    best = min(times, key=times.get)
    cache = dict(load_cache())
    cache[batch_key()] = {"tile": best, "ms": round(times[best], 4), "sequences": len(ns),
                          "tried_tile": {str(k): round(v, 4) for k, v in times.items()}}
    with open(out, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return cache


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-lg", type=int, default=28)
    ap.add_argument("--max-L", type=int, default=20)
    ap.add_argument("--batch-limit", type=int, default=2048)
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--skip-buckets", action="store_true")
    args = ap.parse_args()
    CACHE = args.out   # read and written from here on
    if not args.skip_buckets:
        tune(max_lg=args.max_lg, max_L=args.max_L, out=args.out)
    _cache = None   # the batch reads the per-bucket tau just written
    tune_batch(limit=args.batch_limit, out=args.out)
