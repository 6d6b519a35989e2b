"""Serving loop: continuous batching of wavelet-matrix builds and queries.

Requests arrive over time: builds (a sequence already resident in HBM) and
query batches (access / rank / select on a built structure).  Two workers
share the GPU:

* the build worker takes every build that has arrived, admits them while
  their images fit the HBM budget (evicting the least recently used built
  structures when needed) and the batch workspace, and builds them with one
  wt_batch_build on its own stream; requests arriving meanwhile form the
  next batch, so batches grow with the load (continuous batching);
* the query worker launches each query batch on a second stream as soon as
  it arrives, so queries overlap with builds on the device.

The "plain" mode is the baseline: one worker serving every request alone, in
arrival order (wm_build or one query launch, then wait).

Every result is the same as when the request runs alone: a build writes the
image wm_build writes, and a query reads an image that is complete before
the query is launched (the query worker only sees structures whose build has
finished).  Latency = completion time - arrival time.

A request that cannot be served fails alone: its error code is set and the
worker goes on.  A sequence the library refuses (bad sigma, too long) fails
at admission with the plan's code; a built image whose status word reports a
symbol >= sigma fails with WT_ERANGE and is not made resident; an exception
while building or querying fails the requests it was serving.
"""
from __future__ import annotations

import collections
import ctypes
import sys
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import binding as B


SWITCH_INTERVAL_S = 2e-4


@dataclass
class Request:
    rid: int
    kind: str                  # "build" or "query"
    arrival: float             # host clock (perf_counter) when it arrived
    seq: int = -1              # build: sequence index; query: target structure
    qtype: str = ""            # "mixed": access, rank and select launches
    args: tuple = ()           # device tensors of the queries
    done: float = 0.0
    result: object = None
    error: int = 0


@dataclass
class Structure:
    image: object              # device uint8 tensor
    nbytes: int
    last_use: float = 0.0


class WaveletServer:
    def __init__(self, seqs, hbm_budget: int, ws_bytes: int = 1 << 30, max_batch: int = 4096,
                 mode: str = "continuous", tau_of=None):
        """seqs: list of (device int tensor S, sigma) the builds refer to."""
        import torch
        self.torch = torch
        self.seqs = seqs
        self.budget = hbm_budget
        self.mode = mode
        self.max_batch = max_batch
        self.tau_of = tau_of or (lambda n, sigma: 0)
        self.build_stream = torch.cuda.Stream()
        self.query_stream = torch.cuda.Stream() if mode == "continuous" else self.build_stream
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        self.resident: dict[int, Structure] = {}
        self.used = 0
        self.lock = threading.Lock()
        # one condition per worker on the shared lock, so that a submitted
        # build wakes only the build worker and a query only the query worker
        self.build_cv = threading.Condition(self.lock)
        self.query_cv = threading.Condition(self.lock) if mode == "continuous" else self.build_cv
        self.builds = collections.deque()
        self.queries = collections.deque()
        self.all_reqs: list[Request] = []
        self.closing = False
        self.batches: list[int] = []
        self.threads = []
        self._cost_cache = {}

    # ---- submission ------------------------------------------------------------
    def submit_build(self, seq: int) -> Request:
        with self.lock:
            r = Request(len(self.all_reqs), "build", time.perf_counter(), seq=seq)
            self.all_reqs.append(r)
            (self.builds if self.mode == "continuous" else self.queries).append(r)
            self.build_cv.notify()
            return r

    def submit_query(self, target: int, args) -> Request:
        """one batch of mixed queries on structure `target`:
        args = (pos, rank symbols, rank positions, select symbols, select ranks)"""
        with self.lock:
            r = Request(len(self.all_reqs), "query", time.perf_counter(), seq=target, qtype="mixed", args=args)
            self.all_reqs.append(r)
            self.queries.append(r)
            self.query_cv.notify()
            return r

    def is_resident(self, sid: int) -> bool:
        with self.lock:
            return sid in self.resident

    def resident_ids(self):
        with self.lock:
            return list(self.resident)

    # ---- workers ------------------------------------------------------------------
    def start(self):
        # Python hands the interpreter between threads every switch interval
        # (5 ms by default); a worker woken while another thread runs Python
        # code would wait that long, so the server shortens it while running
        self._switch = sys.getswitchinterval()
        sys.setswitchinterval(SWITCH_INTERVAL_S)
        if self.mode == "continuous":
            self.threads = [threading.Thread(target=self._build_loop, daemon=True),
                            threading.Thread(target=self._query_loop, daemon=True)]
        else:
            self.threads = [threading.Thread(target=self._plain_loop, daemon=True)]
        for t in self.threads:
            t.start()

    def close(self):
        with self.lock:
            self.closing = True
            self.build_cv.notify_all()
            self.query_cv.notify_all()
        for t in self.threads:
            t.join()
        sys.setswitchinterval(self._switch)

    def _costs(self, seq):
        """(image bytes, batch-workspace bytes) of one sequence, cached; the
        workspace of a batch is at most the sum over its sequences"""
        c = self._cost_cache.get(seq)
        if c is None:
            S, sigma = self.seqs[seq]
            tau = self.tau_of(S.numel(), sigma)
            ob = B.plan(B.KIND_WM, S.numel(), sigma, S.element_size(), tune=B.make_tuning(tau=tau)).out_bytes
            # sizing only: any non-null, 16-byte aligned addresses pass the plan's checks
            d = B.wt_seq_desc()
            d.S, d.n, d.sigma, d.sym_bytes, d.out, d.out_bytes, d.tau = 256, S.numel(), sigma, S.element_size(), 256, ob, tau
            c = (ob, B.batch_plan(B.KIND_WM, [d]))
            self._cost_cache[seq] = c
        return c

    def _image_bytes(self, seq):
        return self._costs(seq)[0]

    def _evict_for(self, need, keep):
        """free least recently used structures until `need` more bytes fit"""
        while self.used + need > self.budget:
            victims = [k for k in self.resident if k not in keep]
            if not victims:
                return False
            k = min(victims, key=lambda v: self.resident[v].last_use)
            self.used -= self.resident.pop(k).nbytes
        return True

    def _admit(self):
        """builds that fit the budget and the batch workspace, in arrival order"""
        take, descs, imgs, nbytes = [], [], [], []
        ws_need = 0
        while self.builds and len(take) < self.max_batch:
            r = self.builds[0]
            S, sigma = self.seqs[r.seq]
            try:
                ob, wsb = self._costs(r.seq)
            except B.WaveletError as e:
                self.builds.popleft()
                r.error, r.done = e.code, time.perf_counter()
                continue
            if ob > self.budget:
                self.builds.popleft()
                r.error, r.done = B.WT_ENOSPC, time.perf_counter()
                continue
            if ws_need + wsb > self.ws.numel():
                if not take:
                    self.builds.popleft()
                    r.error, r.done = B.WT_ENOSPC, time.perf_counter()
                    continue
                break
            if not self._evict_for(ob + sum(nbytes), keep={q.seq for q in take}):
                break
            d = B.wt_seq_desc()
            d.S, d.n, d.sigma, d.sym_bytes = S.data_ptr(), S.numel(), sigma, S.element_size()
            d.tau = self.tau_of(S.numel(), sigma)
            with self.torch.cuda.stream(self.build_stream):
                img = self.torch.empty(ob, dtype=self.torch.uint8, device="cuda")
            d.out, d.out_bytes = img.data_ptr(), ob
            ws_need += wsb
            self.builds.popleft()
            take.append(r)
            descs.append(d)
            imgs.append(img)
            nbytes.append(ob)
        return take, descs, imgs, nbytes

    def _statuses(self, imgs, rc):
        """per-image status after a build call that returned rc: the call's
        code if it failed, else WT_ERANGE for an image whose header status word
        (what wt_check reads) reports a symbol >= sigma"""
        if rc != B.WT_OK:
            return [rc] * len(imgs)
        if len(imgs) == 1:
            return [B.check(imgs[0], stream=self.build_stream)]
        torch = self.torch
        with torch.cuda.stream(self.build_stream):
            words = torch.cat([img[36:40] for img in imgs]).view(torch.int32).cpu().numpy()
        return [B.WT_OK if w == 0 else B.WT_ERANGE for w in words]

    def _launch_builds(self, descs, imgs):
        torch = self.torch
        with torch.cuda.stream(self.build_stream):
            if len(descs) == 1:
                # a batch of one: the single-sequence build has less set-up
                d = descs[0]
                tn = B.make_tuning(tau=d.tau)
                rc = B.lib().wm_build(d.S, d.n, d.sigma, d.sym_bytes, None, ctypes.byref(tn), d.out,
                                      d.out_bytes, self.ws.data_ptr(), self.ws.numel(),
                                      B._stream(self.build_stream))
            else:
                rc = B.batch_build(B.KIND_WM, descs, self.ws, stream=self.build_stream)
            self.build_stream.synchronize()
        return self._statuses(imgs, rc)

    def _build_loop(self):
        while True:
            with self.lock:
                while not self.builds and not self.closing:
                    self.build_cv.wait()
                if self.closing and not self.builds:
                    return
                take, descs, imgs, nbytes = self._admit()
                self.used += sum(nbytes)
            if not take:
                time.sleep(0.0005)
                continue
            try:
                codes = self._launch_builds(descs, imgs)
            except Exception as e:   # fail this batch, keep serving
                codes = [getattr(e, "code", B.WT_EHIP)] * len(take)
            t = time.perf_counter()
            with self.lock:
                self.batches.append(len(take))
                for r, img, nb, rc in zip(take, imgs, nbytes, codes):
                    r.done, r.error = t, rc
                    if rc == B.WT_OK:
                        old = self.resident.pop(r.seq, None)
                        if old is not None:
                            self.used -= old.nbytes
                        self.resident[r.seq] = Structure(img, nb, t)
                    else:
                        self.used -= nb

    def _take_structure(self, r, stream):
        """(under the lock) the structure a query reads, or None.  The
        caller's reference keeps the image alive if it is evicted while the
        query runs; record_stream keeps its memory from being reused before
        the query stream is past this point."""
        st = self.resident.get(r.seq)
        if st is not None:
            st.last_use = time.perf_counter()
            st.image.record_stream(stream)
        return st

    def _run_query(self, r, st, stream):
        """launch one mixed batch: args = (pos, rank c, rank i, select c, select k)"""
        pos, rc, ri, sc, sk = r.args
        with self.torch.cuda.stream(stream):
            r.result = (B.access(st.image, pos, stream=stream), B.rank(st.image, rc, ri, stream=stream),
                        B.select(st.image, sc, sk, stream=stream))

    def _serve_query(self, r, st, stream):
        if st is None:
            r.error = B.WT_EINVAL
            return
        try:
            self._run_query(r, st, stream)
            stream.synchronize()
        except Exception as e:   # fail this query, keep serving
            r.result, r.error = None, getattr(e, "code", B.WT_EHIP)

    def _query_loop(self):
        while True:
            with self.lock:
                while not self.queries and not self.closing:
                    self.query_cv.wait()
                if self.closing and not self.queries:
                    return
                r = self.queries.popleft()
                st = self._take_structure(r, self.query_stream)
            self._serve_query(r, st, self.query_stream)
            r.done = time.perf_counter()

    def _plain_build(self, r):
        torch = self.torch
        S, sigma = self.seqs[r.seq]
        try:
            tn = B.make_tuning(tau=self.tau_of(S.numel(), sigma))
            info = B.plan(B.KIND_WM, S.numel(), sigma, S.element_size(), tune=tn)
        except B.WaveletError as e:
            r.error, r.done = e.code, time.perf_counter()
            return
        ob = info.out_bytes
        if ob > self.budget or self.ws.numel() < info.workspace_bytes:
            r.error, r.done = B.WT_ENOSPC, time.perf_counter()
            return
        with self.lock:
            self._evict_for(ob, keep=set())
            self.used += ob
        try:
            with torch.cuda.stream(self.build_stream):
                img = torch.empty(ob, dtype=torch.uint8, device="cuda")
            rc = B.lib().wm_build(S.data_ptr(), S.numel(), sigma, S.element_size(), None,
                                  ctypes.byref(tn), img.data_ptr(), ob, self.ws.data_ptr(),
                                  self.ws.numel(), B._stream(self.build_stream))
            self.build_stream.synchronize()
            r.error = self._statuses([img], rc)[0]
        except Exception as e:   # fail this build, keep serving
            r.error = getattr(e, "code", B.WT_EHIP)
        r.done = time.perf_counter()
        with self.lock:
            if r.error == B.WT_OK:
                old = self.resident.pop(r.seq, None)
                if old is not None:
                    self.used -= old.nbytes
                self.resident[r.seq] = Structure(img, ob, r.done)
            else:
                self.used -= ob

    def _plain_loop(self):
        while True:
            with self.lock:
                while not self.queries and not self.closing:
                    self.build_cv.wait()
                if self.closing and not self.queries:
                    return
                r = self.queries.popleft()
            if r.kind == "build":
                self._plain_build(r)
            else:
                with self.lock:
                    st = self._take_structure(r, self.build_stream)
                self._serve_query(r, st, self.build_stream)
                r.done = time.perf_counter()

    # ---- results ----------------------------------------------------------------------
    def latencies(self, kind):
        return np.array([r.done - r.arrival for r in self.all_reqs if r.kind == kind and r.done and not r.error])


def percentile_ms(x, q):
    return round(float(np.percentile(x, q)) * 1e3, 3) if len(x) else None


def make_query_batch(S: np.ndarray, m: int, rng):
    """m mixed queries on sequence S (host copy): a third each of access at
    uniform positions, rank of symbols drawn from S at uniform positions, and
    select of symbols drawn from S with k uniform in [1, occurrences]"""
    import torch
    n = S.size
    a = m // 3
    pos = rng.integers(0, n, a).astype(np.int64)
    rc = S[rng.integers(0, n, a)].astype(np.int64)
    ri = rng.integers(0, n, a).astype(np.int64)
    sc = S[rng.integers(0, n, m - 2 * a)].astype(np.int64)
    vals, cnts = np.unique(S, return_counts=True)
    cnt = cnts[np.searchsorted(vals, sc)]
    sk = (rng.random(sc.size) * cnt).astype(np.int64) + 1
    dev = lambda x, dt: torch.from_numpy(x.astype(dt)).cuda()
    return (dev(pos, np.int64), dev(rc, np.int32), dev(ri, np.int64), dev(sc, np.int32), dev(sk, np.int64))
