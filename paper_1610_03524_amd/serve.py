"""Serving loop: continuous batching of wavelet-matrix builds and queries.

Requests arrive over time: builds (a sequence already resident in HBM) and
query batches (access / rank / select on a built structure).  One dispatcher
thread serves both, on two streams:

* builds: when no build batch is on the device, every build that has
  arrived is admitted while the images fit the HBM budget (evicting the least
  recently used built structures when needed) and the batch workspace, and
  launched with one wt_batch_build (wm_build for a batch of one); requests
  arriving meanwhile form the next batch, so batches grow with the load
  (continuous batching);
* queries: every query batch that has arrived is launched (before the builds
  that arrived with them) and one wait covers them all; while builds are on
  the device they go on the second stream, so queries overlap with builds
  and group up under load, otherwise on the build stream.

A lone request thus takes the same path as in the plain mode: one hand-off
to one worker, its launches, one wait.  A few builds (SINGLES_MAX) are queued
as single builds back to back; more go to one batched build.  The dispatcher
blocks on builds of up to BLOCK_SYMBOLS symbols; while a larger batch runs it
checks for finished work and new queries every POLL_S seconds.

Plan figures (image and workspace sizes, pass width) of every sequence are
taken when the server is created, so admission does no planning.

From start() to close() the server shortens the interpreter's thread switch
interval and turns Python's cyclic garbage collector off (a full collection
would stall every thread for tens of milliseconds); close() restores both.

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
import gc
import sys
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import binding as B


SWITCH_INTERVAL_S = 2e-4
POLL_S = 2e-4
# a batch of at most this many builds is queued as single builds one after
# another (less set-up than a batched build for a few sequences)
SINGLES_MAX = 4
# a batch of at most this many symbols is waited for (blocking); a larger one
# is polled so that queries arriving meanwhile are served
BLOCK_SYMBOLS = 1 << 22


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
                 mode: str = "continuous", tau_of=None, batch_tile: int = 0):
        """seqs: list of (device int tensor S, sigma) the builds refer to;
        tau_of(n, sigma): pass width of a sequence (0 = automatic);
        batch_tile: tiles per chunk of batched builds (0 = automatic)."""
        import torch
        self.torch = torch
        self.seqs = seqs
        self.budget = hbm_budget
        self.mode = mode
        self.max_batch = max_batch
        self.tau_of = tau_of or (lambda n, sigma: 0)
        self.batch_tune = B.make_tuning(tile=batch_tile)
        self.build_stream = torch.cuda.Stream()
        self._build_handle = B._stream(self.build_stream)
        self._tunings = {}
        self.query_stream = torch.cuda.Stream() if mode == "continuous" else self.build_stream
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        # status words of a batch's images, copied here on the build stream
        # and read after the one wait for the batch
        self.status_host = torch.empty(max_batch, dtype=torch.int32, pin_memory=True)
        self.resident: dict[int, Structure] = {}
        self.used = 0
        self.lock = threading.Lock()
        # one condition per worker on the shared lock, so that a submitted
        # build wakes only the build worker and a query only the query worker
        self.cv = threading.Condition(self.lock)   # new requests, closing
        self.builds = collections.deque()
        self.queries = collections.deque()
        self.all_reqs: list[Request] = []
        self.closing = False
        self.batches: list[int] = []
        self.query_batches: list[int] = []
        self.threads = []
        # plan figures of every sequence, taken before serving starts (a
        # sequence the library refuses keeps its error code)
        self._cost_cache = {}
        for k in range(len(seqs)):
            try:
                self._costs(k)
            except B.WaveletError as e:
                self._cost_cache[k] = e.code

    # ---- submission ------------------------------------------------------------
    def submit_build(self, seq: int) -> Request:
        with self.lock:
            r = Request(len(self.all_reqs), "build", time.perf_counter(), seq=seq)
            self.all_reqs.append(r)
            (self.builds if self.mode == "continuous" else self.queries).append(r)
            self.cv.notify()
            return r

    def submit_query(self, target: int, args) -> Request:
        """one batch of mixed queries on structure `target`:
        args = (pos, rank symbols, rank positions, select symbols, select ranks)"""
        with self.lock:
            r = Request(len(self.all_reqs), "query", time.perf_counter(), seq=target, qtype="mixed", args=args)
            self.all_reqs.append(r)
            self.queries.append(r)
            self.cv.notify()
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
        # a full collection of the cyclic garbage collector walks every
        # object of the process (hundreds of thousands once torch is
        # imported) with the interpreter held: tens of milliseconds during
        # which no request is dispatched.  Requests make no reference cycles,
        # so collection is off while serving; the objects made before are
        # moved out of the collector's generations for good measure.
        self._gc = gc.isenabled()
        gc.freeze()
        gc.disable()
        if self.mode == "continuous":
            self.threads = [threading.Thread(target=self._dispatch_loop, daemon=True)]
        else:
            self.threads = [threading.Thread(target=self._plain_loop, daemon=True)]
        for t in self.threads:
            t.start()

    def close(self):
        with self.lock:
            self.closing = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()
        sys.setswitchinterval(self._switch)
        gc.unfreeze()
        if self._gc:
            gc.enable()

    def _costs(self, seq):
        """(image bytes, batch-workspace bytes, single-build workspace bytes,
        tau) of one sequence, cached; the workspace of a batch is at most the
        sum over its sequences.  Raises WaveletError for a sequence the library
        refuses."""
        c = self._cost_cache.get(seq)
        if isinstance(c, int):
            raise B.WaveletError(c, "wt_plan")
        if c is None:
            S, sigma = self.seqs[seq]
            tau = self.tau_of(S.numel(), sigma)
            info = B.plan(B.KIND_WM, S.numel(), sigma, S.element_size(), tune=B.make_tuning(tau=tau))
            ob = info.out_bytes
            # sizing only: any non-null, 16-byte aligned addresses pass the plan's checks
            d = B.wt_seq_desc()
            d.S, d.n, d.sigma, d.sym_bytes, d.out, d.out_bytes, d.tau = 256, S.numel(), sigma, S.element_size(), 256, ob, tau
            c = (ob, B.batch_plan(B.KIND_WM, [d], self.batch_tune), info.workspace_bytes, tau)
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
        taken, pending = set(), 0    # sequences and image bytes of this batch so far
        while self.builds and len(take) < self.max_batch:
            r = self.builds[0]
            S, sigma = self.seqs[r.seq]
            try:
                ob, wsb, _, tau = self._costs(r.seq)
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
            if not self._evict_for(ob + pending, keep=taken):
                break
            d = B.wt_seq_desc()
            d.S, d.n, d.sigma, d.sym_bytes = S.data_ptr(), S.numel(), sigma, S.element_size()
            d.tau = tau
            # images are allocated on the build stream (their first use)
            img = self.torch.empty(ob, dtype=self.torch.uint8, device="cuda")
            d.out, d.out_bytes = img.data_ptr(), ob
            ws_need += wsb
            self.builds.popleft()
            take.append(r)
            taken.add(r.seq)
            pending += ob
            descs.append(d)
            imgs.append(img)
            nbytes.append(ob)
        return take, descs, imgs, nbytes

    def _status_copy(self, imgs):
        """(on the build stream, after the build launches) copy every image's
        header status word (what wt_check reads) to pinned host memory"""
        torch = self.torch
        k = len(imgs)
        words = imgs[0][36:40] if k == 1 else torch.cat([img[36:40] for img in imgs])
        self.status_host[:k].copy_(words.view(torch.int32), non_blocking=True)

    def _codes(self, k, rc, first=0):
        """(after the build stream has passed the status copy) the codes of
        images first..first+k-1: the call's code if it failed, else WT_ERANGE
        for a status word that reports a symbol >= sigma"""
        if rc != B.WT_OK:
            return [rc] * k
        return [B.WT_OK if w == 0 else B.WT_ERANGE for w in self.status_host[first:first + k].tolist()]

    def _finish(self, imgs, rc):
        """(plain mode) wait once for a build launched on the build stream;
        image codes"""
        if rc == B.WT_OK:
            self._status_copy(imgs)
        self.build_stream.synchronize()
        return self._codes(len(imgs), rc)

    def _launch_builds(self, take, descs, imgs):
        """queue the builds on the build stream, each segment of the batch
        followed by the copy of its status words and an event; returns (rc,
        [(first, end, event)]): rc is the code of the first launch that failed
        (the segments before it stand).  The last segment's event is the
        build stream itself (nothing else is queued on it while a batch is on
        the device).  A few sequences are built one by one when each one's
        own workspace fits (admission counted their batched workspace, which
        can be smaller), else as one batch."""
        torch = self.torch
        segs = []
        if len(descs) <= SINGLES_MAX and all(self._costs(r.seq)[2] <= self.ws.numel() for r in take):
            # a few sequences: single builds in stream order (one workspace),
            # each finishing on its own
            for i, d in enumerate(descs):
                tn = self._tunings.get(d.tau)
                if tn is None:
                    tn = self._tunings[d.tau] = B.make_tuning(tau=d.tau)
                rc = B.lib().wm_build(d.S, d.n, d.sigma, d.sym_bytes, None, ctypes.byref(tn), d.out,
                                      d.out_bytes, self.ws.data_ptr(), self.ws.numel(), self._build_handle)
                if rc != B.WT_OK:
                    return rc, segs
                self.status_host[i:i + 1].copy_(imgs[i][36:40].view(torch.int32), non_blocking=True)
                if i + 1 < len(descs):
                    ev = torch.cuda.Event()
                    ev.record(self.build_stream)
                else:
                    ev = self.build_stream
                segs.append((i, i + 1, ev))
            return B.WT_OK, segs
        rc = B.batch_build(B.KIND_WM, descs, self.ws, self.batch_tune, stream=self.build_stream)
        if rc != B.WT_OK:
            return rc, segs
        self._status_copy(imgs)
        return B.WT_OK, [(0, len(descs), self.build_stream)]

    def _complete_builds(self, take, imgs, nbytes, codes):
        t = time.perf_counter()
        with self.lock:
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

    def _take_queries(self, stream):
        """(under the lock) every query that has arrived, with its structure,
        to be run on `stream`"""
        work = []
        while self.queries and len(work) < self.max_batch:
            r = self.queries.popleft()
            work.append((r, self._take_structure(r, stream)))
        return work

    def _launch_queries(self, work, stream):
        """launch every query of `work` on `stream`; the launched ones"""
        launched = []
        for r, st in work:
            if st is None:
                r.error = B.WT_EINVAL
                continue
            try:
                self._run_query(r, st, stream)
                launched.append(r)
            except Exception as e:   # fail this query, keep serving
                r.result, r.error = None, getattr(e, "code", B.WT_EHIP)
        return launched

    def _wait_queries(self, work, launched, stream):
        """one wait for the queries of `work` launched on `stream`"""
        try:
            stream.synchronize()
        except Exception as e:
            for r in launched:
                r.result, r.error = None, getattr(e, "code", B.WT_EHIP)
        t = time.perf_counter()
        with self.lock:
            self.query_batches.append(len(work))
        for r, _ in work:
            r.done = t

    def _dispatch_loop(self):
        torch = self.torch
        # builds on the device: (take, imgs, nbytes, pending segments, short)
        flight = None
        while True:
            batch, qwork = None, []
            with self.lock:
                while (not self.builds and not self.queries and flight is None and not self.closing):
                    self.cv.wait()
                if self.closing and not self.builds and not self.queries and flight is None:
                    return
                if flight is None and self.builds:
                    with torch.cuda.stream(self.build_stream):
                        batch = self._admit()
                    self.used += sum(batch[3])
                # queries overlap builds on their own stream; with no build on
                # the device they take the build stream, the one in recent use
                # (measured at low load: a query batch on the second stream,
                # idle between queries, finished 0.02-0.03 ms later)
                qstream = (self.build_stream if flight is None and not (batch and batch[0])
                           else self.query_stream)
                qwork = self._take_queries(qstream)
            # queries are launched before the builds that arrived with them
            launched = self._launch_queries(qwork, qstream) if qwork else None
            if batch is not None and batch[0]:
                take, descs, imgs, nbytes = batch
                self.batches.append(len(take))
                try:
                    with torch.cuda.stream(self.build_stream):
                        rc, segs = self._launch_builds(take, descs, imgs)
                except Exception as e:   # fail the batch, keep serving
                    rc, segs = getattr(e, "code", B.WT_EHIP), []
                    try:   # whatever was queued finishes before the images are dropped
                        self.build_stream.synchronize()
                    except Exception:
                        pass
                queued = segs[-1][1] if segs else 0
                if queued < len(take):
                    self._complete_builds(take[queued:], imgs[queued:], nbytes[queued:],
                                          [rc if rc != B.WT_OK else B.WT_EHIP] * (len(take) - queued))
                if segs:
                    flight = (take, imgs, nbytes, segs, sum(d.n for d in descs) <= BLOCK_SYMBOLS)
            if qwork:
                self._wait_queries(qwork, launched, qstream)
            if flight is not None:
                take, imgs, nbytes, segs, short = flight
                # finish the segments the device is done with, in order; wait
                # for short builds as the plain mode does, poll long ones
                while segs:
                    lo, hi, ev = segs[0]
                    if short and not self.queries:
                        ev.synchronize()
                    elif not ev.query():
                        break
                    segs.pop(0)
                    try:
                        codes = self._codes(hi - lo, B.WT_OK, lo)
                    except Exception as e:
                        codes = [getattr(e, "code", B.WT_EHIP)] * (hi - lo)
                    self._complete_builds(take[lo:hi], imgs[lo:hi], nbytes[lo:hi], codes)
                if segs:
                    with self.lock:
                        if not self.queries and not self.closing:
                            self.cv.wait(POLL_S)
                    continue
                flight = None
            elif batch is not None and not batch[0] and not qwork:
                time.sleep(0.0005)   # builds wait for room (budget or workspace)

    def _plain_build(self, r):
        torch = self.torch
        S, sigma = self.seqs[r.seq]
        try:
            ob, _, wsb, tau = self._costs(r.seq)
        except B.WaveletError as e:
            r.error, r.done = e.code, time.perf_counter()
            return
        tn = B.make_tuning(tau=tau)
        if ob > self.budget or self.ws.numel() < wsb:
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
                r.error = self._finish([img], rc)[0]
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
                    self.cv.wait()
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
