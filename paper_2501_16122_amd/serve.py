"""Continuous-batching server for map-making solves on one GPU.

Requests (each a complete map-making problem: pointing, timeline, noise
model) arrive over time.  The server admits a request as soon as a slot is
free and its device footprint fits the memory budget, uploads its arrays,
builds its pointing (and precomputed pointing weights) and noise handles,
and starts a resumable solver on a stream of its own.  Every scheduler tick
enqueues one chunk of iterations for every active solve, so the work of
different requests overlaps on the device; solves whose state copy shows
convergence are finished (true residual, full-grid map), their memory is
released, and waiting requests are admitted in their place.

Two ways to overlap the active solves: one stream per solve (the default),
or batched, where every tick enqueues one shared step for all active solves
(mm_batch_step: one operator launch per iteration over the tiles of every
solve, one launch per PCG vector step over all of them) on a single stream.

Admission (the upload, the builds, the solver's creation) runs on builder
threads of their own by default (prefetch, two builders): while requests'
arrays cross PCIe and their handles are built, the scheduler keeps the
active solves supplied with work.  The library's calls release the
interpreter lock.

``Server.cancel(rid)`` withdraws a request at any stage: a queued one is
dropped; one being built, or active, stops at the next scheduler tick once
the work already queued on its stream has finished, and its memory is freed.

All computation runs in libmapmaker's kernels; this module only schedules.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import threading
import time
from typing import Callable, Optional

import numpy as np

from . import binding as b
from . import synth


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the start of the run
    workload: synth.Workload
    # host inputs (filled by ``materialize``)
    pix: Optional[np.ndarray] = None
    psi: Optional[np.ndarray] = None
    d: Optional[np.ndarray] = None
    coeff: Optional[np.ndarray] = None
    chunks: Optional[np.ndarray] = None


@dataclasses.dataclass
class Result:
    rid: int
    map: np.ndarray                # f64[n_pix, 3]
    info: dict
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def footprint_bytes(w: synth.Workload, opts: b.SolveOpts, weights: bool) -> int:
    """Upper bound of the device memory one request holds while in flight."""
    lib = b.load()
    esz = 4 if w.precision == "f32" else 8
    n = w.n_samples
    total = n * (4 + esz + esz)                      # pix, psi, d
    if weights:
        total += n * esz                              # stored tangent per sample
    sz = b._c.c_size_t()
    b._check(lib.mm_pointing_workspace_size(n, w.n_det, w.n_pix, b.MM_F32 if w.precision == "f32" else b.MM_F64,
                                            b._c.byref(sz)))
    total += sz.value
    if w.toeplitz:
        offs = synth.chunk_offsets(w)
        b._check(lib.mm_noise_toeplitz_workspace_size(w.lam, 1, offs.ctypes.data_as(b._pi64), offs.size - 1,
                                                      b._c.byref(sz)))
        total += sz.value
    else:
        total += 8 * w.n_det
    # solver vectors, state and history with every pixel kept (the library's bound)
    b._check(lib.mm_solver_workspace_bound(w.n_pix, 3, 1, b._c.byref(opts), b._c.byref(sz)))
    total += sz.value
    return int(total)


def materialize(req: Request, make_d: Callable) -> Request:
    """Draw the request's seeded inputs on the host.  ``make_d(w, pix, psi)``
    forms the timeline (the caller chooses how; tests use the oracle)."""
    w = req.workload
    pix, psi = synth.pointing(w)
    req.pix = pix
    req.psi = synth.storage(w, psi)
    req.d = synth.storage(w, make_d(w, pix, req.psi))
    if w.toeplitz:
        req.coeff = synth.toeplitz_coeff(w)
        req.chunks = synth.chunk_offsets(w)
    return req


class _Slot:
    def __init__(self, req: Request, dev, stream, opts, use_weights, now):
        import torch
        w = req.workload
        self.req = req
        self.admitted = now
        self.stream = stream
        with torch.cuda.stream(stream):
            self.t_pix = torch.from_numpy(req.pix).to(dev, non_blocking=False)
            self.t_psi = torch.from_numpy(req.psi).to(dev, non_blocking=False)
            self.t_d = torch.from_numpy(req.d).to(dev, non_blocking=False)
            self.pt = b.Pointing(self.t_pix, self.t_psi, synth.det_offsets(w), synth.det_weight(w), w.n_pix,
                                 w.min_hits, w.cond_max, stream=stream)
            if w.toeplitz:
                if use_weights:
                    self.pt.attach_weights(stream=stream)
                self.nz = b.Noise.toeplitz(req.coeff, req.chunks, dev, stream=stream)
            else:
                self.nz = b.Noise.white(synth.det_weight(w), dev, stream=stream)
            self.solver = b.AsyncSolver(self.pt, self.nz, self.t_d, stream=stream, **opts)

    def release(self):
        self.solver.close()
        self.pt.close()
        self.nz.close()
        del self.t_pix, self.t_psi, self.t_d


class Server:
    """Admit, advance and retire map-making solves with overlapping work."""

    def __init__(self, device="cuda:0", hbm_budget: Optional[int] = None, max_slots: int = 8, k_chunk: int = 8,
                 n_streams: int = 8, use_weights: bool = True, batched: bool = False, prefetch: bool = True,
                 builders: int = 2, **solve_opts):
        import torch
        self.dev = torch.device(device)
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.dev)
            hbm_budget = int(0.9 * free)
        self.budget = hbm_budget
        self.max_slots = max_slots
        self.k_chunk = k_chunk
        self.opts = dict(tol=1e-10, mixed=1, check_every=k_chunk)
        self.opts.update(solve_opts)
        self._sopts = b.solve_opts(**self.opts)
        # batched: every active solve advances in the same launches
        # (mm_batch_step, at most 16 right-hand sides), on one stream;
        # otherwise each solve runs on a stream of its own and the streams overlap
        self.batched = batched
        if batched and max_slots > 16:
            raise ValueError("batched serving takes at most 16 slots")
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(1 if batched else n_streams)]
        self.use_weights = use_weights
        self.pending: collections.deque = collections.deque()
        self.active: list = []
        self.in_use = 0
        self.results: list = []
        self.peak_slots = 0
        self.peak_bytes = 0
        self.depth = 0  # batched mode: shared steps in flight
        # the builder thread (prefetch): admission state shared with it
        self.prefetch = prefetch
        self.builders = max(1, builders)
        self._lock = threading.Lock()
        self._ready: collections.deque = collections.deque()  # built, not yet active
        self._building = 0
        self._stop = False
        self._err: Optional[BaseException] = None
        # cancellation: requested rids, and (rid, stage, seconds after the
        # start) of every request withdrawn ("queued", "built" or "active")
        self._cancel: set = set()
        self.cancelled: list = []
        self._t0 = time.perf_counter()

    def submit(self, req: Request):
        self.pending.append(req)

    def cancel(self, rid: int) -> None:
        """Withdraw request ``rid`` (thread-safe; a finished or unknown rid is
        ignored).  It appears in ``cancelled`` instead of the results."""
        with self._lock:
            self._cancel.add(rid)

    def _drop_cancelled(self):
        """Under the lock: drop cancelled requests from the queue and from the
        built ones not yet active; returns the slots that must be released."""
        if not self._cancel:
            return []
        now = time.perf_counter() - self._t0
        keep = collections.deque()
        for r in self.pending:
            if r.rid in self._cancel:
                self._cancel.discard(r.rid)
                self.cancelled.append((r.rid, "queued", now))
            else:
                keep.append(r)
        self.pending = keep
        gone, ready = [], collections.deque()
        for sl in self._ready:
            (gone if sl.req.rid in self._cancel else ready).append(sl)
        self._ready = ready
        for sl in gone:
            self._cancel.discard(sl.req.rid)
            self.cancelled.append((sl.req.rid, "built", now))
        return gone

    def _release_cancelled(self, slot, stage=None):
        """Free a withdrawn slot once the work queued on its stream is done
        (its solver may still have chunks of iterations in flight)."""
        sync = getattr(getattr(slot, "stream", None), "synchronize", None)
        if sync is not None:
            sync()
        slot.release()
        with self._lock:
            self.in_use -= slot.fp
            if stage is not None:
                self.cancelled.append((slot.req.rid, stage, time.perf_counter() - self._t0))

    def _cancel_active(self):
        """Stop the active solves that were cancelled; returns True if any."""
        with self._lock:
            if not self._cancel:
                return False
            gone = [sl for sl in self.active if sl.req.rid in self._cancel]
            if gone:
                self.active = [sl for sl in self.active if sl.req.rid not in self._cancel]
                self._cancel.difference_update(sl.req.rid for sl in gone)
        for sl in gone:
            self._release_cancelled(sl, "active")
        return bool(gone)

    def _fp(self, req: Request) -> int:
        return footprint_bytes(req.workload, self._sopts, self.use_weights and req.workload.toeplitz)

    def _admit(self, now: float, t0: float):
        with self._lock:
            self._drop_cancelled()
        while self.pending and len(self.active) < self.max_slots:
            req = self.pending[0]
            if req.arrival > now - t0:
                break
            fp = self._fp(req)
            if fp > self.budget:
                raise MemoryError(f"request {req.rid} needs {fp} bytes, more than the whole budget")
            if self.in_use + fp > self.budget:
                break  # wait for memory to free up
            self.pending.popleft()
            stream = self.streams[req.rid % len(self.streams)]
            slot = _Slot(req, self.dev, stream, self.opts, self.use_weights, now - t0)
            slot.fp = fp
            slot.depth = 0
            self.in_use += fp
            self.active.append(slot)
            self.peak_slots = max(self.peak_slots, len(self.active))
            self.peak_bytes = max(self.peak_bytes, self.in_use)

    def _reserve(self, now_rel: float):
        """Under the lock: the next request to build, its memory reserved, or
        None (none has arrived, no slot is free, or memory must free up)."""
        while self.pending and self.pending[0].rid in self._cancel:
            rid = self.pending.popleft().rid
            self._cancel.discard(rid)
            self.cancelled.append((rid, "queued", now_rel))
        if not self.pending or len(self.active) + self._building + len(self._ready) >= self.max_slots:
            return None
        req = self.pending[0]
        if req.arrival > now_rel:
            return None
        fp = self._fp(req)
        if fp > self.budget:
            raise MemoryError(f"request {req.rid} needs {fp} bytes, more than the whole budget")
        if self.in_use + fp > self.budget:
            return None
        self.pending.popleft()
        self.in_use += fp
        self.peak_bytes = max(self.peak_bytes, self.in_use)
        self._building += 1
        return req, fp

    def _builder(self, t0: float):
        """Builder thread: admit and build requests one at a time."""
        try:
            while True:
                with self._lock:
                    if self._stop:
                        return
                    got = self._reserve(time.perf_counter() - t0)
                if got is None:
                    time.sleep(0.0005)
                    continue
                req, fp = got
                stream = self.streams[req.rid % len(self.streams)]
                slot = _Slot(req, self.dev, stream, self.opts, self.use_weights, time.perf_counter() - t0)
                slot.fp = fp
                slot.depth = 0
                with self._lock:
                    self._building -= 1
                    self._ready.append(slot)
        except BaseException as e:  # reported by the scheduler loop
            with self._lock:
                self._err = e
                self._stop = True

    def run(self, requests=None, realtime=True, on_result=None):
        """Serve ``requests`` (sorted by arrival); returns the results in
        completion order.  With realtime=False arrival times are ignored and
        every request is admitted as soon as it fits."""
        for r in sorted(requests or [], key=lambda r: r.arrival):
            if not realtime:
                r.arrival = 0.0
            self.submit(r)
        t0 = time.perf_counter()
        self._t0 = t0
        if self.prefetch:
            return self._run_prefetch(t0, on_result)
        while self.pending or self.active:
            now = time.perf_counter()
            self._admit(now, t0)
            self._cancel_active()
            if not self.active:
                # nothing admitted yet: wait for the next arrival
                nxt = self.pending[0].arrival - (time.perf_counter() - t0)
                if nxt > 0:
                    time.sleep(min(nxt, 0.01))
                continue
            if self.batched:
                self._tick_batched(t0, on_result)
                continue
            progressed = False
            still = []
            for slot in self.active:
                done, in_flight = slot.solver.poll()
                if done:
                    self._retire(slot, t0, on_result)
                    progressed = True
                    continue
                still.append(slot)
                if not in_flight:
                    slot.depth = 0
                if slot.depth < 2:  # at most two chunks queued per solve
                    slot.solver.step(self.k_chunk)
                    slot.depth += 1
                    progressed = True
            self.active = still
            if not progressed:
                time.sleep(0.0002)
        return self.results

    def _run_prefetch(self, t0, on_result):
        """The scheduler loop with admission on the builder thread."""
        self._stop = False
        ths = [threading.Thread(target=self._builder, args=(t0,), daemon=True) for _ in range(self.builders)]
        for th in ths:
            th.start()
        try:
            while True:
                with self._lock:
                    if self._err is not None:
                        raise self._err
                    gone = self._drop_cancelled()
                for sl in gone:
                    self._release_cancelled(sl)
                self._cancel_active()
                with self._lock:
                    while self._ready:
                        self.active.append(self._ready.popleft())
                    self.peak_slots = max(self.peak_slots, len(self.active))
                    busy = bool(self.pending or self.active or self._building)
                if not busy:
                    break
                if not self.active:
                    time.sleep(0.0005)
                    continue
                if self.batched:
                    self._tick_batched(t0, on_result)
                    continue
                progressed = False
                still = []
                for slot in list(self.active):
                    done, in_flight = slot.solver.poll()
                    if done:
                        self._retire(slot, t0, on_result)
                        progressed = True
                        continue
                    still.append(slot)
                    if not in_flight:
                        slot.depth = 0
                    if slot.depth < 2:  # at most two chunks queued per solve
                        slot.solver.step(self.k_chunk)
                        slot.depth += 1
                        progressed = True
                with self._lock:
                    self.active = still
                if not progressed:
                    time.sleep(0.0002)
        finally:
            with self._lock:
                self._stop = True
            for th in ths:
                th.join()
        return self.results

    def _retire(self, slot, t0, on_result):
        out = slot.solver.finish()
        w = slot.req.workload
        res = Result(slot.req.rid, out["maps"][0].cpu().numpy().reshape(w.n_pix, 3), out["info"][0],
                     slot.req.arrival, slot.admitted, time.perf_counter() - t0)
        with self._lock:
            self.in_use -= slot.fp
            self._cancel.discard(slot.req.rid)  # finished before its cancel was seen
        slot.release()
        self.results.append(res)
        if on_result:
            on_result(res)

    def _tick_batched(self, t0, on_result):
        """One scheduler tick of the batched mode: retire finished solves, then
        enqueue one shared step of k iterations for all the others (at most two
        steps in flight)."""
        still, in_flight = [], False
        for slot in list(self.active):
            done, flight = slot.solver.poll()
            if done:
                self._retire(slot, t0, on_result)
            else:
                still.append(slot)
                in_flight = in_flight or flight
        with self._lock:
            self.active = still
        if not in_flight:
            self.depth = 0
        if still and self.depth < 2:
            b.batch_step([sl.solver for sl in still], self.k_chunk)
            self.depth += 1
        elif still:
            time.sleep(0.0002)


def poisson_requests(n: int, rate: float, sizes: Callable[[np.random.Generator, int], synth.Workload],
                     seed_id: int = 5) -> list:
    """n requests with exponential inter-arrival times (mean 1/rate s) and
    workloads drawn by ``sizes(rng, i)`` (seeded, stream 4)."""
    rng = np.random.default_rng(np.random.SeedSequence([synth.ROOT_SEED, seed_id, synth.STREAM_SERVE]))
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    return [Request(i, float(t[i]), sizes(rng, i)) for i in range(n)]


def log_uniform_int(rng: np.random.Generator, lo: float, hi: float) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
