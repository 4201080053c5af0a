"""Continuous-batching solve server.

Requests (a CNF plus solve parameters) arrive at any time and queue in arrival
order.  A worker thread (each with its own HIP stream) that becomes free takes
the head of the queue, if its estimated device footprint fits the budget, and
with it every queued request of the same kind that fits too; it builds and
uploads their plans and solves them, so requests taken while others run overlap
on the device.  Under light load a request is taken alone as soon as it arrives;
as the queue grows, the requests taken together grow with it.  Requests of the
same kind have the same step count, restart count, counting period, optimizer,
Adam constants, loss mode and schedule (learning rates and seeds may differ):
those small enough for the resident solver share one launch (one
workgroup per instance and restart), the others share one launch per kernel per
step (a work queue over their units).
Every instance's result is bitwise what a solo ``solve`` gives: the kernels'
summation order depends on the instance only, never on the batch.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

from . import _lib

# instances at most this large (n + m) are grouped for the resident solver
SMALL_ROWS = 12000
# instances with more literals run as jobs of their own: one of them keeps the
# device busy alone, and a job's plans are built one after the other, so a
# request grouped with a large one would wait for its build and its solve
GROUP_MAX_LITS = 1 << 21


def footprint_bytes(n: int, m: int, n_lits: int, restarts: int = 1, weighted: bool = False) -> int:
    """Device bytes of one solve: plan (both sparse layouts, tiles, offsets,
    clause weights) plus per-restart state (x, m, v, t, adjoint, best bytes,
    heavy partials)."""
    L = max(n_lits, 0)
    # clause-side and variable-side entries and the map between them
    struct = 4 * (3 * L + m + n + 2) + 16 * (m + n) // 64 + 4 * n + 8 * L // 64 + (8 * (m + 64) if weighted else 0)
    state = restarts * (16 * (n + 1) + 4 * (m + 64) + (n + 1) + 8 * L // 64) + 4096
    if restarts == 1:
        state += 4 * L + 4 * L // 8  # occurrence slots of the slot schedule
    return int(1.25 * (struct + state)) + (1 << 16)


@dataclass
class Request:
    n: int
    lits: np.ndarray
    params: dict
    arrival: float = 0.0
    future: Future = field(default_factory=Future)
    footprint: int = 0
    n_lits: int = 0
    small: bool = False
    rid: int = 0
    weights: object = None  # clause weights (weighted MaxSAT) or None


@dataclass
class ServeResult:
    rid: int
    output: object          # SolveOutput
    arrival: float
    admitted: float
    done: float

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Server:
    """Admit by footprint, overlap on device, batch the small ones."""

    def __init__(self, workers: int = 8, hbm_budget: int | None = None, small_batch: int = 64,
                 tiled_batch: int = 8, device: int = 0, trace: bool = False):
        import torch
        self._torch = torch
        torch.cuda.set_device(device)
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(device)
            hbm_budget = int(0.5 * free)
        self.budget = int(hbm_budget)
        self.in_use = 0
        self.small_batch = int(small_batch)
        # tiled groups stay small: their plans are built on the host by the
        # worker that takes the group, which is the slow part of a request
        self.tiled_batch = int(tiled_batch)
        self._queue: collections.deque[Request] = collections.deque()
        self._cv = threading.Condition()
        # admission statistics: the largest footprint admitted at once, the
        # times a worker found the head of the queue over budget and waited,
        # and (with trace) one (admitted, done, footprint, over budget alone)
        # record per job
        self.peak_in_use = 0
        self.deferrals = 0
        self.jobs: list | None = [] if trace else None
        self.job_rids: list | None = [] if trace else None  # with trace: the request ids of each job
        self._closed = False
        self._ids = 0
        self._workers = []
        for w in range(workers):
            t = threading.Thread(target=self._work, args=(w, device), daemon=True)
            t.start()
            self._workers.append(t)

    # -- client side -------------------------------------------------------------
    def submit(self, n: int, lits, arrival: float | None = None, weights=None, **params) -> Future:
        """Queue one instance (``weights``: one positive integer per clause for
        weighted MaxSAT); the future resolves to a ServeResult."""
        lits = np.ascontiguousarray(lits, dtype=np.int32)
        m = int(np.count_nonzero(lits == 0))
        R = int(params.get("restarts", 1))
        req = Request(n=int(n), lits=lits, params=params,
                      arrival=time.perf_counter() if arrival is None else arrival,
                      weights=None if weights is None else np.ascontiguousarray(weights, dtype=np.int64))
        if req.weights is not None and req.weights.size != m:
            raise ValueError(f"{req.weights.size} clause weights for {m} clauses")
        req.footprint = footprint_bytes(n, m, lits.size - m, R, req.weights is not None)
        req.n_lits = lits.size - m
        req.small = (n + m) <= SMALL_ROWS
        with self._cv:
            if self._closed:
                raise RuntimeError("server is closed")
            req.rid = self._ids
            self._ids += 1
            self._queue.append(req)
            self._cv.notify_all()
        return req.future

    def close(self, wait: bool = True):
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        if wait:
            for t in self._workers:
                t.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- workers: admission control, grouping, solving -------------------------
    def _take(self):
        """Under the lock: the next job (the admitted head of the queue and the
        queued requests of its kind that fit), or None once closed and empty."""
        while True:
            if self._queue:
                head = self._queue[0]
                # a request larger than the whole budget runs only on an idle device
                if self.in_use + head.footprint <= self.budget or self.in_use == 0:
                    break
                self.deferrals += 1
            elif self._closed:
                return None
            self._cv.wait()
        job = [self._queue.popleft()]
        self.in_use += job[0].footprint
        key = _group_key(job[0])
        cap = self.small_batch if job[0].small else self.tiled_batch
        if job[0].n_lits > GROUP_MAX_LITS:
            cap = 1
        keep = collections.deque()
        while self._queue and len(job) < cap:
            r = self._queue.popleft()
            if (_group_key(r) == key and r.n_lits <= GROUP_MAX_LITS
                    and self.in_use + r.footprint <= self.budget):
                job.append(r)
                self.in_use += r.footprint
            else:
                keep.append(r)
        keep.extend(self._queue)
        self._queue = keep
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        now = time.perf_counter()
        for r in job:
            r.params["_admitted"] = now
        return job

    def _work(self, w: int, device: int):
        torch = self._torch
        torch.cuda.set_device(device)
        stream = torch.cuda.Stream(device=device)
        while True:
            with self._cv:
                job = self._take()
                if job is None:
                    self._cv.notify_all()  # let the other workers see the end too
                    return
            try:
                self._run(job, stream)
            except Exception as e:  # deliver the failure to every request of the job
                for r in job:
                    if not r.future.done():
                        r.future.set_exception(e)
            finally:
                with self._cv:
                    foot = sum(r.footprint for r in job)
                    if self.jobs is not None:
                        self.job_rids.append(tuple(r.rid for r in job))
                        self.jobs.append((job[0].params["_admitted"], time.perf_counter(), foot,
                                          foot > self.budget))
                    self.in_use -= foot
                    self._cv.notify_all()

    def _run(self, job, stream):
        cnfs = []
        try:
            for r in job:
                cnfs.append(_lib.load_cnf(r.n, r.lits, stream=stream, weights=r.weights))
            clean = [{k: v for k, v in r.params.items() if not k.startswith("_")} for r in job]
            if len(job) == 1:
                try:
                    outs = [_lib.solve(cnfs[0], stream=stream, **clean[0])]
                except _lib.HipMsatError as e:
                    if getattr(e, "result", None) is None:
                        raise
                    outs = [e]  # non-finite loss or cancelled: the error carries the best so far
            else:
                # a job holds requests of one kind (_group_key): every parameter
                # that changes a solve goes through per instance
                kw = {k: [p.get(k, d) for p in clean] for k, d in _BATCH_DEFAULTS.items()}
                outs = _lib.solve_batch(cnfs, seeds=[p.get("seed", 0) for p in clean], stream=stream, **kw)
                for i, o in enumerate(outs):
                    if o.status != 0:
                        # as the solo path reports it: an error with the partial result
                        e = _lib.HipMsatError(o.status, f"instance {job[i].rid} of a batched job")
                        e.result = o
                        outs[i] = e
        finally:
            for c in cnfs:
                c.free()
        done = time.perf_counter()
        for r, o in zip(job, outs):
            if isinstance(o, Exception):
                r.future.set_exception(o)
            else:
                r.future.set_result(ServeResult(r.rid, o, r.arrival, r.params["_admitted"], done))


# solve parameters a batched job passes per instance, with their defaults
# (use_graph and autotune change the speed only, never a result)
_BATCH_DEFAULTS = {"steps": 1000, "restarts": 1, "eval_every": 1, "optimizer": _lib.ADAM, "lr": 1e-4,
                   "beta1": 0.9, "beta2": 0.999, "eps": 1e-8, "loss_mode": _lib.LOSS_UNSAT, "schedule": 0}


def _runs_alone(p: dict) -> bool:
    """A time limit or cancel flag applies to one solve, and a start point,
    a resumed state, x_T or the state handed back belong to one request."""
    return ((p.get("time_limit_s") or 0.0) > 0 or any(p.get(k) is not None for k in ("x0", "cancel", "resume"))
            or bool(p.get("want_x")) or bool(p.get("want_state")))


def _group_key(r: Request):
    """Requests that can share launches: same resident/tiled kind and the same
    value of every solve parameter a batched job shares (steps, restarts,
    counting period, optimizer, Adam constants, loss mode, schedule).  A
    request with a time limit, a cancel flag, a start point, a resumed state,
    or asking for x_T or its state is a job of its own (solved as alone)."""
    p = r.params
    if _runs_alone(p):
        return ("alone", r.rid)
    # lr and seed are per instance in a batch; the rest must match
    return (r.small,) + tuple(p.get(k, d) for k, d in _BATCH_DEFAULTS.items() if k != "lr")


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    f = int(np.floor(k))
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)
