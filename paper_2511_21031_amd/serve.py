"""Continuous-batching server for parameter-sweep solves on one GPU.

Requests arrive over time (each is one ensemble-averaged problem with its own
grid, bins, void fraction, drive and step count).  The server

* admits arrived requests in arrival order as soon as a batch slot is free and
  the request's device footprint (state, the two work copies of the stage
  results, the context's own buffers, the initial primitives) fits the HBM
  budget (the batch enforces it too); the context and the
  initial state are created on the server stream without a host
  synchronisation;
* keeps every admitted problem's state resident and advances all of them
  together with one batch call per chunk: bub_batch_run (default), which
  counts each member's steps down and flags its completion, or bub_batch_step
  (`use_run=False`); either way the members' own kernels overlap over the
  batch's streams; chunks have at most `chunk` steps and never run past the
  member with the fewest steps left, so that a member leaves the batch exactly
  at its last step;
* retires a problem when the stream event after its last step has completed:
  its error word (and, if asked, its state) is copied out, its memory returns
  to the budget, and waiting requests are admitted into the freed slot while
  the other problems keep running.

Latency is measured from a request's arrival to the moment the host sees its
result complete.  The scheduling (admission, chunking, retirement) is plain
host code in `Server.run`; the device work is behind a few methods (`_setup`,
`_admit`, `_step`, `_remove`, `_finish`, `_collect`, `_drain`) so that the
policy can be exercised without a GPU.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


def footprint_bytes(case) -> int:
    """Device bytes a problem holds while resident: its state, the two work copies of the
    stage results, the context's own buffers (plus alignment slack), and the device copy of its
    initial primitives ([ndim+3][N] doubles), which stays alive until the problem retires because
    the state is built from it asynchronously."""
    from ._binding import ctx_buffer_bytes
    state = 8 * case.nvar * case.ncells
    return 3 * state + ctx_buffer_bytes(case.ndim, case.n, case.nb) + 256 + 8 * (case.ndim + 3) * case.ncells


@dataclass
class Record:
    rid: int
    arrival: float
    steps: int
    footprint: int
    admitted: float = -1.0
    finished: float = -1.0
    remaining: int = 0
    slot: int = -1
    error: int = 0
    error_cell: int = -1
    error_bin: int = -1
    result: np.ndarray | None = None
    _keep: tuple = field(default=(), repr=False)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    """Continuous batching of ensemble-averaged solves under an HBM budget (bytes)."""

    def __init__(self, hbm_budget: int, max_slots: int = 64, precision=None, bubble_mode=None,
                 chunk: int = 10, keep_results: bool = False, autotune: bool = True, footprint=footprint_bytes,
                 lanes: int = 4, use_run: bool = True, tune_cache: str | None = None):
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.precision = precision
        self.bubble_mode = bubble_mode
        self.chunk = int(chunk)
        self.keep_results = keep_results
        self.autotune = autotune
        self.footprint = footprint
        self.lanes = int(lanes)
        self.use_run = bool(use_run)   # chunks through bub_batch_run (step counts) or bub_batch_step
        self.tune_cache = tune_cache   # tile-shape cache file of the class autotuner (persists across runs)
        self.used = 0
        self.peak_used = 0
        self.peak_active = 0
        self.classes = set()      # (ndim, nb) classes seen; a new one triggers the batch autotuner
        self._tune = False
        self.chunks = []          # (member request ids, steps) of every batched step call
        self._setup()

    # -- device side ------------------------------------------------------------------
    def _setup(self):
        import torch
        from ._binding import Batch, PREC_MIXED, BUBBLES_SPLIT
        if self.precision is None:
            self.precision = PREC_MIXED
        if self.bubble_mode is None:
            self.bubble_mode = BUBBLES_SPLIT
        self.stream = torch.cuda.Stream()
        self.batch = Batch(self.precision, self.max_slots, hbm_budget=self.budget)
        self.batch.set_lanes(self.lanes)
        if self.tune_cache:
            self.batch.set_tune_cache(self.tune_cache)

    def _admit(self, rec: Record, case) -> int:
        import torch
        from ._binding import context_from_case
        # Every allocation is made on the server stream, so the caching allocator hands memory
        # freed by a retired problem only to work ordered after that problem's last step.
        with torch.cuda.stream(self.stream):
            ctx = context_from_case(case, precision=self.precision, bubble_mode=self.bubble_mode,
                                    torch_buffer=True, stream=self.stream)
            host = torch.from_numpy(case.prim).pin_memory()
            prim = host.to("cuda", non_blocking=True)
            q = ctx.init_state(prim, stream=self.stream)
            work = ctx.new_work()
        rec._keep = (ctx, q, work, prim, host)
        key = (case.ndim, case.nb)
        if key not in self.classes:
            self.classes.add(key)
            self._tune = True
        return self.batch.add(ctx, q, work, steps=rec.steps)

    def _step(self, nsteps: int, nactive: int):
        if self.autotune and self._tune:
            # tile shape of each new (ndim, nb) class (synchronises the server stream once per class)
            self.batch.autotune(reps=2, stream=self.stream)
            self._tune = False
        if self.use_run:
            taken = self.batch.run(nsteps, stream=self.stream)
            if taken != nsteps:
                raise RuntimeError(f"batch chunk took {taken} steps, {nsteps} planned")
        else:
            self.batch.step(nsteps, stream=self.stream)

    def _remove(self, slot: int):
        self.batch.remove(slot)

    def _finish(self, done):
        """Enqueue the error-word and result copies of problems whose last step is queued;
        returns (event, copies)."""
        import torch
        with torch.cuda.stream(self.stream):
            err = torch.empty((len(done), 3), dtype=torch.int64, device="cuda")
            for i, rec in enumerate(done):
                rec._keep[0].error_copy(err[i], stream=self.stream)
            err_host = err.to("cpu", non_blocking=True)
            res = [rec._keep[1].to("cpu", non_blocking=True) if self.keep_results else None for rec in done]
            ev = torch.cuda.Event()
            ev.record(self.stream)
        return ev, (err, err_host, res)

    def _collect(self, copies, i):
        _, err_host, res = copies
        code, cell, b = (int(v) for v in err_host[i])
        return code, cell, b, (res[i].numpy() if res[i] is not None else None)

    def _drain(self):
        self.stream.synchronize()

    # -- scheduling -------------------------------------------------------------------
    def _retire(self, item, now: float):
        _, done, copies = item
        for i, rec in enumerate(done):
            rec.error, rec.error_cell, rec.error_bin, rec.result = self._collect(copies, i)
            rec._keep = ()
            rec.finished = now
            self.used -= rec.footprint

    def run(self, requests, make_case, time_scale: float = 1.0, progress=None):
        """Serve `requests` (objects with rid, arrival, steps); make_case(request) -> workloads.Case.

        Arrival times are seconds from the start of the call, multiplied by time_scale.
        progress(retired, total), if given, is called after every retirement.
        Returns the Records in request-id order.
        """
        retired = 0
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        records = {}
        active: dict[int, Record] = {}
        finishing = []   # (event, records, copies) of problems whose last step is queued
        t0 = time.perf_counter()
        while pending or active or finishing:
            now = time.perf_counter() - t0
            # admission: arrived requests, in order, while a slot and the budget allow
            while pending and pending[0].arrival * time_scale <= now and len(active) < self.max_slots:
                r = pending[0]
                case = make_case(r)
                fp = self.footprint(case)
                if fp > self.budget:
                    raise ValueError(f"request {r.rid} needs {fp} bytes, more than the whole budget")
                if self.used + fp > self.budget:
                    break
                pending.popleft()
                rec = Record(r.rid, r.arrival * time_scale, int(r.steps), fp)
                rec.admitted = now
                rec.remaining = rec.steps
                rec.slot = self._admit(rec, case)
                self.used += fp
                records[r.rid] = rec
                active[rec.slot] = rec
            self.peak_used = max(self.peak_used, self.used)
            self.peak_active = max(self.peak_active, len(active))
            # retire problems whose last step has completed on the device
            still = []
            for item in finishing:
                if item[0].query():
                    self._retire(item, time.perf_counter() - t0)
                    retired += len(item[1])
                    if progress is not None:
                        progress(retired, len(requests))
                else:
                    still.append(item)
            finishing = still
            if not active:
                if finishing:
                    finishing[0][0].synchronize()
                elif pending:
                    wait = pending[0].arrival * time_scale - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.005))
                continue
            k = min(self.chunk, min(rec.remaining for rec in active.values()))
            self._step(k, len(active))
            self.chunks.append((sorted(rec.rid for rec in active.values()), k))
            done = []
            for slot, rec in list(active.items()):
                rec.remaining -= k
                if rec.remaining == 0:
                    self._remove(slot)
                    del active[slot]
                    done.append(rec)
            if done:
                ev, copies = self._finish(done)
                finishing.append((ev, done, copies))
            # keep the host at most a few chunks ahead of the device
            if len(finishing) > 4:
                finishing[0][0].synchronize()
        self._drain()
        return [records[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


def summarize(records, t_total: float) -> dict:
    lat = np.array([r.latency for r in records])
    return {"solves": len(records), "solves_per_s": len(records) / t_total, "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
            "errors": int(sum(1 for r in records if r.error))}


def run_sequential(requests, make_case, precision, bubble_mode, time_scale: float = 1.0, keep_results=False,
                   progress=None):
    """Baseline: the same requests one at a time, in arrival order, each on its own context
    with plain bub_rk3_step calls.  A request starts when it has arrived and the previous one
    has finished; its latency is its finish time minus its arrival time."""
    import torch
    from ._binding import context_from_case
    out = []
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda r: (r.arrival, r.rid)):
        arr = r.arrival * time_scale
        now = time.perf_counter() - t0
        if now < arr:
            time.sleep(arr - now)
        case = make_case(r)
        ctx = context_from_case(case, precision=precision, bubble_mode=bubble_mode)
        q = ctx.init_state(torch.from_numpy(case.prim).cuda())
        work = ctx.new_work()
        for _ in range(int(r.steps)):
            ctx.rk3_step(q, work)
        code, cell, b = ctx.last_error()
        rec = Record(r.rid, arr, int(r.steps), footprint_bytes(case))
        rec.finished = time.perf_counter() - t0
        rec.error, rec.error_cell, rec.error_bin = code, cell, b
        if keep_results:
            rec.result = q.cpu().numpy()
        ctx.close()
        out.append(rec)
        if progress is not None:
            progress(len(out), len(requests))
    return sorted(out, key=lambda x: x.rid)
