"""Continuous-batching request server for surface-source subproblems.

A request is one subproblem family: a model, a grid, a record length, its
shots (all shots of a request advance together in one launch per time step)
and their data.  Requests are admitted in arrival order as soon as device
memory (by the library's exact footprint) and an execution slot are free;
each admitted request runs on its own HIP stream with its state resident in
a workspace taken from the PyTorch caching allocator (the library itself
allocates nothing), so requests that arrive while others run overlap with
them on the device.  With batch > 1, a slot takes the first queued request
together with up to batch - 1 later queued ones that can share its solve
(same stencil order, field type, iteration count and preconditioning, all
within the free memory) and solves them as one heterogeneous batch, their
propagations merged into one launch per time step (ssx_batch_*).  Only
small requests are batched (at most batch_cells grid cells over all their
shots: the merged launch pays where single launches are bound by latency),
and only with records within batch_nt_ratio of each other's length (the
members run in lockstep, so a short record waits for the longest).  When a
request (or batch) completes its memory and slot go to the queue.  Results
do not depend on what else is running or on batching: each request's
arithmetic is fixed by its shape (kernel choices are keyed by shape only,
and a batch member's results are bitwise those of its own solve).

The server records, per request, arrival, admission and completion times
and reports throughput and latency percentiles.
"""
from __future__ import annotations

import dataclasses
import threading
import time
from collections import deque
from typing import Any

import numpy as np

from . import Batch, Context, footprint


@dataclasses.dataclass
class Request:
    rid: int
    prob: Any                 # problem description (see Context)
    kappa: np.ndarray
    rho: float
    d: Any                    # device tensor [nshots][nt][nr], float32/float64
    alpha_rel: float = 1e-3
    K: int = 20
    field_dtype: str = "f16"
    use_precond: bool = True
    arrival: float = 0.0      # seconds after the start of the run

    @property
    def nshots(self) -> int:
        return len(self.prob.xs)


@dataclasses.dataclass
class Result:
    rid: int
    h: Any
    hist: np.ndarray
    iters: int
    status: int
    t_arrival: float
    t_admit: float
    t_done: float

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


def request_bytes(req: Request) -> int:
    """Device bytes a request holds while resident: the context plus its
    solution vector (the data is owned by the caller)."""
    vsz = 8 if req.field_dtype == "f64" else 4
    return footprint(req.prob, req.field_dtype, req.nshots) + \
        req.nshots * req.prob.nt * req.prob.ns * vsz


def batch_key(req: Request) -> tuple:
    """Requests with equal keys can share a batch solve."""
    return (req.prob.order, req.field_dtype, req.K, bool(req.use_precond))


def request_cells(req: Request) -> int:
    """Cells of the padded grid over all the request's shots."""
    p = req.prob
    return (p.nz + 2 * p.npml) * (p.nx + 2 * p.npml) * req.nshots


def take_group(queue: deque, sizes: dict, free: int, batch: int, batch_cells: int,
               batch_nt_ratio: float) -> tuple[list, int]:
    """Removes from the queue the request at its head, with (batch > 1 and
    the head small enough) up to batch - 1 later ones that can share its
    solve: equal batch_key, at most batch_cells cells, records within
    batch_nt_ratio of the head's, all within `free` bytes.  Returns the group
    and its bytes.  The head must fit `free`."""
    group = [queue.popleft()]
    nb = sizes[group[0].rid]
    if batch > 1 and request_cells(group[0]) <= batch_cells:
        key = batch_key(group[0])
        nt0 = group[0].prob.nt
        for r in list(queue):
            if len(group) >= batch:
                break
            ratio = max(r.prob.nt, nt0) / min(r.prob.nt, nt0)
            if (batch_key(r) == key and request_cells(r) <= batch_cells
                    and ratio <= batch_nt_ratio and nb + sizes[r.rid] <= free):
                queue.remove(r)
                group.append(r)
                nb += sizes[r.rid]
    return group, nb


class Server:
    """Admission by footprint and slots, FIFO order, one stream per request
    (or per batch of requests, batch > 1)."""

    def __init__(self, budget_bytes: int, slots: int = 4, graphs: bool = False,
                 tuner=None, on_done=None, batch: int = 1, batch_cells: int = 2_000_000,
                 batch_nt_ratio: float = 1.5):
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.batch = max(1, int(batch))
        self.batch_cells = int(batch_cells)
        self.batch_nt_ratio = float(batch_nt_ratio)
        self.graphs = bool(graphs)
        self.tuner = tuner            # callable(ctx, req) applying kernel choices, or None
        self.on_done = on_done        # callable(Result) after each completion, or None
        self._cv = threading.Condition()
        self._free = self.budget
        self._busy = 0
        self._results: list[Result] = []
        self._errors: list[BaseException] = []

    # -- one request, or a batch of them ---------------------------------------
    def _serve(self, group: list, t0: float, t_admit: float, nbytes: int):
        import torch
        try:
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                wss, ctxs = [], []
                for req in group:
                    ws = torch.empty(footprint(req.prob, req.field_dtype, req.nshots),
                                     dtype=torch.uint8, device="cuda")
                    ctx = Context(req.prob, req.kappa, req.rho, field_dtype=req.field_dtype,
                                  stream=stream, workspace=ws)
                    if self.tuner is not None:
                        self.tuner(ctx, req)
                    ctx.set_graphs(self.graphs)
                    wss.append(ws)
                    ctxs.append(ctx)
                if len(group) == 1:
                    req, ctx = group[0], ctxs[0]
                    h, hist, iters, st = ctx.pcg_solve(req.d, req.alpha_rel, req.K,
                                                       use_precond=req.use_precond,
                                                       h=ctx.empty_s(), raise_on_breakdown=False)
                    out = [(h, hist, iters, st)]
                else:
                    b = Batch(ctxs)
                    hs, hists, its, sts = b.pcg_solve(
                        [r.d for r in group], [r.alpha_rel for r in group], group[0].K,
                        use_precond=group[0].use_precond, raise_on_breakdown=False)
                    b.close()
                    out = list(zip(hs, hists, its, sts))
                for ctx in ctxs:
                    ctx.close()
                del wss
            stream.synchronize()
            t_done = time.perf_counter() - t0
            for req, (h, hist, iters, st) in zip(group, out):
                res = Result(req.rid, h, hist, iters, st, req.arrival, t_admit, t_done)
                with self._cv:
                    self._results.append(res)
                if self.on_done is not None:
                    self.on_done(res)
        except BaseException as e:  # reported by run()
            with self._cv:
                self._errors.append(e)
        finally:
            with self._cv:
                self._free += nbytes
                self._busy -= 1
                self._cv.notify_all()

    # -- a whole stream -----------------------------------------------------
    def run(self, requests: list[Request], realtime: bool = True) -> list[Result]:
        """Serve the requests.  With realtime=True each is released at its
        arrival offset; otherwise all are queued at once (closed loop)."""
        order = sorted(requests, key=lambda r: r.arrival)
        sizes = {r.rid: request_bytes(r) for r in order}
        for r in order:
            if sizes[r.rid] > self.budget:
                raise ValueError(f"request {r.rid} needs {sizes[r.rid]} bytes, above the "
                                 f"budget of {self.budget}")
        pending = deque(order)
        queue: deque[Request] = deque()
        threads = []
        t0 = time.perf_counter()
        with self._cv:
            self._results = []
            self._errors = []
        while pending or queue:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                r = pending.popleft()
                if not realtime:
                    r.arrival = 0.0
                queue.append(r)
            with self._cv:
                while queue and self._busy < self.slots and sizes[queue[0].rid] <= self._free:
                    group, nb = take_group(queue, sizes, self._free, self.batch,
                                           self.batch_cells, self.batch_nt_ratio)
                    self._free -= nb
                    self._busy += 1
                    th = threading.Thread(target=self._serve,
                                          args=(group, t0, time.perf_counter() - t0, nb),
                                          daemon=True)
                    th.start()
                    threads.append(th)
                if self._errors:
                    break
                if queue or pending:
                    timeout = 0.05
                    if pending and not queue:
                        timeout = max(0.0, min(0.05, pending[0].arrival - now))
                    self._cv.wait(timeout=timeout)
        for th in threads:
            th.join()
        if self._errors:
            raise self._errors[0]
        return sorted(self._results, key=lambda r: r.rid)


def summarize(results: list[Result], wall: float) -> dict:
    lat = np.array([r.latency for r in results])
    solves = sum(int(r.h.shape[0]) for r in results)
    return {"requests": len(results), "solves": solves, "wall_s": wall,
            "requests_per_s": len(results) / wall, "solves_per_s": solves / wall,
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "latency_max_s": float(lat.max())}
