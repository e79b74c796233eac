"""Continuous-batching reconstruction server.

Requests (a stack of slices of one geometry, sinograms already on the device)
arrive at any time.  The scheduler admits them in arrival order while their
device footprint (sinograms, filtered rows, images) fits an HBM budget, packs
every admitted request into the next batch as soon as one of several streams is
free, and launches that batch with one fbp_reconstruct_batch call (grouped
filter GEMMs plus one persistent backprojection launch per tile shape, from a
captured HIP graph).  Requests that arrive while earlier batches are on the GPU
join the next batch; batches on different streams overlap on the device.  A
waiter per stream resolves each request's future when its batch completes,
returns its bytes to the budget, and records latency from arrival to
completion.

A batch is closed once its estimated cost (pixel-angle updates, N^2 K per
slice) or slice count would pass a bound, so a request that arrives behind a
long queue waits for bounded batches rather than for one batch holding
everything admitted before it; up to n_streams bounded batches run at once.

Every image equals the image the same request gets alone: bitwise for
quarter-turn geometries (N >= 2, angles closed under +pi/2), whose tile shape
and summation order depend on the geometry alone, and within the FP32 tolerance
otherwise, where a geometry with 4 or more slices in a batch takes its stack
shape and a shorter run its single-slice shape (see include/fbp.h).

The executor is an interface, so the scheduling logic runs on the CPU in tests
with a fake executor; GpuExecutor drives libfbp.
"""
from __future__ import annotations

import collections
import itertools
import math
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field


class RequestTooLarge(ValueError):
    """The request alone needs more device memory than the whole budget."""


@dataclass
class Request:
    geom: object            # Geometry
    sino: object            # device tensor [B][K][D]
    n_slices: int
    nbytes: int = 0         # device footprint while admitted
    cost: int = 0           # pixel-angle updates
    arrival: float = 0.0
    rid: int = -1
    future: Future = field(default_factory=Future)
    output: object = None   # device tensor [B][N][N], allocated at admission


def footprint_bytes(K: int, D: int, N: int, n_slices: int) -> int:
    """Device bytes a request holds while admitted: sinogram + filtered rows + image."""
    return n_slices * (2 * K * D + N * N) * 4


def request_cost(K: int, N: int, n_slices: int) -> int:
    """Work of a request in pixel-angle updates (the backprojection's N^2 K per slice)."""
    return n_slices * N * N * K


# Default bound on a batch's cost: about two milliseconds of backprojection at the
# single-GPU rate (~5e12 updates/s); one request larger than this runs alone.
DEFAULT_BATCH_COST = 10 ** 10


class Executor:
    """What the server needs from a device backend."""
    n_streams: int = 2

    def allocate_output(self, req: Request):
        raise NotImplementedError

    def launch(self, stream_idx: int, reqs: list):
        """Queue one batch on stream `stream_idx`; return a completion handle."""
        raise NotImplementedError

    def wait(self, handle) -> None:
        """Block until the batch of `handle` has finished (raise on failure)."""
        raise NotImplementedError


class GpuExecutor(Executor):
    """libfbp on one GPU: one torch stream and one batch workspace per stream slot."""

    def __init__(self, n_streams: int = 2, precision: str = "fp32", device: str = "cuda"):
        import torch
        self.torch = torch
        self.n_streams = n_streams
        self.precision = precision
        self.device = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self.workspaces = [None] * n_streams

    def allocate_output(self, req: Request):
        g = req.geom
        return self.torch.empty((req.n_slices, g.image_size, g.image_size), dtype=self.torch.float32,
                                device=self.device)

    def launch(self, stream_idx: int, reqs: list):
        from . import _binding as fbp
        torch = self.torch
        jobs = []
        for r in reqs:
            for b in range(r.n_slices):
                jobs.append((r.geom, r.sino[b], r.output[b]))
        stream = self.streams[stream_idx]
        need = fbp.fbp_batch_workspace_bytes(jobs, self.precision)
        ws = self.workspaces[stream_idx]
        if ws is None or ws.numel() < need:
            # grown outside any captured region; the old buffer's last use is ordered
            # before this point on the same stream
            with torch.cuda.stream(stream):
                ws = fbp.alloc_workspace(max(need, 1 << 20), self.device)
            self.workspaces[stream_idx] = ws
        with torch.cuda.stream(stream):
            fbp.fbp_reconstruct_batch(jobs, workspace=ws, precision=self.precision, stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev

    def wait(self, handle) -> None:
        handle.synchronize()


class Server:
    """Continuous batching over `executor.n_streams` streams under an HBM budget."""

    def __init__(self, executor: Executor, hbm_budget_bytes: int, max_batch_slices: int = 4096,
                 max_batch_cost: int = DEFAULT_BATCH_COST, clock=time.perf_counter):
        self.ex = executor
        self.budget = int(hbm_budget_bytes)
        self.max_batch_slices = max_batch_slices
        self.max_batch_cost = max_batch_cost
        self.clock = clock
        self._lock = threading.Condition()
        self._pending = collections.deque()      # arrived, not admitted (FIFO)
        self._admitted = collections.deque()     # admitted, not launched
        self._free_streams = list(range(executor.n_streams))
        self._in_use = 0
        self._ids = itertools.count()
        self._stop = False
        self.latencies = []                      # seconds, per completed request
        self.completed_slices = 0
        self.failed = 0
        self.batches = 0
        self.max_in_use = 0
        self._waiters = []
        self._inflight = [collections.deque() for _ in range(executor.n_streams)]
        self._sched = threading.Thread(target=self._schedule_loop, daemon=True)
        for s in range(executor.n_streams):
            th = threading.Thread(target=self._wait_loop, args=(s,), daemon=True)
            th.start()
            self._waiters.append(th)
        self._sched.start()

    # -------------------------------------------------------------- client side
    def submit(self, geom, sino, n_slices: int = None) -> Future:
        n = int(sino.shape[0]) if n_slices is None else int(n_slices)
        req = Request(geom=geom, sino=sino, n_slices=n,
                      nbytes=footprint_bytes(geom.n_angles, geom.n_det, geom.image_size, n),
                      cost=request_cost(geom.n_angles, geom.image_size, n))
        req.arrival = self.clock()
        req.rid = next(self._ids)
        if req.nbytes > self.budget:
            req.future.set_exception(RequestTooLarge(
                f"request needs {req.nbytes} bytes, budget is {self.budget}"))
            return req.future
        with self._lock:
            if self._stop:
                raise RuntimeError("server is shut down")
            self._pending.append(req)
            self._lock.notify_all()
        return req.future

    def drain(self, timeout: float = None) -> bool:
        """Wait until every submitted request has completed."""
        deadline = None if timeout is None else self.clock() + timeout
        with self._lock:
            while self._pending or self._admitted or self._in_use:
                left = None if deadline is None else deadline - self.clock()
                if left is not None and left <= 0:
                    return False
                self._lock.wait(timeout=0.05 if left is None else min(0.05, left))
        return True

    def shutdown(self):
        with self._lock:
            self._stop = True
            self._lock.notify_all()
        self._sched.join(timeout=5)
        for th in self._waiters:
            th.join(timeout=5)

    def stats(self) -> dict:
        lat = sorted(self.latencies)

        def pct(p):
            if not lat:
                return math.nan
            return lat[min(len(lat) - 1, int(math.ceil(p / 100.0 * len(lat))) - 1)]
        return {"completed": len(lat), "failed": self.failed, "slices": self.completed_slices,
                "batches": self.batches, "p50_ms": pct(50) * 1e3, "p99_ms": pct(99) * 1e3,
                "max_in_use_bytes": self.max_in_use}

    # -------------------------------------------------------------- scheduler
    def _admit_locked(self):
        # strict arrival order: the head waits for memory, later requests wait behind it
        while self._pending and self._in_use + self._pending[0].nbytes <= self.budget:
            req = self._pending.popleft()
            try:
                req.output = self.ex.allocate_output(req)
            except Exception as e:   # allocation failure fails this request only
                self.failed += 1
                req.future.set_exception(e)
                continue
            self._in_use += req.nbytes
            self.max_in_use = max(self.max_in_use, self._in_use)
            self._admitted.append(req)

    def _schedule_loop(self):
        while True:
            with self._lock:
                while not self._stop:
                    self._admit_locked()
                    if self._admitted and self._free_streams:
                        break
                    self._lock.wait(timeout=0.05)
                if self._stop:
                    return
                s = self._free_streams.pop(0)
                batch, n, cost = [], 0, 0
                while self._admitted and (not batch or (n + self._admitted[0].n_slices <= self.max_batch_slices and
                                                        cost + self._admitted[0].cost <= self.max_batch_cost)):
                    r = self._admitted.popleft()
                    batch.append(r)
                    n += r.n_slices
                    cost += r.cost
            try:
                handle = self.ex.launch(s, batch)
            except Exception as e:   # launch failure: fail the batch, free its memory and stream
                with self._lock:
                    for r in batch:
                        self._in_use -= r.nbytes
                        self.failed += 1
                        r.future.set_exception(e)
                    self._free_streams.append(s)
                    self._lock.notify_all()
                continue
            with self._lock:
                self.batches += 1
                self._inflight[s].append((handle, batch))
                self._lock.notify_all()

    def _wait_loop(self, s: int):
        while True:
            with self._lock:
                while not self._inflight[s] and not self._stop:
                    self._lock.wait(timeout=0.05)
                if not self._inflight[s] and self._stop:
                    return
                handle, batch = self._inflight[s][0]
            err = None
            try:
                self.ex.wait(handle)
            except Exception as e:
                err = e
            done = self.clock()
            with self._lock:
                self._inflight[s].popleft()
                for r in batch:
                    self._in_use -= r.nbytes
                    if err is None:
                        self.latencies.append(done - r.arrival)
                        self.completed_slices += r.n_slices
                    else:
                        self.failed += 1
                self._free_streams.append(s)
                self._lock.notify_all()
            for r in batch:
                if err is None:
                    r.future.set_result(r.output)
                else:
                    r.future.set_exception(err)
