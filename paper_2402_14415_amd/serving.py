"""Serving form: SDF + normal queries against several resident grids, continuously batched.

A request asks for the field value and the unit normal (gradient / |gradient|, zero where the
gradient vanishes) of one resident grid (Sec. 3.1, Eq. 2-4) at n points.  The server

  * admits requests in arrival order while their in-flight footprint fits an HBM budget
    (footprint = bytes of the request's points and outputs: 4 * n * (2 * dim + 1));
  * cuts admitted requests into chunks of at most ``chunk_points`` and forms each launch
    from the chunks of up to ``max_reqs`` requests (any mix of grids), round robin, so a
    small request that arrives behind a huge one rides in the next launch instead of
    waiting for the huge one to finish;
  * keeps up to ``depth`` launches in flight over ``streams`` HIP streams, so launches
    overlap on the device, and admits new requests as soon as earlier ones complete and
    release their footprint.

Every launch is one ``tg_query`` call (one kernel per 32 requests / 16 grids) whose
per-point arithmetic does not depend on the rest of the launch, so a request's result is
the same alone and in any mix.

The scheduler is host logic only; ``GpuExecutor`` is the piece that touches the device.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np


@dataclass(eq=False)
class Request:
    rid: int
    grid: int
    n: int
    q: object                      # [n, dim] FP32 points (device tensor for the GPU executor)
    t_arrival: float
    sdf: object = None             # [n] output, allocated at admission
    normal: object = None          # [n, dim] output, allocated at admission
    footprint: int = 0
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    next: int = 0                  # first point not yet handed to a launch
    pending: int = 0               # launches in flight that carry a chunk of this request
    ready: object = None           # executor-specific marker that q is ready

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival

    @property
    def done(self) -> bool:
        return self.t_done is not None


@dataclass
class _Launch:
    token: object
    chunks: List[Tuple[Request, int, int]] = field(default_factory=list)


def request_footprint(n: int, dim: int) -> int:
    """HBM bytes a request holds while in flight: points (dim floats), value, normal."""
    return 4 * int(n) * (2 * int(dim) + 1)


class Server:
    """Continuous-batching request loop with HBM-footprint admission.

    ``grids`` are resident grids (``TaylorGrid``); ``executor`` defaults to a GPU executor
    on the grids' device.  ``clock`` returns seconds.
    """

    def __init__(self, grids: Sequence, budget_bytes: int = 1 << 30, *, streams: int = 2, depth: int = 4,
                 chunk_points: int = 1 << 20, max_reqs: int = 32, executor=None,
                 clock: Callable[[], float] = time.perf_counter):
        if not grids:
            raise ValueError("at least one grid is required")
        dims = {int(g.dim) for g in grids}
        if len(dims) != 1:
            raise ValueError("all grids of a server must have the same dimension")
        if budget_bytes <= 0 or depth < 1 or streams < 1 or chunk_points < 1 or not 1 <= max_reqs <= 32:
            raise ValueError("invalid server limits")
        self.grids = list(grids)
        self.dim = dims.pop()
        self.budget = int(budget_bytes)
        self.depth = int(depth)
        self.chunk_points = int(chunk_points)
        self.max_reqs = int(max_reqs)
        self.clock = clock
        self.executor = executor if executor is not None else GpuExecutor(self.grids, streams)
        self._waiting: collections.deque = collections.deque()
        self._active: collections.deque = collections.deque()
        self._inflight: List[_Launch] = []
        self._next_rid = 0
        self.used_bytes = 0
        self.peak_bytes = 0
        self.launches = 0
        self.completed: List[Request] = []

    # ------------------------------------------------------------------ client side
    def submit(self, grid: int, q, arrival: Optional[float] = None) -> Request:
        """Queue a request for grid index ``grid`` at points ``q`` ([n, dim] FP32)."""
        if not 0 <= int(grid) < len(self.grids):
            raise IndexError(f"grid {grid} out of range")
        n = self.executor.check_points(q, self.dim)
        fp = request_footprint(n, self.dim)
        if fp > self.budget:
            raise ValueError(f"request of {n} points needs {fp} bytes, above the budget of {self.budget}")
        t = self.clock() if arrival is None else float(arrival)
        r = Request(self._next_rid, int(grid), n, q, t, footprint=fp)
        self._next_rid += 1
        r.ready = self.executor.mark_ready(q)
        self._waiting.append(r)
        self._admit()
        self._launch()
        return r

    def poll(self) -> List[Request]:
        """Retire finished launches, admit and launch more; returns requests finished now."""
        finished: List[Request] = []
        still: List[_Launch] = []
        for L in self._inflight:
            if self.executor.done(L.token):
                now = self.clock()
                for r, _, _ in L.chunks:
                    r.pending -= 1
                    if r.pending == 0 and r.next == r.n:
                        r.t_done = now
                        self.used_bytes -= r.footprint
                        finished.append(r)
            else:
                still.append(L)
        self._inflight = still
        self._admit()
        self._launch()
        self.completed.extend(finished)
        return finished

    def reset_stats(self) -> None:
        """Forget finished requests and reset the peak-footprint and launch counters."""
        self.completed = []
        self.peak_bytes = self.used_bytes
        self.launches = 0

    def busy(self) -> bool:
        return bool(self._waiting or self._active or self._inflight)

    def drain(self) -> List[Request]:
        """Poll until every submitted request has finished."""
        out: List[Request] = []
        while self.busy():
            out.extend(self.poll())
        return out

    # ------------------------------------------------------------------ scheduler
    def _admit(self) -> None:
        while self._waiting and self.used_bytes + self._waiting[0].footprint <= self.budget:
            r = self._waiting.popleft()
            r.t_admit = self.clock()
            self.used_bytes += r.footprint
            self.peak_bytes = max(self.peak_bytes, self.used_bytes)
            if r.n == 0:
                r.sdf, r.normal = self.executor.alloc(0, self.dim)
                r.t_done = r.t_admit
                self.used_bytes -= r.footprint
                self.completed.append(r)
                continue
            r.sdf, r.normal = self.executor.alloc(r.n, self.dim)
            self._active.append(r)

    def _launch(self) -> None:
        while len(self._inflight) < self.depth and self._active:
            chunks: List[Tuple[Request, int, int]] = []
            for r in self._active:
                if len(chunks) == self.max_reqs:
                    break
                take = min(r.n - r.next, self.chunk_points)
                chunks.append((r, r.next, r.next + take))
                r.next += take
                r.pending += 1
            # requests whose points are all handed out leave the active list; the rest
            # rotate to the back so the next launch starts with a different request
            head = len(chunks)
            rest = [self._active.popleft() for _ in range(head)]
            for r in rest:
                if r.next < r.n:
                    self._active.append(r)
            token = self.executor.launch(chunks)
            self._inflight.append(_Launch(token, chunks))
            self.launches += 1


# ---------------------------------------------------------------------- GPU executor
class GpuExecutor:
    """Runs launches with ``tg_query`` on a small pool of HIP streams (default priority)."""

    def __init__(self, grids, streams: int = 2):
        import torch

        self._torch = torch
        self.grids = list(grids)
        self.device = self.grids[0].device
        self.streams = [torch.cuda.Stream(self.device) for _ in range(streams)]
        self._turn = 0

    def check_points(self, q, dim: int) -> int:
        torch = self._torch
        if not isinstance(q, torch.Tensor) or q.dtype != torch.float32 or q.device != self.device:
            raise TypeError(f"points must be a float32 tensor on {self.device}")
        if q.dim() != 2 or q.shape[1] != dim or not q.is_contiguous():
            raise ValueError(f"points must be a contiguous [n, {dim}] tensor")
        return int(q.shape[0])

    def mark_ready(self, q):
        ev = self._torch.cuda.Event()
        ev.record(self._torch.cuda.current_stream(self.device))
        return ev

    def alloc(self, n: int, dim: int):
        torch = self._torch
        return (torch.empty(n, dtype=torch.float32, device=self.device),
                torch.empty((n, dim), dtype=torch.float32, device=self.device))

    def launch(self, chunks):
        from .grid import query

        s = self.streams[self._turn % len(self.streams)]
        self._turn += 1
        # The server keeps every chunk's tensors referenced until the launch's event has
        # been seen complete, so no record_stream is needed for the caching allocator.
        reqs = []
        for r, a, b in chunks:
            s.wait_event(r.ready)
            reqs.append((r.grid, r.q[a:b], r.sdf[a:b], r.normal[a:b]))
        query(self.grids, reqs, stream=s)
        ev = self._torch.cuda.Event()
        ev.record(s)
        return ev

    def done(self, token) -> bool:
        return token.query()


# ---------------------------------------------------------------------- workload driver
def latency_stats(reqs: Sequence[Request]) -> dict:
    lat = np.array([r.latency for r in reqs], dtype=np.float64)
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "mean_ms": None, "max_ms": None}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3)}


def run_trace(server: Server, trace: Sequence[Tuple[float, int, object]]) -> dict:
    """Replay ``trace`` = [(arrival offset in s, grid, points)] in real time on ``server``.

    Requests are submitted when the clock passes their arrival time (latency counts from
    the scheduled arrival, so a late submit is charged to the server); returns latency
    percentiles, points per second over the makespan and the peak in-flight footprint.
    """
    if server.busy():
        raise RuntimeError("run_trace needs an idle server")
    order = sorted(range(len(trace)), key=lambda i: trace[i][0])
    server.reset_stats()
    t0 = server.clock()
    i = 0
    while i < len(order) or server.busy():
        now = server.clock() - t0
        while i < len(order) and trace[order[i]][0] <= now:
            t, g, q = trace[order[i]]
            server.submit(g, q, arrival=t0 + t)
            i += 1
        server.poll()
    t1 = server.clock()
    done = list(server.completed)
    pts = sum(r.n for r in done)
    out = latency_stats(done)
    out.update({"requests": len(done), "points": int(pts), "seconds": t1 - t0,
                "queries_per_s": pts / (t1 - t0) if t1 > t0 else None,
                "peak_inflight_bytes": int(server.peak_bytes), "launches": int(server.launches)})
    return out
