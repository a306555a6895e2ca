"""Continuous-batching server for FRNN graph building.

Requests (one event each) arrive over time.  The server admits a request when a
slot is free and its device footprint fits the HBM budget, starts its upload at
once, and groups admitted requests into batches that run on one of several
streams, so requests that arrive while others are on the GPU join the next batch
and their work overlaps on the device with batches already running.  Grids and
edge buffers stay on the device; a request completes when its edge range is
known, and its memory is released then.

The executor is pluggable: GpuExecutor drives the HIP library through
frnn_build_batch_async; tests use a CPU executor with a simulated clock.
"""

from __future__ import annotations

import dataclasses
import time
from collections import deque
from typing import Callable, Protocol

import numpy as np

OK, REJECTED, FAILED, CANCELLED, TIMED_OUT = 0, -1, -2, -3, -4


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float              # seconds on the server clock
    points: object              # float32 [n, d]: a numpy array or a device tensor
    admitted: float | None = None
    started: float | None = None
    done: float | None = None
    status: int | None = None   # OK, REJECTED, FAILED or a library status
    edges: object = None        # int64 [2, E] (device tensor for the GPU executor)
    batch: int | None = None
    timeout: float | None = None  # seconds after arrival by which the request must have started

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def latency(self) -> float | None:
        return None if self.done is None else self.done - self.arrival


class Executor(Protocol):
    def footprint(self, req: Request) -> int: ...
    def admit(self, req: Request) -> None: ...
    def start(self, batch: list[Request]) -> object: ...
    def poll(self, handle: object) -> bool: ...
    def finish(self, handle: object) -> list[tuple[int, object]]: ...
    def abort(self, handle: object) -> None: ...
    def release(self, req: Request) -> None: ...
    def free_streams(self) -> int: ...


@dataclasses.dataclass
class ServerStats:
    completed: int
    rejected: int
    failed: int
    cancelled: int
    timed_out: int
    batches: int
    wall: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    events_per_s: float
    max_in_flight: int
    mean_batch: float

    def as_dict(self) -> dict:
        return dataclasses.asdict(self)


class Server:
    """Admission by slots and HBM budget, batching, completion tracking.

    A request that has not started may be cancelled (cancel(rid)) or may carry a
    timeout (seconds after its arrival by which it must have started); either way
    it completes without running, with status CANCELLED or TIMED_OUT, and its
    admission (slot and budget) is returned.  Work already on the GPU runs to its
    end."""

    def __init__(self, executor: Executor, hbm_budget: int, max_slots: int = 256, max_batch: int = 64,
                 clock: Callable[[], float] | None = None, idle: Callable[[float], None] | None = None):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_slots = max_slots
        self.max_batch = max_batch
        self.clock = clock or time.perf_counter
        self.idle = idle or (lambda until: None)
        self.used = 0
        self.in_flight: list[tuple[object, list[Request]]] = []
        self.slots = 0
        self._cancel: set[int] = set()
        self._timeouts = False

    def cancel(self, rid: int) -> None:
        """Cancels request rid if it has not started by the server's next look at it."""
        self._cancel.add(rid)

    def _dropped(self, req: Request, now: float) -> int | None:
        if req.rid in self._cancel:
            return CANCELLED
        if req.timeout is not None and now > req.arrival + req.timeout:
            return TIMED_OUT
        return None

    def run(self, trace: list[Request]) -> ServerStats:
        pending = deque(sorted(trace, key=lambda q: q.arrival))
        self._timeouts = any(q.timeout is not None for q in trace)
        waiting: deque[Request] = deque()    # arrived, not admitted
        admitted: deque[Request] = deque()   # admitted, not started
        done: list[Request] = []
        t0 = self.clock()
        batches = 0
        batch_sizes = []
        max_in_flight = 0
        while pending or waiting or admitted or self.in_flight:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # Cancelled or expired requests leave before they take (or after they
            # return) a slot and their share of the budget.
            for queue, holds in ((waiting, False), (admitted, True)):
                if not queue or not (self._cancel or self._timeouts):
                    continue
                keep = deque()
                for req in queue:
                    why = self._dropped(req, now)
                    if why is None:
                        keep.append(req)
                    elif holds:
                        self._complete(req, why, None, now, done)
                    else:
                        req.status, req.done = why, now
                        done.append(req)
                queue.clear()
                queue.extend(keep)
            # Admission in arrival order: a free slot and room in the budget.
            while waiting and self.slots < self.max_slots:
                req = waiting[0]
                need = self.ex.footprint(req)
                if need > self.budget:
                    waiting.popleft()
                    req.status, req.done = REJECTED, now
                    done.append(req)
                    continue
                if self.used + need > self.budget:
                    break
                waiting.popleft()
                self.used += need
                self.slots += 1
                req.admitted = now
                self.ex.admit(req)
                admitted.append(req)
            # Dispatch: every admitted request joins the next batch on a free stream.
            while admitted and self.ex.free_streams() > 0:
                batch = [admitted.popleft() for _ in range(min(self.max_batch, len(admitted)))]
                for req in batch:
                    req.started, req.batch = now, batches
                try:
                    handle = self.ex.start(batch)
                except Exception:
                    for req in batch:
                        self._complete(req, FAILED, None, self.clock() - t0, done)
                    continue
                self.in_flight.append((handle, batch))
                batches += 1
                batch_sizes.append(len(batch))
            max_in_flight = max(max_in_flight, sum(len(b) for _, b in self.in_flight))
            # Completions.  A batch whose poll or finish raises fails as a whole and
            # gives its stream back through abort().
            still = []
            for handle, batch in self.in_flight:
                try:
                    ready = self.ex.poll(handle)
                except Exception:
                    ready = None
                if ready is False:
                    still.append((handle, batch))
                    continue
                t_done = self.clock() - t0
                results = None
                if ready:
                    try:
                        results = self.ex.finish(handle)
                    except Exception:
                        results = None
                if results is None:
                    self.ex.abort(handle)
                for k, req in enumerate(batch):
                    st, edges = results[k] if results is not None else (FAILED, None)
                    self._complete(req, st, edges, t_done, done)
            self.in_flight = still
            if not self.in_flight and not admitted and not waiting and pending:
                self.idle(pending[0].arrival + t0)
        wall = self.clock() - t0
        lat = np.array([r.latency for r in done if r.status == OK], dtype=np.float64) * 1e3
        n_ok = int(lat.size)
        return ServerStats(
            completed=n_ok, rejected=sum(r.status == REJECTED for r in done),
            failed=sum(r.status not in (OK, REJECTED, CANCELLED, TIMED_OUT) for r in done),
            cancelled=sum(r.status == CANCELLED for r in done), timed_out=sum(r.status == TIMED_OUT for r in done),
            batches=batches, wall=wall,
            p50_ms=float(np.percentile(lat, 50)) if n_ok else float("nan"),
            p99_ms=float(np.percentile(lat, 99)) if n_ok else float("nan"),
            mean_ms=float(lat.mean()) if n_ok else float("nan"),
            events_per_s=n_ok / wall if wall > 0 else float("nan"),
            max_in_flight=max_in_flight, mean_batch=float(np.mean(batch_sizes)) if batch_sizes else 0.0)

    def _complete(self, req: Request, status: int, edges, t_done: float, done: list) -> None:
        req.status, req.edges, req.done = status, edges, t_done
        self.used -= self.ex.footprint(req)
        self.slots -= 1
        self.ex.release(req)
        done.append(req)


def plain_loop(trace: list[Request], build: Callable[[Request], object],
               clock: Callable[[], float] | None = None,
               idle: Callable[[float], None] | None = None) -> ServerStats:
    """The baseline: one call per event in arrival order, each waiting for the last."""
    clock = clock or time.perf_counter
    idle = idle or (lambda until: None)
    t0 = clock()
    lat = []
    for req in sorted(trace, key=lambda q: q.arrival):
        now = clock() - t0
        if now < req.arrival:
            idle(req.arrival + t0)
        req.started = clock() - t0
        req.edges = build(req)
        req.done = clock() - t0
        req.status = OK
        lat.append(req.latency * 1e3)
    wall = clock() - t0
    lat = np.array(lat)
    return ServerStats(completed=len(lat), rejected=0, failed=0, cancelled=0, timed_out=0, batches=len(lat), wall=wall,
                       p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                       mean_ms=float(lat.mean()), events_per_s=len(lat) / wall, max_in_flight=1, mean_batch=1.0)


class GpuExecutor:
    """Runs batches through frnn_build_events_async on a few streams.

    Requests hold their points on the device already (the embedding stage that
    produces them runs on the GPU).  A batch passes the events' device pointers to
    the library, which searches each event on its own grid.  Its workspace and edge
    buffer come from PyTorch's caching allocator on the batch's stream (a memory
    pool: no device allocation call once the pool is warm).  When the batch
    completes, the workspace goes back to the pool at once; each request receives a
    view of the edge buffer, recorded on the completing thread's current stream so
    that the pool does not hand the memory out again while that stream may still
    read it; the buffer returns to the pool when the last view is dropped.
    `live_bytes` counts the workspace and edge-buffer bytes of batches not yet
    completed.
    """

    def __init__(self, r: float, K: int, d: int, n_streams: int = 3, config=None, edges_per_point: int = 16,
                 device: str = "cuda:0"):
        import torch

        from . import frnn
        self.torch, self.frnn = torch, frnn
        self.r, self.K, self.d = r, K, d
        self.config = config
        self.epp = edges_per_point
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.busy = [False] * n_streams
        self.live_bytes = 0

    def footprint(self, req: Request) -> int:
        n = max(req.n, 1)
        offs = np.array([0, n], dtype=np.int64)
        return int(self.frnn.batch_workspace_bytes(offs, self.d)) + 16 * self.epp * n

    def admit(self, req: Request) -> None:
        pass

    def free_streams(self) -> int:
        return self.busy.count(False)

    def start(self, batch: list[Request]):
        torch, frnn = self.torch, self.frnn
        k = self.busy.index(False)
        s = self.streams[k]
        sizes = [req.n for req in batch]
        offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        rows = int(offsets[-1])
        cap = max(1024, self.epp * rows)
        s.wait_stream(torch.cuda.current_stream(self.device))  # the points were produced there
        with torch.cuda.stream(s):
            ws = torch.empty(frnn.batch_workspace_bytes(offsets, self.d), dtype=torch.uint8, device=self.device)
            out = torch.empty((2, cap), dtype=torch.int64, device=self.device)
            eo = torch.empty(len(batch) + 2, dtype=torch.int64, device=self.device)
            if rows > 0:
                st = frnn.build_events_async([req.points for req in batch], self.r, self.K, ws, out[0], out[1],
                                             eo, self.config)
                if st != frnn.FRNN_OK:
                    raise frnn.FrnnError(st, frnn.status_string(st))
            else:
                eo.zero_()
            done = torch.cuda.Event()
            done.record(s)
        self.busy[k] = True
        held = ws.numel() + out.numel() * 8
        self.live_bytes += held
        return {"stream": k, "event": done, "out": out, "eo": eo, "batch": batch, "ws": ws, "held": held}

    def poll(self, handle) -> bool:
        return handle["event"].query()

    def _drop(self, handle) -> None:
        """Gives the batch's stream back and its workspace to the pool (once)."""
        if handle.get("held"):
            self.busy[handle["stream"]] = False
            self.live_bytes -= handle["held"]
            handle["held"] = 0
            handle["ws"] = None

    def abort(self, handle) -> None:
        self._drop(handle)
        handle["out"] = None

    def finish(self, handle):
        torch, frnn = self.torch, self.frnn
        self._drop(handle)
        eo = handle["eo"].cpu().numpy()
        batch = handle["batch"]
        out = handle.pop("out")
        status = int(eo[-1])
        if status == 3:  # more edges than the guess: rebuild each event with exact room
            return [(OK, frnn.build(req.points, self.r, self.K, self.config)) for req in batch]
        if status != 0:
            return [(status, None) for _ in batch]
        out.record_stream(torch.cuda.current_stream(self.device))
        return [(OK, out[:, int(eo[k]):int(eo[k + 1])]) for k in range(len(batch))]

    def release(self, req: Request) -> None:
        pass
