"""Serving: continuous batching of counting requests on one GPU.

A request asks for the colour-coding estimate of one tree template on one resident graph with B
colourings (Algorithm 1's outer loop). Requests arrive over time; the server

  * admits work by count-table memory: a request's colourings are cut into slots of one
    colouring each, and a slot is admitted only when the device memory its tables need
    (the plan's table arena, the graph's chunk partials, the per-vertex root counts) fits in the
    budget next to everything in flight;
  * forms batches continuously: whenever fewer than `max_inflight` batches are on the device, it
    packs admissible slots of the oldest waiting requests (first come, first served, several
    requests per batch) into one batch and launches it on its own stream, so that newly arrived
    requests join while others are still running and their work overlaps on the device;
  * optionally caps the colourings one request puts into one batch (`slot_colourings`): a large
    request then advances a slice per batch and the requests behind it share every batch, instead
    of waiting behind it (head-of-line blocking); memory admission stays first come, first
    served (a request that does not fit stops the scan);
  * completes a request when all of its colourings are back, and records its latency
    (arrival to completion) and estimate.

Every colouring of a request is counted by the same kernels and in the same order as a plain
count, so a request's result does not depend on what it was batched with.

The scheduling logic is independent of the GPU: `Server` drives an `Executor`; `GpuExecutor`
runs batches through the C ABI, and tests substitute a simulated executor and clock.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass(eq=False)
class Request:
    rid: int
    graph_id: int
    tree_edges: np.ndarray
    B: int
    seed: int
    arrival: float
    # filled by the server
    X: np.ndarray = None
    estimate: float = None
    std_err: float = None
    done: float = None
    status: str = "waiting"  # waiting | running | done | failed | cancelled
    error: str = None
    next_colouring: int = 0   # first colouring not yet admitted
    finished: int = 0         # colourings whose X is back

    @property
    def k(self) -> int:
        return len(self.tree_edges) + 1

    @property
    def latency(self) -> float | None:
        return None if self.done is None else self.done - self.arrival


@dataclass(eq=False)
class Slot:
    """Colourings [first, first + count) of one request, all in one batch."""
    req: Request
    first: int
    count: int
    nbytes: int


class Executor:
    """What the server needs from a device."""

    def slot_bytes(self, req: Request, count: int = 1) -> int:  # memory of `count` colourings of `req`
        raise NotImplementedError

    def launch(self, slots: list[Slot]):  # returns a handle
        raise NotImplementedError

    def poll(self, handle) -> bool:
        raise NotImplementedError

    def collect(self, handle) -> list[np.ndarray]:  # X values per slot, in order
        raise NotImplementedError

    def estimate(self, req: Request, X: np.ndarray) -> tuple[float, float]:
        raise NotImplementedError


@dataclass
class Stats:
    batches: int = 0
    slots: int = 0
    max_inflight_bytes: int = 0
    max_inflight_batches: int = 0
    batch_sizes: list = field(default_factory=list)


class Server:
    def __init__(self, executor: Executor, memory_budget: int, max_inflight: int = 2,
                 max_colourings_per_batch: int = 256, clock=time.perf_counter, on_complete=None,
                 slot_colourings: int = 0):
        self.ex = executor
        self.on_complete = on_complete
        self.budget = int(memory_budget)
        self.max_inflight = max_inflight
        self.max_slots = max_colourings_per_batch
        self.slot_cap = int(slot_colourings)  # 0: a request takes as many colourings as fit
        self.clock = clock
        self.queue: deque[Request] = deque()
        self.inflight: list = []  # (handle, slots, nbytes)
        self.inflight_bytes = 0
        self.completed: list[Request] = []
        self.stats = Stats()

    # -- request side ------------------------------------------------------------------------
    def submit(self, req: Request):
        req.X = np.full(req.B, np.nan)
        req.status = "waiting"
        need = self.ex.slot_bytes(req)
        if need > self.budget:
            req.status = "failed"
            req.error = f"one colouring needs {need} bytes, more than the budget {self.budget}"
            req.done = self.clock()
            self.completed.append(req)
            return
        self.queue.append(req)

    def cancel(self, rid: int) -> bool:
        """Cancel a request none of whose colourings has been admitted yet."""
        for r in list(self.queue):
            if r.rid == rid and r.next_colouring == 0:
                self.queue.remove(r)
                r.status = "cancelled"
                r.done = self.clock()
                self.completed.append(r)
                return True
        return False

    # -- device side -------------------------------------------------------------------------
    def _form_batch(self) -> list[Slot]:
        """Pack admissible colourings of the oldest waiting requests into one batch. Requests are
        served first come, first served: a request whose colourings do not fit in the memory left
        stops the scan, so later requests never overtake it; a request that reached its per-batch
        cap (`slot_colourings`) lets the next ones in."""
        slots: list[Slot] = []
        free = self.budget - self.inflight_bytes
        left = self.max_slots
        for req in self.queue:
            per = self.ex.slot_bytes(req, 1)
            want = min(req.B - req.next_colouring, left)
            if self.slot_cap > 0:
                want = min(want, self.slot_cap)
            cnt = int(min(want, free // per))
            # a slot's memory need not be exactly linear in its colourings: shrink until it fits
            while cnt > 0 and self.ex.slot_bytes(req, cnt) > free:
                cnt = cnt - max(1, cnt // 8)
            if cnt > 0:
                need = int(self.ex.slot_bytes(req, cnt))
                slots.append(Slot(req, req.next_colouring, cnt, need))
                req.next_colouring += int(cnt)
                req.status = "running"
                left -= cnt
                free -= need
            if cnt < want or left == 0:
                break
        self.queue = deque(r for r in self.queue if r.next_colouring < r.B)
        return slots

    def _finish(self, r: Request, now: float):
        r.done = now
        self.completed.append(r)
        if self.on_complete is not None:
            self.on_complete(r)

    def _complete(self, handle, slots: list[Slot], nbytes: int):
        try:
            values = self.ex.collect(handle)
            error = None
        except Exception as exc:  # the batch failed: fail its requests, free its memory
            values = None
            error = f"{type(exc).__name__}: {exc}"
        now = self.clock()
        self.inflight_bytes -= nbytes
        for i, s in enumerate(slots):
            r = s.req
            r.finished += s.count
            if error is not None:
                if r.status != "failed":
                    r.status = "failed"
                    r.error = error
                    if r in self.queue:
                        self.queue.remove(r)  # admit nothing more of it
            else:
                r.X[s.first:s.first + s.count] = values[i]
            if r.status == "failed":
                if r.done is None and r.finished >= r.next_colouring:
                    self._finish(r, now)
            elif r.finished >= r.B:
                r.estimate, r.std_err = self.ex.estimate(r, r.X)
                r.status = "done"
                self._finish(r, now)

    def step(self) -> bool:
        """Retire finished batches and launch new ones; returns True if anything happened."""
        progressed = False
        still = []
        for entry in self.inflight:
            if self.ex.poll(entry[0]):
                self._complete(*entry)
                progressed = True
            else:
                still.append(entry)
        # drop every reference to finished batches (their device memory) before launching more
        entry = None
        self.inflight = still
        while len(self.inflight) < self.max_inflight and self.queue:
            slots = self._form_batch()
            if not slots:
                break
            nbytes = sum(s.nbytes for s in slots)
            handle = self.ex.launch(slots)
            self.inflight.append((handle, slots, nbytes))
            self.inflight_bytes += nbytes
            self.stats.batches += 1
            self.stats.slots += len(slots)
            self.stats.batch_sizes.append(sum(s.count for s in slots))
            self.stats.max_inflight_bytes = max(self.stats.max_inflight_bytes, self.inflight_bytes)
            self.stats.max_inflight_batches = max(self.stats.max_inflight_batches, len(self.inflight))
            progressed = True
        return progressed

    def idle(self) -> bool:
        return not self.queue and not self.inflight

    def run(self, requests: list[Request], sleep=time.sleep, poll_interval: float = 2e-4):
        """Feed `requests` at their arrival times (seconds after start) and serve until all are done."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        t0 = self.clock()
        for r in pending:
            r.arrival += t0
        while pending or not self.idle():
            now = self.clock()
            while pending and pending[0].arrival <= now:
                self.submit(pending.popleft())
            if not self.step():
                nxt = pending[0].arrival - now if pending else poll_interval
                sleep(max(0.0, min(poll_interval, nxt)))
        return self.completed


class _Fixed:
    """An already allocated workspace (the Workspace interface that count_packed uses)."""

    def __init__(self, buf):
        self.buf = buf

    def get(self, nbytes, device):
        if self.buf.numel() < nbytes:
            raise ValueError("workspace too small")
        return self.buf


def latency_summary(reqs: list[Request]) -> dict:
    lat = np.array([r.latency for r in reqs if r.status == "done"])
    if len(lat) == 0:
        return {"n": 0}
    return {"n": int(len(lat)), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max())}


# ------------------------------------------------------------------------------------------------
# GPU executor
# ------------------------------------------------------------------------------------------------

class GpuExecutor(Executor):
    """Runs each slot of a batch as one packed count (cc_count_packed: the slot's colourings share
    every table row and every pass over the graph), the batch's slots back to back on the batch's
    HIP stream, batches on alternating streams; graphs stay resident in `graphs` (a list of
    Graph)."""

    def __init__(self, graphs, device="cuda:0", seed_base: int = 0, n_streams: int = 2):
        import torch
        from . import Plan
        self.torch = torch
        self.graphs = graphs
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self._rr = 0
        self._plans: dict = {}
        self._bytes: dict = {}
        self._Plan = Plan
        self.seed_base = seed_base

    def plan(self, req: Request):
        key = req.tree_edges.tobytes()
        p = self._plans.get(key)
        if p is None:
            p = self._Plan(req.tree_edges, device=self.device)
            self._plans[key] = p
        return p

    def slot_bytes(self, req: Request, count: int = 1) -> int:
        """Device bytes of `count` colourings of `req` counted together: the packed-count
        workspace of its plan on its graph (table arena, chunk partials, root counts, colour
        transpose), plus the colours and results."""
        from . import count_packed_workspace_bytes
        g = self.graphs[req.graph_id]
        key = (req.tree_edges.tobytes(), req.graph_id, int(count))
        b = self._bytes.get(key)
        if b is None:
            b = count_packed_workspace_bytes(self.plan(req), g, int(count)) + count * (g.n + 8) + 256
            self._bytes[key] = b
        return b

    def launch(self, slots: list[Slot]):
        import paper_1804_09764_amd as cc
        torch = self.torch
        st = self.streams[self._rr % len(self.streams)]
        self._rr += 1
        keep, outs = [], []
        # device buffers come from the allocator's default-stream pool and are marked as used on
        # the batch's stream, so memory freed by one batch can be reused by the next on any stream
        for s in slots:
            g = self.graphs[s.req.graph_id]
            p = self.plan(s.req)
            C = torch.empty((s.count, g.n), dtype=torch.uint8, device=self.device)
            X = torch.empty(s.count, dtype=torch.float64, device=self.device)
            ws = torch.empty(max(cc.count_packed_workspace_bytes(p, g, s.count), 256), dtype=torch.uint8,
                             device=self.device)
            for t in (C, X, ws):
                t.record_stream(st)
            cc.colour(g, p.k, seed=self.seed_base + s.req.seed, first_iter=s.first, B=s.count, out=C, stream=st)
            cc.count_packed(p, g, C, workspace=_Fixed(ws), out=X, stream=st)
            keep += [C, X, ws]
            outs.append(X)
        ev = torch.cuda.Event()
        ev.record(st)
        return {"event": ev, "keep": keep, "outs": outs, "stream": st}

    def poll(self, handle) -> bool:
        return handle["event"].query()

    def collect(self, handle) -> list[np.ndarray]:
        import paper_1804_09764_amd as cc
        handle["event"].synchronize()
        cc.stream_check(handle["stream"])  # a device error on the batch's stream fails the batch
        return [x.cpu().numpy() for x in handle["outs"]]

    def estimate(self, req: Request, X: np.ndarray):
        import paper_1804_09764_amd as cc
        return cc.estimate(self.plan(req), X)
