"""Continuous-batching BC server over resident graphs.

Requests (graph id, source set) arrive at any time.  A scheduler thread keeps a
queue per graph; whenever an executor slot is free and the HBM budget admits
the launch, it packs every queued request of the graph that has waited
longest (up to `max_lanes` sources) into one launch, in which the requests'
sources share the 64-source batches of the library's batched path
(`bc_run_multi`).  Requests that arrive while launches are on the GPU join
the next launch of their graph; launches of different slots run concurrently
on their own HIP streams, so work of different graphs and requests overlaps
on the device.

Admission counts the device memory the launches really hold: the library
keeps each graph's workspaces pooled after a launch (`bc_workspace_held`), so
the budget covers every graph's pool, the workspaces of launches in flight
(`bc_workspace_bytes`, of which a graph's idle pool covers what it can) and
the output arrays.  When a launch does not fit but would once idle graphs'
pools are freed (`bc_trim_workspaces`), they are freed until it fits, those of
graphs with no queued request first, each group least recently used first;
otherwise it waits for launches in flight to finish.  A request that could
never fit alone is rejected with BC_ERR_OUT_OF_MEMORY.

Each result is the same whether the request runs alone or in a mix: a
request of at most 64 sources never straddles two batches and every lane's
arithmetic is independent of the other lanes (see `bc_run_multi`).

The executor is pluggable so that the scheduling logic can be tested without
a GPU; the default executor calls the HIP library.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

from . import BC_ERR_INVALID_ARG, BC_ERR_OUT_OF_MEMORY, BCError


@dataclass
class Request:
    graph_id: object
    sources: np.ndarray
    arrival: float
    future: Future = field(default_factory=Future)
    started: float = 0.0
    finished: float = 0.0

    @property
    def k(self) -> int:
        return int(self.sources.size)


class GpuExecutor:
    """Runs one launch (several requests of one graph) with bc_run_multi on a
    private stream per slot."""

    def __init__(self, graphs: dict, slots: int):
        import torch
        self.graphs = graphs
        self.streams = [torch.cuda.Stream() for _ in range(slots)]

    def bytes_needed(self, graph_id, k: int, nreq: int) -> int:
        """Workspace plus output bytes of one launch."""
        from . import BC_MODE_BATCHED, make_options
        G = self.graphs[graph_id]
        # bc_run_multi runs its batches as one part (or in the device loop)
        ws = G.workspace_bytes(max(k, 1), make_options(BC_MODE_BATCHED, concurrency=1))
        return int(ws) + self.output_bytes(graph_id, nreq)

    def output_bytes(self, graph_id, nreq: int) -> int:
        return nreq * 8 * self.graphs[graph_id].n

    def held_bytes(self, graph_id) -> int:
        """Device bytes the graph's workspace pools hold now."""
        return int(self.graphs[graph_id].workspace_held())

    def trim(self, graph_id) -> None:
        self.graphs[graph_id].trim_workspaces()

    def run(self, slot: int, graph_id, requests):
        import torch
        G = self.graphs[graph_id]
        s = self.streams[slot]
        with torch.cuda.stream(s):
            outs = [torch.empty(G.n, dtype=torch.float64, device="cuda") for _ in requests]
            G.run_multi([r.sources for r in requests], outs, stream=s)
            host = [o.to("cpu", non_blocking=False) for o in outs]
        s.synchronize()
        return [h.numpy() for h in host]


class BCServer:
    """Continuous-batching scheduler.

    graphs      {graph_id: Graph} resident graphs (bc_graph_t handles)
    budget      HBM bytes the in-flight launches may reserve
    slots       launches in flight at once (one HIP stream each)
    max_lanes   sources packed into one launch
    executor    object with bytes_needed(graph_id, k, nreq) and
                run(slot, graph_id, requests) -> [np.ndarray]; default: GPU
    """

    def __init__(self, graphs: dict, budget: int, slots: int = 4, max_lanes: int = 256,
                 executor=None):
        self.graphs = graphs
        self.budget = int(budget)
        self.slots = int(slots)
        self.max_lanes = int(max_lanes)
        self.executor = executor if executor is not None else GpuExecutor(graphs, slots)
        self._lock = threading.Condition()
        self._queues = collections.OrderedDict((g, collections.deque()) for g in graphs)
        self._free_slots = list(range(self.slots))
        self._reserved = 0           # workspace + output bytes of launches in flight
        self._inflight_ws = collections.Counter()   # per graph: workspace bytes in flight
        self._out_reserved = 0
        self._last_used = {g: 0.0 for g in graphs}  # completion time (pool LRU)
        self.trims = 0
        self._closing = False
        self._workers = []
        self.completed = []          # finished requests (for statistics)
        self.launches = 0
        self.max_reserved = 0
        self._sched = threading.Thread(target=self._schedule, name="bc-scheduler", daemon=True)
        self._sched.start()

    # -- client side -------------------------------------------------------
    def submit(self, graph_id, sources) -> Future:
        src = np.ascontiguousarray(np.asarray(sources), dtype=np.int32)
        req = Request(graph_id, src, time.perf_counter())
        if graph_id not in self._queues:
            req.future.set_exception(KeyError(f"unknown graph {graph_id!r}"))
            return req.future
        # a source outside the graph fails the request here: inside a launch
        # it would fail every request batched with it
        n = getattr(self.graphs[graph_id], "n", None)
        if n is not None and src.size and (int(src.min()) < 0 or int(src.max()) >= int(n)):
            req.future.set_exception(BCError(BC_ERR_INVALID_ARG, "submit"))
            return req.future
        need = self.executor.bytes_needed(graph_id, req.k, 1)
        if need > self.budget:
            req.future.set_exception(BCError(BC_ERR_OUT_OF_MEMORY, "admission"))
            return req.future
        with self._lock:
            if self._closing:
                raise RuntimeError("server is closed")
            self._queues[graph_id].append(req)
            self._lock.notify_all()
        return req.future

    def close(self, wait: bool = True):
        with self._lock:
            self._closing = True
            self._lock.notify_all()
        if wait:
            self._sched.join()
            for w in list(self._workers):
                w.join()

    # -- scheduler ---------------------------------------------------------
    def _held(self):
        fn = getattr(self.executor, "held_bytes", None)
        return {g: (int(fn(g)) if fn else 0) for g in self._queues}

    def _split(self, gid, k, nreq):
        """(workspace, output) bytes of a launch."""
        need = self.executor.bytes_needed(gid, k, nreq)
        fn = getattr(self.executor, "output_bytes", None)
        out = int(fn(gid, nreq)) if fn else 0
        return need - out, out

    def _projected(self, held, gid, ws, out):
        """Device bytes in use once a launch of `ws` workspace and `out`
        output bytes starts on gid: every graph's pool (the part launches in
        flight do not use stays held), the workspaces in flight, the outputs;
        the new launch reuses what gid's idle pool holds."""
        total = self._out_reserved + out
        for g, h in held.items():
            busy = self._inflight_ws[g]
            idle = max(0, h - busy)
            total += busy + idle
            if g == gid:
                total += max(0, ws - idle)
        return total

    def _pick(self):
        """Graph whose oldest queued request has waited longest, and the
        requests of that graph that fit one launch and the budget (after
        freeing idle graphs' pools: those with nothing queued first)."""
        best, best_t = None, None
        for gid, q in self._queues.items():
            if q and (best_t is None or q[0].arrival < best_t):
                best, best_t = gid, q[0].arrival
        if best is None:
            return None
        q = self._queues[best]
        held = self._held()
        # the first request alone must fit: free idle pools until it does
        ws0, out0 = self._split(best, q[0].k, 1)
        if self._projected(held, best, ws0, out0) > self.budget:
            trim = getattr(self.executor, "trim", None)
            # idle pools of graphs with nothing queued go first (least recently
            # used first), then those whose requests wait (their next launch
            # would build the pool again); never the pool this launch reuses
            idle = sorted((g for g in held
                           if g != best and held[g] > 0 and self._inflight_ws[g] == 0),
                          key=lambda g: (len(self._queues[g]) > 0, self._last_used[g]))
            # trim only if that lets the launch start now; otherwise it waits
            # for launches in flight, and the pools stay for their graphs
            if self._projected({g: (0 if g in idle else h) for g, h in held.items()},
                               best, ws0, out0) > self.budget:
                idle = []
            for g in idle:
                if trim is None:
                    break
                trim(g)
                self.trims += 1
                held = self._held()
                if self._projected(held, best, ws0, out0) <= self.budget:
                    break
        take, lanes = [], 0
        for r in q:
            if take and lanes + r.k > self.max_lanes:
                break
            trial = take + [r]
            ws, out = self._split(best, lanes + r.k, len(trial))
            if self._projected(held, best, ws, out) > self.budget:
                break
            take, lanes = trial, lanes + r.k
        if not take:
            return None
        ws, out = self._split(best, lanes, len(take))
        for _ in take:
            q.popleft()
        return best, take, (ws, out)

    def _schedule(self):
        with self._lock:
            while True:
                while self._free_slots:
                    picked = self._pick()
                    if picked is None:
                        break
                    gid, reqs, need = picked
                    slot = self._free_slots.pop()
                    self._reserved += need[0] + need[1]
                    self._inflight_ws[gid] += need[0]
                    self._out_reserved += need[1]
                    self.max_reserved = max(self.max_reserved, self._reserved)
                    self.launches += 1
                    w = threading.Thread(target=self._run, args=(slot, gid, reqs, need),
                                         daemon=True)
                    self._workers.append(w)
                    w.start()
                idle = all(not q for q in self._queues.values())
                if self._closing and idle and len(self._free_slots) == self.slots:
                    return
                self._lock.wait()

    def _run(self, slot, gid, reqs, need):
        t0 = time.perf_counter()
        for r in reqs:
            r.started = t0
        try:
            results = self.executor.run(slot, gid, reqs)
            err = None
        except Exception as exc:  # delivered to every request of the launch
            results, err = None, exc
        t1 = time.perf_counter()
        for i, r in enumerate(reqs):
            r.finished = t1
            if err is None:
                r.future.set_result(results[i])
            else:
                r.future.set_exception(err)
        with self._lock:
            self.completed.extend(reqs)
            self._reserved -= need[0] + need[1]
            self._inflight_ws[gid] -= need[0]
            self._out_reserved -= need[1]
            self._last_used[gid] = t1
            self._free_slots.append(slot)
            self._workers = [w for w in self._workers if w is not threading.current_thread()]
            self._lock.notify_all()

    # -- statistics --------------------------------------------------------
    def latency_stats(self):
        lat = np.array([r.finished - r.arrival for r in self.completed if r.finished > 0])
        if lat.size == 0:
            return {}
        return {"requests": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3)}
