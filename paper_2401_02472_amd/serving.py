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

Admission: a launch reserves its workspace bytes (`bc_workspace_bytes`) plus
its output arrays against the budget and releases them when it completes; a
request that could never fit alone is rejected with BC_ERR_OUT_OF_MEMORY.

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

from . import BC_ERR_OUT_OF_MEMORY, BCError


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
        from . import BC_MODE_BATCHED, make_options
        G = self.graphs[graph_id]
        # bc_run_multi runs its batches as one part (or in the device loop)
        ws = G.workspace_bytes(max(k, 1), make_options(BC_MODE_BATCHED, concurrency=1))
        return int(ws) + nreq * 8 * G.n

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
        self._reserved = 0
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
    def _pick(self):
        """Graph whose oldest queued request has waited longest, and the
        requests of that graph that fit one launch and the budget."""
        best, best_t = None, None
        for gid, q in self._queues.items():
            if q and (best_t is None or q[0].arrival < best_t):
                best, best_t = gid, q[0].arrival
        if best is None:
            return None
        q = self._queues[best]
        take, lanes = [], 0
        for r in q:
            if take and lanes + r.k > self.max_lanes:
                break
            trial = take + [r]
            need = self.executor.bytes_needed(best, lanes + r.k, len(trial))
            if self._reserved + need > self.budget:
                break
            take, lanes = trial, lanes + r.k
        if not take:
            return None
        need = self.executor.bytes_needed(best, lanes, len(take))
        for _ in take:
            q.popleft()
        return best, take, need

    def _schedule(self):
        with self._lock:
            while True:
                while self._free_slots:
                    picked = self._pick()
                    if picked is None:
                        break
                    gid, reqs, need = picked
                    slot = self._free_slots.pop()
                    self._reserved += need
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
            self._reserved -= need
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
