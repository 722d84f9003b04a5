"""Scheduler logic of the serving loop, on the CPU with a fake executor that
answers from the oracle (no GPU)."""
import threading
import time

import numpy as np
import pytest

import graphgen as gg
import oracle
from paper_2401_02472_amd import BCError
from paper_2401_02472_amd.serving import BCServer


class FakeExecutor:
    def __init__(self, graphs, delay=0.01, per_source=1000, per_request=100):
        self.graphs = graphs
        self.delay = delay
        self.per_source = per_source
        self.per_request = per_request
        self.lock = threading.Lock()
        self.inflight = 0
        self.max_inflight = 0
        self.launch_sizes = []

    def bytes_needed(self, gid, k, nreq):
        return self.per_source * k + self.per_request * nreq

    def run(self, slot, gid, reqs):
        with self.lock:
            self.inflight += 1
            self.max_inflight = max(self.max_inflight, self.inflight)
            self.launch_sizes.append(len(reqs))
        time.sleep(self.delay)
        g = self.graphs[gid]
        out = [oracle.bc(g.row_ptr, g.col_idx, r.sources)[0] for r in reqs]
        with self.lock:
            self.inflight -= 1
        return out


@pytest.fixture(scope="module")
def graphs():
    return {"a": gg.rmat(8, 8, seed=1), "b": gg.rmat(9, 8, seed=2), "c": gg.path(30)}


def test_results_match_oracle_and_requests_share_launches(graphs):
    ex = FakeExecutor(graphs, delay=0.05)
    srv = BCServer(graphs, budget=10**9, slots=2, max_lanes=256, executor=ex)
    rng = np.random.default_rng(0)
    reqs = []
    for i in range(40):
        gid = ["a", "b", "c"][i % 3]
        g = graphs[gid]
        k = int(rng.choice([1, 8, 64]))
        src = rng.choice(g.n, size=min(k, g.n), replace=False).astype(np.int32)
        reqs.append((gid, src, srv.submit(gid, src)))
    for gid, src, fut in reqs:
        g = graphs[gid]
        want, _ = oracle.bc(g.row_ptr, g.col_idx, src)
        np.testing.assert_array_equal(fut.result(timeout=30), want)
    srv.close()
    assert ex.max_inflight <= 2
    assert max(ex.launch_sizes) > 1          # queued requests were packed together
    assert srv.latency_stats()["requests"] == 40


def test_budget_limits_concurrency(graphs):
    # each launch of one 8-source request needs 8100 bytes; the budget admits one at a time
    ex = FakeExecutor(graphs, delay=0.02)
    srv = BCServer(graphs, budget=9000, slots=4, max_lanes=8, executor=ex)
    futs = [srv.submit("a", np.arange(8, dtype=np.int32) + i) for i in range(6)]
    for f in futs:
        f.result(timeout=30)
    srv.close()
    assert ex.max_inflight == 1
    assert srv.max_reserved <= 9000


def test_request_that_can_never_fit_is_rejected(graphs):
    ex = FakeExecutor(graphs)
    srv = BCServer(graphs, budget=500, slots=2, executor=ex)
    fut = srv.submit("a", np.arange(4, dtype=np.int32))
    with pytest.raises(BCError):
        fut.result(timeout=5)
    with pytest.raises(KeyError):
        srv.submit("zzz", [0]).result(timeout=5)
    srv.close()


def test_executor_failure_reaches_every_request_of_the_launch(graphs):
    class Boom(FakeExecutor):
        def run(self, slot, gid, reqs):
            raise RuntimeError("device lost")

    srv = BCServer(graphs, budget=10**9, slots=1, executor=Boom(graphs))
    futs = [srv.submit("a", [i]) for i in range(3)]
    for f in futs:
        with pytest.raises(RuntimeError):
            f.result(timeout=5)
    srv.close()


def test_close_drains_the_queue(graphs):
    ex = FakeExecutor(graphs, delay=0.01)
    srv = BCServer(graphs, budget=10**9, slots=1, max_lanes=1, executor=ex)
    futs = [srv.submit("c", [i]) for i in range(10)]
    srv.close()
    assert all(f.done() for f in futs)


def test_trims_idle_pools_of_graphs_without_queued_requests_first(graphs):
    """A launch that does not fit frees idle pools: first those of graphs with
    nothing queued, then (least recently used first) those whose requests wait;
    never the pool of the graph being launched."""
    class PoolExecutor(FakeExecutor):
        def __init__(self, graphs, held):
            super().__init__(graphs)
            self.held = dict(held)
            self.trimmed = []

        def held_bytes(self, gid):
            return self.held[gid]

        def trim(self, gid):
            self.trimmed.append(gid)
            self.held[gid] = 0

    # a launch of 8 sources on "a" needs 8100 bytes; the pools of "b" and "c"
    # hold 5000 each, so one of them must go for it to fit 13500
    ex = PoolExecutor(graphs, {"a": 0, "b": 5000, "c": 5000})
    srv = BCServer(graphs, budget=13500, slots=0, executor=ex)  # no slot: nothing runs
    try:
        srv.submit("a", np.arange(8, dtype=np.int32))
        srv.submit("b", np.arange(4, dtype=np.int32))
        with srv._lock:
            srv._last_used.update({"a": 3.0, "b": 1.0, "c": 2.0})  # "b" least recent
            picked = srv._pick()
        assert picked is not None and picked[0] == "a"
        assert ex.trimmed == ["c"]      # "b" has a queued request: kept
        # next the oldest request is "b"'s (4100 bytes); "b"'s own idle pool is
        # not trimmed for its launch (it covers part of the workspace): "a"'s
        # goes, although "a" has a request waiting
        ex.held.update({"a": 5000, "b": 3000, "c": 0})
        ex.trimmed.clear()
        srv.submit("a", np.arange(8, dtype=np.int32) + 8)
        with srv._lock:
            srv.budget = 8000
            picked = srv._pick()
        assert picked is not None and picked[0] == "b"
        assert ex.trimmed == ["a"]
    finally:
        srv.close(wait=False)


def test_no_trim_when_the_launch_would_still_wait(graphs):
    """Pools are not freed for a launch that would not fit even with every idle
    pool gone (launches in flight hold the memory): it waits instead."""
    class PoolExecutor(FakeExecutor):
        def __init__(self, graphs, held):
            super().__init__(graphs)
            self.held = dict(held)
            self.trimmed = []

        def held_bytes(self, gid):
            return self.held[gid]

        def trim(self, gid):
            self.trimmed.append(gid)
            self.held[gid] = 0

    ex = PoolExecutor(graphs, {"a": 0, "b": 2000, "c": 2000})
    srv = BCServer(graphs, budget=13500, slots=0, executor=ex)
    try:
        srv.submit("a", np.arange(8, dtype=np.int32))   # 8100 bytes
        with srv._lock:
            srv._inflight_ws["c"] = 0
            srv._out_reserved = 9000    # memory held by launches in flight
            picked = srv._pick()
        assert picked is None and ex.trimmed == []
    finally:
        srv.close(wait=False)


def test_source_outside_the_graph_fails_only_its_request(graphs):
    from paper_2401_02472_amd import BC_ERR_INVALID_ARG
    ex = FakeExecutor(graphs, delay=0.05)
    srv = BCServer(graphs, budget=10**9, slots=1, max_lanes=256, executor=ex)
    g = graphs["a"]
    good = [np.array([i, i + 1], np.int32) for i in range(4)]
    futs = [srv.submit("a", s) for s in good[:2]]
    bad = [srv.submit("a", [0, g.n]), srv.submit("a", [-1])]
    futs += [srv.submit("a", s) for s in good[2:]]
    for f in bad:
        with pytest.raises(BCError) as ei:
            f.result(timeout=5)
        assert ei.value.status == BC_ERR_INVALID_ARG
    for s, f in zip(good, futs):
        np.testing.assert_array_equal(f.result(timeout=10), oracle.bc(g.row_ptr, g.col_idx, s)[0])
    srv.close()
    assert sum(ex.launch_sizes) == len(good)
