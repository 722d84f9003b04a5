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
