"""GPU parity of the benchmark workloads, run exactly as bench.py runs them.

Each workload is built by graphgen.workload (the bench's graph and sources) and
run the way bench.py times it: the autotuner first, then BC_MODE_AUTO with the
library's default concurrency (the scale-22 and Erdos-Renyi graphs run as two
concurrent parts of landmark-sorted batches, summed in part order).  BC is
compared with the threaded CPU oracle over all the workload's sources; the
per-source state of every lane (bc_run_detail, same batching) with the oracle's
single-source pass, one source per worker thread (the oracle releases the GIL);
and the BC total with the distance-sum invariant
    sum_v BC(v) = sum over sources s of sum over reached t != s of (d(s, t) - 1),
computed from the exported distances alone.  Compare rules: tests/gpu_checks.py.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2401_02472_amd as bcm
from tests.gpu_checks import check_bc, check_sigma, run_mode

pytestmark = pytest.mark.gpu

WORKERS = 16


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    bcm.load_library()


def _oracle_bc(g, src, directed=False):
    want, st = oracle.bc(g.row_ptr, g.col_idx, np.asarray(src, np.int32),
                         threads=min(WORKERS, oracle.max_threads()), directed=directed)
    assert st == oracle.OK
    return want


def _check_lanes(g, src, dist, sigma, lanes, directed=False):
    """dist equal and sigma as check_sigma for the given rows, oracle passes in
    parallel."""
    rp = np.ascontiguousarray(g.row_ptr, np.int32)
    ci = np.ascontiguousarray(g.col_idx, np.int32)

    def one(i):
        od, osg, _, st = oracle.single_source(rp, ci, int(src[i]), with_delta=False,
                                              directed=directed)
        assert st == oracle.OK
        assert np.array_equal(dist[i], od), f"dist differs for source {src[i]} (row {i})"
        check_sigma(sigma[i], osg)
        return i

    with ThreadPoolExecutor(WORKERS) as ex:
        done = []
        for i in ex.map(one, lanes):
            done.append(i)
            if len(done) % 32 == 0:
                _say(f"{len(done)} lanes checked")
    assert done == list(lanes)


def _distance_sum(dist):
    """sum over rows of sum over reached t (d >= 1) of d - 1."""
    total = 0
    for row in dist:
        r = row[row >= 1].astype(np.int64)
        total += int((r - 1).sum())
    return total


def _say(msg):
    print(f"# {msg}", flush=True)


def _benchmarked(name, flags, directed=False):
    g, src = gg.workload(name)
    _say(f"{name}: n={g.n} nnz={g.nnz} k={len(src)}")
    with bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=flags) as G:
        tuning = G.autotune(src)
        got = run_mode(G, src, bcm.BC_MODE_AUTO)
        again = run_mode(G, src, bcm.BC_MODE_AUTO)
        bc2, dist, sigma = G.run_detail(src, bcm.make_options(bcm.BC_MODE_AUTO))
    _say(f"{name}: GPU runs done, tuning {tuning}")
    assert tuning["batch_width"] in (32, 64, 128)
    # same batches, parts and sums whether or not the state is exported
    assert np.array_equal(got, again)
    assert np.array_equal(got, bc2)
    check_bc(got, _oracle_bc(g, src, directed))
    _say(f"{name}: BC matches the oracle")
    if not directed:
        tot = float(np.sum(got))
        want = float(_distance_sum(dist))
        assert abs(tot - want) <= 1e-9 * want
    _check_lanes(g, src, dist, sigma, range(len(src)), directed)
    _say(f"{name}: dist / sigma of all {len(src)} lanes match")
    return g, src


@pytest.mark.timeout(900)
def test_rmat22_as_benchmarked():
    """Scale-22 R-MAT, 256 sources: autotune, AUTO, two concurrent parts of
    landmark-sorted batches (the bench's headline configuration)."""
    _benchmarked("rmat-s22-ef16", bcm.BC_GRAPH_TRUST_SYMMETRIC)


@pytest.mark.timeout(900)
def test_erdos_renyi_2_23_as_benchmarked():
    """Erdos-Renyi n = 2^23, average degree 16, 128 sources, as the bench runs it."""
    _benchmarked("er-n8388608-d16", bcm.BC_GRAPH_TRUST_SYMMETRIC)


@pytest.mark.timeout(900)
def test_directed_rmat22_as_benchmarked():
    """Directed scale-22 R-MAT (each sampled edge one arc), 256 sources."""
    _benchmarked("rmat-s22-ef16-dir", bcm.BC_GRAPH_DIRECTED, directed=True)


@pytest.mark.parametrize("loop", [bcm.BC_LOOP_HOST, bcm.BC_LOOP_DEVICE], ids=["host", "device"])
def test_erdos_renyi_small_all_sources(loop):
    """A small Erdos-Renyi graph (n = 4096, average degree 16) from every vertex:
    64 batches on either level loop, and the one-source path."""
    g = gg.erdos_renyi(4096, 16, seed=5)
    src = np.arange(g.n, dtype=np.int32)
    want = _oracle_bc(g, src)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        check_bc(run_mode(G, src, bcm.BC_MODE_BATCHED, level_loop=loop), want)
        if loop == bcm.BC_LOOP_HOST:
            check_bc(run_mode(G, src[:300], bcm.BC_MODE_PLAIN), _oracle_bc(g, src[:300]))


@pytest.mark.timeout(900)
def test_road_grid_full_size_as_benchmarked():
    """The 1024 x 1024 road-like grid with shortcuts, 64 sources: the plain path,
    the batched path and AUTO after the autotuner; path counts pass 2^53 on part
    of the vertices (compared at 1e-12 there)."""
    g, src = gg.workload("grid-1024x1024")
    want = _oracle_bc(g, src)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_TRUST_SYMMETRIC) as G:
        check_bc(run_mode(G, src, bcm.BC_MODE_PLAIN), want)
        check_bc(run_mode(G, src, bcm.BC_MODE_BATCHED), want)
        G.autotune(src)
        got = run_mode(G, src, bcm.BC_MODE_AUTO)
        _, dist, sigma = G.run_detail(src, bcm.make_options(bcm.BC_MODE_AUTO))
    check_bc(got, want)
    assert sigma.max() > 2.0 ** 53
    _check_lanes(g, src, dist, sigma, range(len(src)))
