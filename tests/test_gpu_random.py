"""Randomised parity sweep (fixed seeds): small graphs of several families,
random source sets and random execution settings of the batched path (batch
width, level loop, sparse threshold, concurrency, work-item thresholds),
each run compared with the oracle, and the settings that must agree bit for
bit (the same plan on the host loop and on its graph replay) compared with
each other."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2401_02472_amd as bcm
from tests.gpu_checks import check_bc, run_mode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    bcm.load_library()


def _graph(rng, i):
    kind = i % 6
    if kind == 0:
        return gg.rmat(int(rng.integers(7, 11)), int(rng.choice([4, 8, 16])), seed=int(rng.integers(1 << 30))), False
    if kind == 1:
        n = int(rng.integers(20, 400))
        return gg.gnp(n, float(rng.uniform(1.5, 8.0)) / n, int(rng.integers(1 << 30))), False
    if kind == 2:
        return gg.grid_road(int(rng.integers(5, 30)), int(rng.integers(5, 30)),
                            seed=int(rng.integers(1 << 30))), False
    if kind == 3:
        return gg.random_tree(int(rng.integers(10, 500)), int(rng.integers(1 << 30))), False
    if kind == 4:
        n = int(rng.integers(20, 300))
        return gg.gnp_directed(n, float(rng.uniform(1.0, 6.0)) / n, int(rng.integers(1 << 30))), True
    return gg.star(int(rng.integers(70, 900))), False


@pytest.mark.parametrize("case", range(96))
def test_random_graphs_and_settings(case):
    rng = np.random.default_rng(7000 + case)
    g, directed = _graph(rng, case)
    k = int(rng.integers(1, min(g.n, 200) + 1))
    src = rng.choice(g.n, size=k, replace=bool(rng.integers(2))).astype(np.int32)
    want, st = oracle.bc(g.row_ptr, g.col_idx, src, directed=directed)
    assert st == oracle.OK
    flags = bcm.BC_GRAPH_DIRECTED if directed else 0
    with bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=flags) as G:
        cut = int(rng.choice([1, 4, 8, 16, 64, 100]))
        chunk = int(rng.choice([64, 128, 512, 1024]))
        G.set_work_items(cut, max(chunk, ((cut + 63) // 64) * 64))
        width = int(rng.choice([1, 7, 32, 64, 100, 128]))
        div = int(rng.choice([-1, 1, 4, 64]))
        conc = int(rng.choice([0, 1, 3]))
        host = run_mode(G, src, bcm.BC_MODE_BATCHED, batch_width=width, sparse_div=div,
                        concurrency=conc, level_loop=bcm.BC_LOOP_HOST)
        check_bc(host, want)
        replay = run_mode(G, src, bcm.BC_MODE_BATCHED, batch_width=width, sparse_div=div,
                          concurrency=conc, level_loop=bcm.BC_LOOP_GRAPH)
        assert np.array_equal(replay, host)
        if width <= 64:
            check_bc(run_mode(G, src, bcm.BC_MODE_BATCHED, batch_width=width,
                              level_loop=bcm.BC_LOOP_DEVICE), want)
        if not directed:
            check_bc(run_mode(G, src, bcm.BC_MODE_PLAIN), want)
        check_bc(run_mode(G, src, bcm.BC_MODE_AUTO), want)
