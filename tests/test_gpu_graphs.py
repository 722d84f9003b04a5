"""GPU parity of bc_run_graphs (several graphs' 64-source batches in one
device-resident launch) against each graph's own device-loop run, bit for
bit, and against the oracle."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2401_02472_amd as bcm
from tests.gpu_checks import check_bc, oracle_bc, oracle_bc_ext, run_mode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    bcm.load_library()


def _own(G, src, loop=bcm.BC_LOOP_DEVICE):
    """The same graph alone: batched, 64-source batches, the given loop."""
    return run_mode(G, src, bcm.BC_MODE_BATCHED, batch_width=64, level_loop=loop)


def _run_graphs(Gs, srcs, loop=bcm.BC_LOOP_DEVICE, with_loops=False):
    import torch
    outs = [torch.full((G.n,), -1.0, dtype=torch.float64, device="cuda") for G in Gs]
    loops = bcm.bc_run_graphs(Gs, srcs, outs, level_loop=loop)
    torch.cuda.synchronize()
    res = [o.cpu().numpy() for o in outs]
    return (res, loops) if with_loops else res


def _want(g, src, directed=False, ext=False):
    if directed:
        want, st = oracle.bc(g.row_ptr, g.col_idx, np.asarray(src, np.int32), directed=True)
        assert st == oracle.OK
        return want
    return oracle_bc_ext(g, src) if ext else oracle_bc(g, src)


def _small_mix():
    graphs = [gg.rmat(9, 8, seed=1), gg.rmat(10, 16, seed=2), gg.grid_full(20, 30), gg.star(500),
              gg.cycle(100), gg.path(50), gg.complete(20), gg.random_tree(300, 4),
              gg.gnp(200, 0.05, 3)]
    ks = [1, 64, 70, 130, 5, 50, 20, 300, 200]
    srcs = [gg.sample_sources(g, min(k, g.n), seed=10 + i) for i, (g, k) in enumerate(zip(graphs, ks))]
    return graphs, srcs


def test_small_graphs_in_one_launch_equal_their_own_runs():
    graphs, srcs = _small_mix()
    Gs = [bcm.Graph(g.n, g.row_ptr, g.col_idx) for g in graphs]
    try:
        got = _run_graphs(Gs, srcs)
        again = _run_graphs(Gs, srcs)
        # another order of the same graphs
        rev = _run_graphs(Gs[::-1], srcs[::-1])[::-1]
        for i, (g, src) in enumerate(zip(graphs, srcs)):
            assert np.array_equal(got[i], _own(Gs[i], src)), g.name
            assert np.array_equal(again[i], got[i]) and np.array_equal(rev[i], got[i]), g.name
            check_bc(got[i], _want(g, src))
    finally:
        for G in Gs:
            G.close()


@pytest.mark.parametrize("loop", [bcm.BC_LOOP_AUTO, bcm.BC_LOOP_HOST])
def test_auto_and_host_choices_equal_the_reported_loops(loop):
    """BC_LOOP_AUTO lets the small graphs join and runs the large one on the
    host loop (BC_LOOP_HOST: all of them); each result equals the graph's own
    run with the loop reported for it."""
    graphs, srcs = _small_mix()
    big = gg.rmat(16, 16, seed=12)
    graphs.append(big)
    srcs.append(gg.sample_sources(big, 64, seed=13))
    Gs = [bcm.Graph(g.n, g.row_ptr, g.col_idx) for g in graphs]
    try:
        got, loops = _run_graphs(Gs, srcs, loop, with_loops=True)
        if loop == bcm.BC_LOOP_HOST:
            assert all(x == bcm.BC_LOOP_HOST for x in loops)
        else:
            assert loops[-1] == bcm.BC_LOOP_HOST       # 2M arcs: too slow on one CU
            assert loops.count(bcm.BC_LOOP_DEVICE) >= 5  # the small ones share the launch
        for i, (g, src) in enumerate(zip(graphs, srcs)):
            assert np.array_equal(got[i], _own(Gs[i], src, loops[i])), g.name
        check_bc(got[-1], _want(big, srcs[-1]))
    finally:
        for G in Gs:
            G.close()


def test_graphs_that_rerun_or_run_alone_join_the_call():
    """A lattice whose path counts pass 2^32 (its batches rerun with double
    rows, on their own), counts beyond double's range (extended range: the
    host loop), a directed graph, an empty graph and a graph with no sources,
    next to ordinary ones."""
    lat = gg.grid_full(40, 40)
    ch = gg.diamond_chain(520, 4)
    dg = gg.gnp_directed(300, 0.02, 5)
    r = gg.rmat(10, 8, seed=6)
    empty = gg.csr_from_edges(0, [], [])
    cases = [(lat, np.array([0, 39, 820, 1599, 5], np.int32), False, False),
             (ch, np.array([0, ch.n - 1, 7], np.int32), False, True),
             (dg, gg.sample_sources(dg, 90, seed=7), True, False),
             (r, gg.sample_sources(r, 100, seed=8), False, False),
             (empty, np.zeros(0, np.int32), False, False),
             (r, np.zeros(0, np.int32), False, False)]
    Gs = []
    for g, _, directed, _ in cases:
        flags = bcm.BC_GRAPH_DIRECTED if directed else 0
        Gs.append(bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=flags))
    srcs = [c[1] for c in cases]
    try:
        got = _run_graphs(Gs, srcs)
        for i, (g, src, directed, ext) in enumerate(cases):
            if g.n == 0:
                continue
            if src.size == 0:
                assert np.all(got[i] == 0)
                continue
            assert np.array_equal(got[i], _own(Gs[i], src)), g.name
            check_bc(got[i], _want(g, src, directed, ext))
    finally:
        for G in Gs:
            G.close()


def test_invalid_calls_are_rejected():
    g = gg.rmat(8, 8, seed=9)
    import torch
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        out = torch.empty(g.n, dtype=torch.float64, device="cuda")
        with pytest.raises(bcm.BCError) as ei:      # a graph given twice
            bcm.bc_run_graphs([G, G], [np.array([0], np.int32)] * 2, [out, out])
        assert ei.value.status == bcm.BC_ERR_INVALID_ARG
        with pytest.raises(bcm.BCError) as ei:      # a source out of range
            bcm.bc_run_graphs([G], [np.array([g.n], np.int32)], [out])
        assert ei.value.status == bcm.BC_ERR_INVALID_ARG
        with pytest.raises(bcm.BCError) as ei:      # not a loop this call takes
            bcm.bc_run_graphs([G], [np.array([0], np.int32)], [out], level_loop=bcm.BC_LOOP_GRAPH)
        assert ei.value.status == bcm.BC_ERR_INVALID_ARG
        bcm.bc_run_graphs([], [], [])                # nothing to do


def test_binding_refuses_short_buffers():
    # outputs shorter than the graph and inputs shorter than the CSR the
    # library would read are refused before any launch; the buffers are left
    # as they were
    import torch
    g = gg.rmat(8, 8, seed=9)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        short = torch.full((g.n - 1,), -1.0, dtype=torch.float64, device="cuda")
        for call in (lambda: bcm.bc_run_async(G.handle, [0], short),
                     lambda: bcm.bc_run_async_noalloc(G.handle, [0], short),
                     lambda: bcm.bc_run_multi(G.handle, [[0]], [short]),
                     lambda: bcm.bc_run_graphs([G], [[0]], [short]),
                     lambda: bcm.bc_pagerank(G.handle, short)):
            with pytest.raises(ValueError, match="entries"):
                call()
        with pytest.raises(ValueError, match="entries"):
            bcm.bc_sssp(G.handle, 0, torch.zeros(g.n - 1, dtype=torch.int32, device="cuda"))
        with pytest.raises(ValueError, match="weights"):
            G.set_weights(np.ones(g.col_idx.size - 1, np.int32))
        torch.cuda.synchronize()
        assert bool((short == -1.0).all())
        # a full-length output still runs
        out = torch.empty(g.n, dtype=torch.float64, device="cuda")
        bcm.bc_run_async(G.handle, [0, 1], out)
        torch.cuda.synchronize()
        check_bc(out.cpu().numpy(), oracle_bc(g, np.array([0, 1], np.int32)))
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    with pytest.raises(ValueError, match="col_idx"):
        bcm.bc_create_graph(g.n, rp, ci[:-1], flags=bcm.BC_GRAPH_INPUT_ON_DEVICE)
    with pytest.raises(ValueError, match="row_ptr"):
        bcm.bc_create_graph(g.n, rp[:-1], ci, flags=bcm.BC_GRAPH_INPUT_ON_DEVICE)
