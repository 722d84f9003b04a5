"""GPU parity on directed graphs (the CSR lists out-arcs; created with
BC_GRAPH_DIRECTED): the batched kernels pull sigma over the reversed CSR and
dependencies over the out-arcs.  Compared with the directed oracle (rules in
tests/gpu_checks.py)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2401_02472_amd as bcm
from tests.gpu_checks import check_bc, check_sigma, run_mode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    bcm.load_library()


def dgraph(g):
    return bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_DIRECTED)


def oracle_dir(g, sources):
    want, st = oracle.bc(g.row_ptr, g.col_idx, np.asarray(sources, np.int32), directed=True)
    assert st == oracle.OK
    return want


def hub_graph(n_leaves, direction):
    """A hub of in-degree (direction 'in') or out-degree ('out') n_leaves, with a
    short chain on the other side, so that the hub is split into chunks in one
    direction only."""
    hub, pairs = 0, []
    leaves = range(1, n_leaves + 1)
    chain = list(range(n_leaves + 1, n_leaves + 6))
    if direction == "in":
        pairs += [(v, hub) for v in leaves] + [(hub, chain[0])]
    else:
        pairs += [(hub, v) for v in leaves] + [(chain[0], hub)]
    pairs += [(chain[i], chain[i + 1]) for i in range(len(chain) - 1)]
    pairs += [(v, v + 1) for v in range(1, n_leaves, 7)]  # some arcs among the leaves
    return gg.directed(n_leaves + 6, pairs, f"hub-{direction}-{n_leaves}")


FAMILIES = [
    gg.directed(150, [(i, i + 1) for i in range(149)], "dpath-150"),
    gg.directed(130, [(i, (i + 1) % 130) for i in range(130)], "dcycle-130"),
    gg.directed(3000, [(0, i) for i in range(1, 3000)], "out-star-3000"),
    gg.directed(3000, [(i, 0) for i in range(1, 3000)], "in-star-3000"),
    gg.directed(4, [(0, 1), (0, 2), (1, 3), (2, 3)], "diamond-dag"),
    gg.gnp_directed(60, 0.05, seed=3), gg.gnp_directed(200, 0.02, seed=4),
    hub_graph(2000, "in"), hub_graph(2000, "out"), hub_graph(300, "in"),
    gg.rmat(10, 8, seed=5, directed=True),
]


@pytest.mark.parametrize("g", FAMILIES, ids=lambda g: g.name)
def test_directed_families_all_sources(g):
    src = np.arange(g.n, dtype=np.int32)
    with dgraph(g) as G:
        check_bc(G.run(src), oracle_dir(g, src))


@pytest.mark.parametrize("loop", [bcm.BC_LOOP_HOST, bcm.BC_LOOP_DEVICE], ids=["host", "device"])
def test_directed_rmat12_all_sources(loop):
    """Directed R-MAT scale 12 from all 4096 sources (hubs split into chunks in
    both directions), on both level loops."""
    g = gg.rmat(12, 8, seed=9, directed=True)
    src = np.arange(g.n, dtype=np.int32)
    with dgraph(g) as G:
        got = run_mode(G, src, bcm.BC_MODE_BATCHED, level_loop=loop)
    check_bc(got, oracle_dir(g, src))


@pytest.mark.parametrize("div", [-1, 1, 64])
def test_directed_sparse_threshold_settings(div):
    """Scan-all and frontier-driven forward steps (the latter marks along
    out-arcs and pulls along in-arcs): BC, dist and sigma."""
    g = gg.rmat(13, 8, seed=11, directed=True)
    src = gg.sample_sources(g, 70, seed=12)
    with dgraph(g) as G:
        opt = bcm.make_options(bcm.BC_MODE_BATCHED, sparse_div=div, level_loop=bcm.BC_LOOP_HOST)
        bc, dist, sigma = G.run_detail(src, opt)
    check_bc(bc, oracle_dir(g, src))
    for i, s in enumerate(src[:6]):
        od, osg, _, st = oracle.single_source(g.row_ptr, g.col_idx, int(s), with_delta=False,
                                              directed=True)
        assert st == oracle.OK
        assert np.array_equal(dist[i], od)
        check_sigma(sigma[i], osg)


def test_directed_symmetric_graph_equals_undirected():
    g = gg.rmat(12, 8, seed=1)
    src = gg.sample_sources(g, 100, seed=2)
    with dgraph(g) as G:
        a = G.run(src)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        b = G.run(src)
    check_bc(a, b, rtol=1e-12)


def test_directed_modes_and_requests():
    """Plain-mode calls run batched; bc_run_multi requests equal their runs alone;
    the one-source state call is not available for directed graphs."""
    import torch
    g = gg.gnp_directed(120, 0.03, seed=6)
    src = np.arange(g.n, dtype=np.int32)
    with dgraph(g) as G:
        check_bc(run_mode(G, src[:5], bcm.BC_MODE_PLAIN), oracle_dir(g, src[:5]))
        reqs = [src[:3], src[10:80], src[100:101]]
        outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for _ in reqs]
        G.run_multi(reqs, outs)
        torch.cuda.synchronize()
        for r, o in zip(reqs, outs):
            check_bc(o.cpu().numpy(), oracle_dir(g, r))
        with pytest.raises(bcm.BCError) as ei:
            G.single_source(0)
        assert ei.value.status == bcm.BC_ERR_UNSUPPORTED


def test_directed_rmat22_full_size_one_batch():
    """Directed R-MAT scale 22 (edge factor 16) in the benchmark's launch
    configuration: one 64-source batch; dist / sigma of 3 lanes bit-exact, BC of
    the batch within 1e-9."""
    g = gg.rmat(22, 16, seed=3, directed=True)
    src = gg.sample_sources(g, 64, seed=103)
    with dgraph(g) as G:
        got = run_mode(G, src, bcm.BC_MODE_BATCHED)
        _, dist, sigma = G.run_detail(src[:3], bcm.make_options(bcm.BC_MODE_BATCHED))
    for i, s in enumerate(src[:3]):
        od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, int(s), with_delta=False,
                                             directed=True)
        assert np.array_equal(dist[i], od)
        check_sigma(sigma[i], osg)
    check_bc(got, oracle_dir(g, src))


def _dclique_and_grid(k=48, side=40, seed=41):
    """A k-clique with arcs both ways, joined both ways to a side x side grid
    whose edges are one-way (random direction) or two-way: dense hit masks in
    the clique, sparse ones on the grid's deep levels, in both directions of
    the walk (forward over in-arcs, reverse over out-arcs)."""
    rng = np.random.default_rng(seed)
    pairs = [(a, b) for a in range(k) for b in range(k) if a != b]
    for r in range(side):
        for c in range(side):
            v = k + r * side + c
            for w in ([v + 1] if c + 1 < side else []) + ([v + side] if r + 1 < side else []):
                x = rng.integers(3)
                if x != 1:
                    pairs.append((v, w))
                if x != 0:
                    pairs.append((w, v))
    for i in range(6):
        t = k + i * (side * side // 6)
        pairs += [(i, t), (t, i)]
    return gg.directed(k + side * side, pairs, f"dclique{k}+grid{side}")


@pytest.mark.parametrize("loop", [bcm.BC_LOOP_HOST, bcm.BC_LOOP_DEVICE], ids=["host", "device"])
def test_directed_dense_and_sparse_groups(loop):
    """Directed batches whose groups take both walks in one run: BC, dist and
    sigma equal the directed oracle's, and the run repeats bit for bit."""
    g = _dclique_and_grid()
    rng = np.random.default_rng(42)
    src = np.concatenate([rng.choice(48, 30, replace=False),
                          48 + rng.choice(g.n - 48, 70, replace=False)]).astype(np.int32)
    rng.shuffle(src)
    with dgraph(g) as G:
        got = run_mode(G, src, bcm.BC_MODE_BATCHED, level_loop=loop)
        again = run_mode(G, src, bcm.BC_MODE_BATCHED, level_loop=loop)
        _, dist, sigma = G.run_detail(src, bcm.make_options(bcm.BC_MODE_BATCHED, level_loop=loop))
    check_bc(got, oracle_dir(g, src))
    assert np.array_equal(got, again)
    for i in (0, 17, 63, 64, 99):
        od, osg, _, st = oracle.single_source(g.row_ptr, g.col_idx, int(src[i]), with_delta=False,
                                              directed=True)
        assert st == oracle.OK
        assert np.array_equal(dist[i], od), f"dist differs for lane {i} (source {src[i]})"
        check_sigma(sigma[i], osg)
