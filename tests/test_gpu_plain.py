"""GPU parity of the one-source-at-a-time path against the CPU oracle
(compare rules in tests/gpu_checks.py)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2401_02472_amd as bcm
from tests.gpu_checks import check_bc, check_sigma, oracle_bc, oracle_bc_ext, plain

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    bcm.load_library()


FAMILIES = [
    gg.path(2), gg.path(37), gg.star(5), gg.star(3000), gg.cycle(9), gg.cycle(64),
    gg.complete(12), gg.complete_bipartite(3, 40), gg.hypercube(7), gg.grid_full(17, 23),
    gg.torus(8, 12), gg.random_tree(300, 4), gg.gnp(60, 0.08, 2),
]


@pytest.mark.parametrize("g", FAMILIES, ids=lambda g: g.name)
def test_families_all_sources(g):
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        src = np.arange(g.n, dtype=np.int32)
        check_bc(plain(G, src), oracle_bc(g, src))


def test_rmat12_all_sources():
    """The scale-12 R-MAT workload: exact BC from all 4096 sources."""
    g, src = gg.workload("rmat-s12-ef8")
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        got = plain(G, src)
    check_bc(got, oracle_bc(g, src))


@pytest.mark.parametrize("g", [gg.rmat(12, 8, seed=1), gg.rmat(16, 16, seed=5),
                               gg.grid_road(64, 64, seed=3), gg.star(9000)],
                         ids=lambda g: g.name)
def test_single_source_state_bit_exact(g):
    deg = g.degrees()
    picks = list(gg.sample_sources(g, 6, seed=21))
    picks.append(int(np.argmax(deg)))            # hub: several 2048-arc chunks
    iso = np.nonzero(deg == 0)[0]
    if iso.size:
        picks.append(int(iso[0]))                 # isolated source
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        for s in picks:
            dist, sigma, delta = G.single_source(s)
            od, osg, odl, st = oracle.single_source(g.row_ptr, g.col_idx, s)
            assert st == oracle.OK
            assert np.array_equal(dist, od), f"dist differs from source {s}"
            check_sigma(sigma, osg)
            check_bc(delta, odl)


def test_road_grid_deep_sigma_beyond_2_53():
    """Road-like grid: ~120 levels, sigma beyond 2**53 on part of the vertices."""
    g = gg.grid_road(256, 256, seed=7)
    src = gg.sample_sources(g, 6, seed=8)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        for s in src[:3]:
            dist, sigma, _ = G.single_source(int(s))
            od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, int(s))
            assert np.array_equal(dist, od)
            check_sigma(sigma, osg)
        check_bc(plain(G, src), oracle_bc(g, src))


def test_additivity_duplicates_and_empty():
    g = gg.rmat(11, 8, seed=9)
    src = gg.sample_sources(g, 24, seed=10)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        assert np.all(plain(G, np.zeros(0, np.int32)) == 0)
        dup = np.concatenate([src[:5], src[:5]])
        check_bc(plain(G, dup), oracle_bc(g, dup))
        a = plain(G, src[:10])
        b = plain(G, src[10:])
        np.testing.assert_allclose(plain(G, src), a + b, rtol=1e-12, atol=0)


def test_tiny_graphs():
    for g in [gg.csr_from_edges(1, [], []), gg.csr_from_edges(7, [], []), gg.path(2)]:
        with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
            src = np.arange(g.n, dtype=np.int32)
            check_bc(plain(G, src), oracle_bc(g, src))


def test_multigraph_and_self_loops():
    rng = np.random.default_rng(5)
    u = rng.integers(0, 40, 200)
    v = rng.integers(0, 40, 200)
    g = gg.csr_from_edges(40, u, v, dedup=False, drop_loops=False)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        src = np.arange(g.n, dtype=np.int32)
        check_bc(plain(G, src), oracle_bc(g, src))


def test_run_to_run_bit_identical():
    g = gg.rmat(14, 16, seed=2)
    src = gg.sample_sources(g, 8, seed=3)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        a = plain(G, src)
        b = plain(G, src)
    assert np.array_equal(a, b)


def test_run_async_on_torch_stream():
    import torch
    g = gg.rmat(13, 8, seed=4)
    src = gg.sample_sources(g, 16, seed=5)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        out = torch.empty(g.n, dtype=torch.float64, device="cuda")
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            G.run_async(src, out, bcm.make_options(bcm.BC_MODE_PLAIN, level_chunk=2))
        s.synchronize()
        check_bc(out.cpu().numpy(), oracle_bc(g, src))


def test_graph_from_device_tensors():
    import torch
    g = gg.rmat(10, 8, seed=6)
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    with bcm.Graph(g.n, rp, ci, flags=bcm.BC_GRAPH_INPUT_ON_DEVICE) as G:
        src = np.arange(0, g.n, 7, dtype=np.int32)
        check_bc(plain(G, src), oracle_bc(g, src))


def test_sigma_overflow_switches_to_extended_range():
    """A plain-mode call whose counts pass double's range is completed by the
    batched path's level-scaled counts (and the graph stays there); the
    per-source state of bc_single_source, in double, still reports the range."""
    g = gg.grid_full(600, 600)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_TRUST_SYMMETRIC) as G:
        check_bc(plain(G, np.array([0], np.int32)), oracle_bc_ext(g, [0]))
        check_bc(plain(G, np.array([7, 9], np.int32)), oracle_bc_ext(g, [7, 9]))
        with pytest.raises(bcm.BCError) as ei:
            G.single_source(0)
        assert ei.value.status == bcm.BC_ERR_RANGE


def test_out_of_range_source_rejected():
    g = gg.path(5)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        with pytest.raises(bcm.BCError) as ei:
            G.run(np.array([5], np.int32))
        assert ei.value.status == bcm.BC_ERR_INVALID_ARG


def test_rmat22_sampled_full_size():
    """Full-size scale-22 R-MAT, in the benchmark's launch configuration:
    dist / sigma of two sources bit-exact, BC of four sources within 1e-9."""
    g = gg.rmat(22, 16, seed=3)
    src = gg.sample_sources(g, 256, seed=103)[:4]
    with bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_TRUST_SYMMETRIC) as G:
        for s in src[:2]:
            dist, sigma, _ = G.single_source(int(s))
            od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, int(s), with_delta=False)
            assert np.array_equal(dist, od)
            check_sigma(sigma, osg)
        got = plain(G, src)
    check_bc(got, oracle_bc(g, src))


def test_road_grid_without_shortcuts_range():
    """Road-like grid with no shortcuts (about 1,700 levels): shortest-path counts
    overflow double on part of the vertices.  The run reports BC_ERR_RANGE, and the
    distances it still returns match the oracle's everywhere; sigma matches where
    it stays far from overflow."""
    g = gg.grid_road(1024, 1024, 0.05, 0.0, seed=2)
    src = gg.sample_sources(g, 2, seed=102)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_TRUST_SYMMETRIC) as G:
        for s in src:
            od, osg, _, ost = oracle.single_source(g.row_ptr, g.col_idx, int(s),
                                                   with_delta=False)
            assert ost == oracle.RANGE
            assert od.max() > 1000
            with pytest.raises(bcm.BCError) as ei:
                G.single_source(int(s))
            assert ei.value.status == bcm.BC_ERR_RANGE
            dist, sigma, _ = ei.value.result
            assert np.array_equal(dist, od)
            far = osg < 1e300
            check_sigma(sigma[far], osg[far])
