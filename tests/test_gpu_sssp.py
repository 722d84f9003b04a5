"""GPU parity of single-source shortest paths (bc_set_weights / bc_sssp)
against the oracle's fixed-point SSSP: distances are integers, compared
exactly."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2401_02472_amd as bcm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    bcm.load_library()


def gpu_dist(G, s):
    return G.sssp(int(s)).cpu().numpy().astype(np.int64)


def flags_of(g):
    return bcm.BC_GRAPH_DIRECTED if g.params.get("directed") else 0


GRAPHS = [
    gg.rmat(12, 8, seed=1), gg.grid_road(128, 128, seed=2), gg.rmat(12, 8, seed=4, directed=True),
    gg.gnp_directed(150, 0.02, seed=5), gg.path(300), gg.star(3000),
    gg.csr_from_edges(9, [0, 1, 5, 6], [1, 2, 6, 7]),   # two components and isolated vertices
]


@pytest.mark.parametrize("g", GRAPHS, ids=lambda g: g.name)
def test_sssp_weighted(g):
    w = gg.edge_weights(g, seed=7)
    src = gg.sample_sources(g, 5, seed=8, min_degree=0)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=flags_of(g)) as G:
        G.set_weights(w)
        for s in src:
            want, _ = oracle.sssp(g.row_ptr, g.col_idx, w, int(s))
            assert np.array_equal(gpu_dist(G, s), want), f"source {s}"


def test_sssp_unit_weights_without_set_weights_and_zero_weights():
    g = gg.rmat(11, 8, seed=3)
    ones = np.ones(g.nnz, np.int32)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        for s in gg.sample_sources(g, 3, seed=4):
            want, _ = oracle.sssp(g.row_ptr, g.col_idx, ones, int(s))
            assert np.array_equal(gpu_dist(G, s), want)
        w = gg.edge_weights(g, seed=9, lo=0, hi=3)   # many zero-weight edges
        G.set_weights(w)
        for s in gg.sample_sources(g, 3, seed=5):
            want, _ = oracle.sssp(g.row_ptr, g.col_idx, w, int(s))
            assert np.array_equal(gpu_dist(G, s), want)


def test_sssp_weight_errors():
    g = gg.path(3)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        with pytest.raises(bcm.BCError) as ei:
            G.set_weights(np.array([1, -1, 1, 1], np.int32))
        assert ei.value.status == bcm.BC_ERR_INVALID_ARG
        with pytest.raises(bcm.BCError) as ei:
            G.set_weights(np.full(4, 1 << 30, np.int32))   # 2 * 2^30 does not fit int32
        assert ei.value.status == bcm.BC_ERR_RANGE
        with pytest.raises(bcm.BCError):
            G.sssp(3)


def test_sssp_rmat22_full_size():
    """Full-size scale-22 R-MAT with weights in [1, 100]: one source, exact."""
    g = gg.rmat(22, 16, seed=3)
    w = gg.edge_weights(g, seed=3)
    s = int(gg.sample_sources(g, 1, seed=103)[0])
    with bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_TRUST_SYMMETRIC) as G:
        G.set_weights(w)
        got = gpu_dist(G, s)
    want, _ = oracle.sssp(g.row_ptr, g.col_idx, w, s)
    assert np.array_equal(got, want)
