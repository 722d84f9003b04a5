"""GPU parity of PageRank (bc_pagerank) against the oracle's pull iteration.
Ranks after a fixed number of iterations (tol 0) agree to 1e-11 relative: the
GPU adds a big vertex's shares in a tree instead of in arc order, and every
later iteration carries that rounding (damped by the factor d)."""
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


def graph(g):
    flags = bcm.BC_GRAPH_DIRECTED if g.params.get("directed") else 0
    return bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=flags)


GRAPHS = [
    gg.rmat(12, 8, seed=1), gg.rmat(12, 8, seed=9, directed=True), gg.grid_road(96, 96, seed=2),
    gg.cycle(50), gg.star(3000), gg.directed(3000, [(i, 0) for i in range(1, 3000)], "in-star"),
    gg.gnp_directed(200, 0.02, seed=5), gg.csr_from_edges(7, [0, 1, 4], [1, 2, 5]),
]


@pytest.mark.parametrize("g", GRAPHS, ids=lambda g: g.name)
def test_pagerank_fixed_iterations(g):
    for d in (0.85, 0.5):
        want, it_o, _ = oracle.pagerank(g.row_ptr, g.col_idx, d, 0.0, 30)
        with graph(g) as G:
            got, it = G.pagerank(d, 0.0, 30)
        got = got.cpu().numpy()
        assert it == it_o
        np.testing.assert_allclose(got, want, rtol=1e-11, atol=0)


def test_pagerank_converges_like_oracle():
    g = gg.rmat(13, 16, seed=3)
    want, it_o, _ = oracle.pagerank(g.row_ptr, g.col_idx, 0.85, 1e-9, 500)
    with graph(g) as G:
        got, it = G.pagerank(0.85, 1e-9, 500)
        again, it2 = G.pagerank(0.85, 1e-9, 500)
    assert abs(it - it_o) <= 1 and it == it2
    assert np.array_equal(got.cpu().numpy(), again.cpu().numpy())  # repeats bit for bit
    np.testing.assert_allclose(got.cpu().numpy(), want, rtol=1e-7)


def test_pagerank_rmat22_full_size():
    """Full-size scale-22 R-MAT, 20 iterations."""
    g = gg.rmat(22, 16, seed=3)
    want, _, _ = oracle.pagerank(g.row_ptr, g.col_idx, 0.85, 0.0, 20)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_TRUST_SYMMETRIC) as G:
        got, it = G.pagerank(0.85, 0.0, 20)
    assert it == 20
    np.testing.assert_allclose(got.cpu().numpy(), want, rtol=1e-11, atol=0)


def test_pagerank_argument_errors():
    g = gg.path(4)
    with graph(g) as G:
        for d, tol, mi in ((1.5, 0.0, 10), (0.85, -1.0, 10), (0.85, 0.0, 0)):
            with pytest.raises(bcm.BCError) as ei:
                G.pagerank(d, tol, mi)
            assert ei.value.status == bcm.BC_ERR_INVALID_ARG
