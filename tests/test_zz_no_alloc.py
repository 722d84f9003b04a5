"""GPU tests of the allocation-free entry point bc_run_async_noalloc.

Its output is compared with bc_run_async's (the batched path with the
host-driven loop, one part) on two calls in a row, the second on a smaller
graph with fewer sources, so stale contents of the shared device array from
the first call must not leak into the second; and with the oracle.  Compare
rules: tests/gpu_checks.py (BC within 1e-9 relative, exact zeros).  A single
batch is the same computation as bc_run_async's in the same lane order, so
there the two agree bit for bit.
"""
import numpy as np
import pytest

import graphgen as gg
import paper_2401_02472_amd as bcm
from tests.gpu_checks import check_bc, oracle_bc, oracle_bc_ext

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    bcm.load_library()


def _say(msg):
    print(f"# {msg}", flush=True)


def _noalloc(G, src):
    import torch
    out = torch.full((G.n,), 7.0, dtype=torch.float64, device="cuda")
    G.run_async_noalloc(np.asarray(src, np.int32), out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _run_async(G, src):
    import torch
    out = torch.empty(G.n, dtype=torch.float64, device="cuda")
    G.run_async(np.asarray(src, np.int32), out,
                bcm.make_options(bcm.BC_MODE_BATCHED, concurrency=1, level_loop=bcm.BC_LOOP_HOST))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_matches_run_async_on_two_calls():
    big = gg.rmat(12, 8, seed=1)
    small = gg.rmat(9, 8, seed=7)
    src_big = gg.sample_sources(big, 150, seed=11)
    src_small = gg.sample_sources(small, 37, seed=12)
    with bcm.Graph(big.n, big.row_ptr, big.col_idx) as GB, \
            bcm.Graph(small.n, small.row_ptr, small.col_idx) as GS:
        _say(f"noalloc call 1: rmat-12 n={big.n} k={src_big.size}")
        got_big = _noalloc(GB, src_big)
        _say(f"noalloc call 2: rmat-9 n={small.n} k={src_small.size}")
        got_small = _noalloc(GS, src_small)
        ref_big = _run_async(GB, src_big)
        ref_small = _run_async(GS, src_small)
    check_bc(got_big, ref_big)
    check_bc(got_big, oracle_bc(big, src_big))
    # one batch, same lanes: the same computation
    assert np.array_equal(got_small, ref_small)
    check_bc(got_small, oracle_bc(small, src_small))


def test_noalloc_repeats_and_empty():
    g = gg.rmat(10, 8, seed=5)
    src = gg.sample_sources(g, 100, seed=9)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        _say("noalloc repeat")
        a = _noalloc(G, src)
        b = _noalloc(G, src)
        assert np.array_equal(a, b)
        z = _noalloc(G, np.zeros(0, np.int32))
        assert np.all(z == 0)
    check_bc(a, oracle_bc(g, src))


def test_noalloc_wide_rows_and_extended_range():
    # lattice: counts pass 2^32 (the batch reruns with double rows) and 2^53
    lat = gg.grid_full(40, 40)
    src = np.array([0, 39, 820, 1599, 5], np.int32)
    # diamond chain: counts 4^i pass double's range (level-scaled counts)
    ch = gg.diamond_chain(520, 4)
    src_ch = np.array([0, ch.n - 1, 7], np.int32)
    with bcm.Graph(lat.n, lat.row_ptr, lat.col_idx) as G:
        _say("noalloc lattice 40x40")
        got = _noalloc(G, src)
    check_bc(got, oracle_bc(lat, src))
    with bcm.Graph(ch.n, ch.row_ptr, ch.col_idx) as G:
        _say(f"noalloc diamond chain n={ch.n}")
        got = _noalloc(G, src_ch)
    check_bc(got, oracle_bc_ext(ch, src_ch))


def test_noalloc_rejects_what_does_not_fit():
    import torch
    g = gg.path(70000)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        out = torch.full((g.n,), 7.0, dtype=torch.float64, device="cuda")
        with pytest.raises(bcm.BCError) as ei:
            G.run_async_noalloc(np.array([0], np.int32), out)
        assert ei.value.status == bcm.BC_ERR_TOO_LARGE
        torch.cuda.synchronize()
        assert np.all(out.cpu().numpy() == 7.0)
        with pytest.raises(bcm.BCError) as ei:
            G.run_async_noalloc(np.array([g.n], np.int32), out)
        assert ei.value.status == bcm.BC_ERR_INVALID_ARG
