"""GPU parity of the batched path (up to 64 sources per level step) against
the CPU oracle and against the one-source-at-a-time path (compare rules in
tests/gpu_checks.py)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2401_02472_amd as bcm
from tests.gpu_checks import (batched, check_bc, check_sigma, check_sigma_ext, oracle_bc,
                              oracle_bc_ext, plain, run_mode)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    bcm.load_library()


FAMILIES = [
    gg.path(2), gg.path(150), gg.star(5), gg.star(3000), gg.cycle(9), gg.cycle(130),
    gg.complete(12), gg.complete_bipartite(3, 40), gg.hypercube(7), gg.grid_full(17, 23),
    gg.torus(8, 12), gg.random_tree(300, 4), gg.gnp(60, 0.08, 2),
    gg.csr_from_edges(1, [], []), gg.csr_from_edges(7, [], []),
]


@pytest.mark.parametrize("g", FAMILIES, ids=lambda g: g.name)
def test_families_all_sources(g):
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        src = np.arange(g.n, dtype=np.int32)
        check_bc(batched(G, src), oracle_bc(g, src))


def test_rmat12_all_sources():
    """The scale-12 R-MAT workload from all 4096 sources: 64 full batches."""
    g, src = gg.workload("rmat-s12-ef8")
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        check_bc(batched(G, src), oracle_bc(g, src))


@pytest.mark.parametrize("width", [1, 7, 32, 64])
def test_batch_widths_and_ragged_last_batch(width):
    g = gg.rmat(13, 8, seed=11)
    src = gg.sample_sources(g, 100, seed=12)          # 100 = ragged for every width
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        check_bc(batched(G, src, batch_width=width), oracle_bc(g, src))


@pytest.mark.parametrize("g", [gg.rmat(12, 8, seed=1), gg.rmat(15, 16, seed=5),
                               gg.grid_road(64, 64, seed=3), gg.star(9000)],
                         ids=lambda g: g.name)
def test_per_source_state_bit_exact(g):
    """dist and sigma of every lane of a batch, from bc_run_detail."""
    deg = g.degrees()
    src = list(gg.sample_sources(g, 40, seed=21))
    src.append(int(np.argmax(deg)))
    iso = np.nonzero(deg == 0)[0]
    if iso.size:
        src.append(int(iso[0]))
    src = np.asarray(src, np.int32)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        bc, dist, sigma = G.run_detail(src, bcm.make_options(bcm.BC_MODE_BATCHED))
    check_bc(bc, oracle_bc(g, src))
    for i, s in enumerate(src):
        od, osg, _, st = oracle.single_source(g.row_ptr, g.col_idx, int(s), with_delta=False)
        assert st == oracle.OK
        assert np.array_equal(dist[i], od), f"dist differs for lane {i} (source {s})"
        check_sigma(sigma[i], osg)


def test_duplicates_in_one_batch_and_additivity():
    g = gg.rmat(11, 8, seed=9)
    src = gg.sample_sources(g, 24, seed=10)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        dup = np.concatenate([src[:5], src[:5], src[:1]])
        check_bc(batched(G, dup), oracle_bc(g, dup))
        a = batched(G, src[:10])
        b = batched(G, src[10:])
        np.testing.assert_allclose(batched(G, src), a + b, rtol=1e-12, atol=0)


def test_batched_equals_plain_and_is_deterministic():
    g = gg.rmat(14, 16, seed=2)
    src = gg.sample_sources(g, 96, seed=3)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        p = plain(G, src)
        b1 = batched(G, src)
        b2 = batched(G, src)
    assert np.array_equal(b1, b2)
    check_bc(b1, p)


def test_deep_graph_grows_level_array():
    """A 2000-vertex path from all ends runs deeper than the initial level array."""
    g = gg.path(2000)
    src = np.array([0, 1999, 1000, 3, 1500], np.int32)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        check_bc(batched(G, src), oracle_bc(g, src))
        check_bc(batched(G, src), oracle_bc(g, src))


def test_road_grid_deep_sigma_beyond_2_53():
    g = gg.grid_road(256, 256, seed=7)
    src = gg.sample_sources(g, 70, seed=8)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        bc, dist, sigma = G.run_detail(src[:8], bcm.make_options(bcm.BC_MODE_BATCHED))
        for i, s in enumerate(src[:8]):
            od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, int(s), with_delta=False)
            assert np.array_equal(dist[i], od)
            check_sigma(sigma[i], osg)
        check_bc(batched(G, src), oracle_bc(g, src))


def test_multigraph_and_self_loops():
    rng = np.random.default_rng(5)
    u = rng.integers(0, 40, 200)
    v = rng.integers(0, 40, 200)
    g = gg.csr_from_edges(40, u, v, dedup=False, drop_loops=False)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        src = np.arange(g.n, dtype=np.int32)
        check_bc(batched(G, src), oracle_bc(g, src))


def test_sigma_overflow_extended_range():
    """Counts past double's range (600x600 lattice: up to C(1198, 599) ~ 2**1194
    from a corner): the batched path switches to level-scaled counts.  BC within
    1e-9 of the extended oracle, distances equal, exported sigma as in
    check_sigma_ext; the graph stays in extended range for the next call."""
    g = gg.grid_full(600, 600)
    src = np.array([0, 5, 1234, g.n - 1], np.int32)
    want = oracle_bc_ext(g, src)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_TRUST_SYMMETRIC) as G:
        bc, dist, sigma = G.run_detail(src, bcm.make_options(bcm.BC_MODE_BATCHED))
        again = batched(G, src[:2])
    check_bc(bc, want)
    check_bc(again, oracle_bc_ext(g, src[:2]))
    for i, s in enumerate(src):
        od, sm, se, _, st = oracle.single_source_ext(g.row_ptr, g.col_idx, int(s),
                                                     with_delta=False)
        assert st == oracle.OK
        assert np.array_equal(dist[i], od)
        check_sigma_ext(sigma[i], sm, se)


@pytest.mark.parametrize("k,width", [(1100, 2), (700, 3)])
def test_diamond_chain_extended_closed_form(k, width):
    """Chain of k diamonds from hub 0 (counts width**i past 2**1024): hub i's BC
    is (width+1)(k-i), a middle vertex of diamond i has (1 + (width+1)(k-i)) /
    width, the source 0."""
    g = gg.diamond_chain(k, width)
    step = width + 1
    want = np.zeros(g.n)
    for i in range(1, k + 1):
        want[i * step] = (width + 1) * (k - i)
        want[i * step - step + 1:i * step] = (1 + (width + 1) * (k - i)) / width
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        check_bc(batched(G, np.array([0], np.int32)), want)


def test_extended_range_device_loop_falls_back():
    """All 3301 sources of a diamond chain: 52 batches, which take the
    device-resident loop by default; its counts overflow double, and the call
    runs again on the host loop with level-scaled counts.  bc_run_multi on the
    same kind of graph clears its outputs and does the same."""
    g = gg.diamond_chain(1100, 2)
    src = np.arange(g.n, dtype=np.int32)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        check_bc(G.run(src), oracle_bc_ext(g, src))
    reqs = [src[:10], src[100:164], src[3000:3001], src[5:6]]
    import torch
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        outs = [torch.full((g.n,), 7.0, dtype=torch.float64, device="cuda") for _ in reqs]
        G.run_multi(reqs, outs)
        torch.cuda.synchronize()
        for r, o in zip(reqs, outs):
            check_bc(o.cpu().numpy(), oracle_bc_ext(g, r))


def test_auto_mode_matches():
    g = gg.rmat(12, 8, seed=4)
    src = gg.sample_sources(g, 40, seed=6)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        check_bc(G.run(src), oracle_bc(g, src))
        check_bc(G.run(src[:3]), oracle_bc(g, src[:3]))


def test_rmat22_full_size_one_batch():
    """Full-size scale-22 R-MAT in the benchmark's launch configuration: one
    64-source batch; dist / sigma of 3 lanes bit-exact, BC of the batch 1e-9."""
    g = gg.rmat(22, 16, seed=3)
    src = gg.sample_sources(g, 256, seed=103)[:64]
    with bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_TRUST_SYMMETRIC) as G:
        got = batched(G, src)
        _, dist, sigma = G.run_detail(src[:3], bcm.make_options(bcm.BC_MODE_BATCHED))
    for i, s in enumerate(src[:3]):
        od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, int(s), with_delta=False)
        assert np.array_equal(dist[i], od)
        check_sigma(sigma[i], osg)
    check_bc(got, oracle_bc(g, src))


def test_detail_rows_follow_caller_order_across_batches():
    """With more sources than one batch, batches are formed in landmark order;
    the per-source rows must still come back in the caller's order."""
    g = gg.rmat(12, 8, seed=13)
    src = gg.sample_sources(g, 40, seed=14)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        bc, dist, sigma = G.run_detail(src, bcm.make_options(bcm.BC_MODE_BATCHED,
                                                             batch_width=16))
    check_bc(bc, oracle_bc(g, src))
    for i, s in enumerate(src):
        od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, int(s), with_delta=False)
        assert np.array_equal(dist[i], od), f"row {i} (source {s})"
        check_sigma(sigma[i], osg)


def test_road_grid_without_shortcuts_extended():
    """Road-like grid with no shortcuts (about 1,700 levels, the level array grows
    several times; counts overflow double): BC within 1e-9 of the extended
    oracle, distances equal, exported sigma as in check_sigma_ext."""
    g = gg.grid_road(1024, 1024, 0.05, 0.0, seed=2)
    src = gg.sample_sources(g, 3, seed=102)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_TRUST_SYMMETRIC) as G:
        bc, dist, sigma = G.run_detail(src, bcm.make_options(bcm.BC_MODE_BATCHED))
    check_bc(bc, oracle_bc_ext(g, src))
    for i, s in enumerate(src):
        od, sm, se, _, ost = oracle.single_source_ext(g.row_ptr, g.col_idx, int(s),
                                                      with_delta=False)
        assert ost == oracle.OK
        assert od.max() > 1000
        assert np.array_equal(dist[i], od)
        check_sigma_ext(sigma[i], sm, se)


@pytest.mark.parametrize("div", [-1, 1, 16, 64])
@pytest.mark.parametrize("g", [gg.rmat(14, 16, seed=11), gg.grid_road(96, 96, seed=12)],
                         ids=lambda g: g.name)
def test_sparse_threshold_settings(g, div):
    """Every setting of the switch between the scan-all step and the
    frontier-driven step (never, always, and two thresholds) gives the oracle's
    BC, and the same distances / sigma bit for bit."""
    src = gg.sample_sources(g, 70, seed=13)
    opt = bcm.make_options(bcm.BC_MODE_BATCHED, sparse_div=div, level_loop=bcm.BC_LOOP_HOST)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        check_bc(batched(G, src, sparse_div=div, level_loop=bcm.BC_LOOP_HOST),
                 oracle_bc(g, src))
        _, dist, sigma = G.run_detail(src[:3], opt)
    for i, s in enumerate(src[:3]):
        od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, int(s), with_delta=False)
        assert np.array_equal(dist[i], od)
        check_sigma(sigma[i], osg)


def test_autotune_then_auto_mode():
    """bc_autotune stores a valid choice; BC_MODE_AUTO runs with it match the
    oracle, on both sides of the chosen crossover."""
    g = gg.rmat(14, 16, seed=14)
    src = gg.sample_sources(g, 100, seed=15)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        t = G.autotune(src)
        assert t["batch_width"] in (32, 64, 128)
        assert t["sparse_div"] in (-1, 16, 64, 256)
        assert t["min_batched"] >= 2
        assert t["sample"] == 100 and not t["cached"]
        assert t["group_cut"] in (4, 8, 16, 32, 64, 128)
        assert t["chunk"] in (64, 128, 256, 512, 1024) and t["chunk"] >= t["group_cut"]
        assert t["plain_ms_per_source"] > 0 and t["batch_ms"] > 0
        for k in (3, 100):
            want = oracle_bc(g, src[:k])
            check_bc(G.run(src[:k]), want)
            check_bc(run_mode(G, src[:k], bcm.BC_MODE_AUTO), want)
    # a graph of the same shape takes the remembered choice without timing
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G2:
        t2 = G2.autotune(src)
        assert t2["cached"] and t2["sample"] == 0
        for f in ("batch_width", "sparse_div", "min_batched"):
            assert t2[f] == t[f]
        check_bc(run_mode(G2, src, bcm.BC_MODE_AUTO), oracle_bc(g, src))


def _shape_line(g, width, div, min_batched, cut=64, chunk=512):
    """A tuning-cache line for g's shape: n, arcs, direction, and the vertex
    counts per degree class (class c: degree of bit length c) in 64ths of n."""
    deg = np.diff(g.row_ptr).astype(np.int64)
    directed = bool(g.params.get("directed"))
    if directed:  # the larger of the out- and in-degree
        deg = np.maximum(deg, np.bincount(g.col_idx, minlength=g.n).astype(np.int64))
    cls = np.zeros(33, np.int64)
    for d in deg:
        cls[min(int(d).bit_length(), 32)] += 1
    q = [int(np.floor(64.0 * c / g.n + 0.5)) for c in cls]
    return (f"bc-tune 1 {g.n} {g.nnz} {int(directed)} " + " ".join(map(str, q)) +
            f" {width} {div} {min_batched} {cut} {chunk} 1.5 2.5\n")


def test_autotune_cache_file(tmp_path, monkeypatch):
    """With BC_MI355X_TUNE_CACHE set, choices are appended to the file, and a
    shape found there is taken from it (last line for the shape wins)."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("BC_MI355X_TUNE_CACHE", str(path))
    g = gg.rmat(12, 16, seed=42)
    src = gg.sample_sources(g, 40, seed=43)
    path.write_text(_shape_line(g, 64, 64, 9) + _shape_line(g, 32, 256, 7, cut=32, chunk=1024))
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        t = G.autotune(src)
        assert t["cached"] and (t["batch_width"], t["sparse_div"], t["min_batched"]) == (32, 256, 7)
        assert (t["group_cut"], t["chunk"]) == (32, 1024)
        check_bc(run_mode(G, src, bcm.BC_MODE_AUTO), oracle_bc(g, src))
    h = gg.rmat(11, 16, seed=44)
    src_h = gg.sample_sources(h, 20, seed=45)
    with bcm.Graph(h.n, h.row_ptr, h.col_idx) as G:
        t = G.autotune(src_h)
        assert not t["cached"]
    lines = path.read_text().splitlines()
    assert len(lines) == 3 and lines[2].startswith(f"bc-tune 1 {h.n} {h.nnz} 0 ")
    fields = lines[2].split()
    assert int(fields[-7]) == t["batch_width"] and int(fields[-6]) == t["sparse_div"]
    assert int(fields[-4]) == t["group_cut"] and int(fields[-3]) == t["chunk"]


def _diamond_chain(k, fan=0):
    """k diamonds in series (0 -> {1, 2} -> 3 -> {4, 5} -> 6 ...): sigma doubles at
    each diamond end, 2**k at the last.  With fan > 0 the last vertex fans out to
    `fan` vertices that all meet in one hub, whose sigma is fan * 2**k."""
    u, v = [], []
    for i in range(k):
        a = 3 * i
        for b in (a + 1, a + 2):
            u += [a, b]
            v += [b, a + 3]
    end = 3 * k
    n = end + 1
    if fan:
        hub = n + fan
        for j in range(fan):
            u += [end, n + j]
            v += [n + j, hub]
        n = hub + 1
    return gg.csr_from_edges(n, np.array(u), np.array(v))


@pytest.mark.parametrize("k,fan", [(31, 0), (32, 0), (33, 0), (22, 1023), (22, 1024)],
                         ids=["2^31", "2^32", "2^33", "hub-below-2^32", "hub-at-2^32"])
def test_path_counts_around_the_uint32_rows(k, fan):
    """Path counts kept as exact uint32 rows while they fit: a count of 2**32 or
    more (also when a split hub's chunks add up to it) reruns the batch with
    double rows; sigma stays bit-exact and BC matches the oracle either way, and
    later runs on the same graph agree."""
    g = _diamond_chain(k, fan)
    src = np.array([0, 1, 3 * k, 5], np.int32)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        opt = bcm.make_options(bcm.BC_MODE_BATCHED)
        got, dist, sigma = G.run_detail(src, opt)
        again, _, _ = G.run_detail(src, opt)
    check_bc(got, oracle_bc(g, src))
    assert np.array_equal(got, again)
    for i, s in enumerate(src):
        od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, int(s), with_delta=False)
        assert np.array_equal(dist[i], od)
        assert np.array_equal(sigma[i], osg)
    if fan:
        assert sigma[0].max() == fan * 2.0 ** k
    else:
        assert sigma[0].max() == 2.0 ** k


@pytest.mark.parametrize("conc", [1, 2, 3, 8])
def test_batches_run_at_once(conc):
    """Batches split over `conc` concurrent parts (own workspace and stream each):
    BC matches the oracle, repeats bit for bit, and the per-source rows of every
    part land in the caller's order."""
    g = gg.rmat(13, 8, seed=16)
    src = gg.sample_sources(g, 300, seed=17)
    kw = dict(concurrency=conc, level_loop=bcm.BC_LOOP_HOST)
    opt = bcm.make_options(bcm.BC_MODE_BATCHED, **kw)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        a = batched(G, src, **kw)
        b = batched(G, src, **kw)
        _, dist, sigma = G.run_detail(src[:130], opt)
    check_bc(a, oracle_bc(g, src))
    assert np.array_equal(a, b)
    for i in (0, 64, 129):
        od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, int(src[i]), with_delta=False)
        assert np.array_equal(dist[i], od)
        assert np.array_equal(sigma[i], osg)


LOOP_GRAPHS = [gg.rmat(12, 8, seed=1), gg.grid_road(64, 64, seed=18), gg.path(300),
               gg.star(3000), gg.complete(40), gg.hypercube(9)]


@pytest.mark.parametrize("g", LOOP_GRAPHS, ids=lambda g: g.name)
@pytest.mark.parametrize("loop", [bcm.BC_LOOP_HOST, bcm.BC_LOOP_DEVICE], ids=["host", "device"])
def test_level_loop_modes(g, loop):
    """The host-driven level loop and the device-resident one (a workgroup per
    batch, all batches in one launch) both give the oracle's BC and the same
    distances / sigma; deep graphs outgrow the device loop's level array and
    run again with a longer one."""
    src = gg.sample_sources(g, min(g.n, 150), seed=19)
    opt = bcm.make_options(bcm.BC_MODE_BATCHED, level_loop=loop)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        got = batched(G, src, level_loop=loop)
        again = batched(G, src, level_loop=loop)
        _, dist, sigma = G.run_detail(src[:66], opt)
    check_bc(got, oracle_bc(g, src))
    assert np.array_equal(got, again)
    for i in (0, min(65, len(src) - 1)):
        od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, int(src[i]), with_delta=False)
        assert np.array_equal(dist[i], od)
        check_sigma(sigma[i], osg)


@pytest.mark.parametrize("g", [gg.grid_full(17, 23), gg.rmat(12, 8, seed=1), gg.complete(40)],
                         ids=lambda g: g.name)
def test_device_loop_repeats_bit_for_bit(g):
    """The device-resident loop, run eight times on all sources: every run gives
    the oracle's BC and the same bits (its waves hand data to one another only
    across workgroup barriers; a race would show as run-to-run differences)."""
    src = np.arange(g.n, dtype=np.int32)
    want = oracle_bc(g, src)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        runs = [batched(G, src, level_loop=bcm.BC_LOOP_DEVICE) for _ in range(8)]
    check_bc(runs[0], want)
    for r in runs[1:]:
        assert np.array_equal(r, runs[0])


def _clique_and_grid(k=48, side=48):
    """A k-clique (vertices 0..k-1) joined by six edges to a side x side grid:
    the clique's arcs carry most sources of a batch at once, the grid's deep
    levels one or two each."""
    src, dst = [], []
    for a in range(k):
        for b in range(a + 1, k):
            src.append(a)
            dst.append(b)
    for r in range(side):
        for c in range(side):
            v = k + r * side + c
            if c + 1 < side:
                src.append(v)
                dst.append(v + 1)
            if r + 1 < side:
                src.append(v)
                dst.append(v + side)
    for i in range(6):
        src.append(i)
        dst.append(k + i * (side * side // 6))
    return gg.csr_from_edges(k + side * side, src, dst, name=f"clique{k}+grid{side}")


@pytest.mark.parametrize("loop,div", [(bcm.BC_LOOP_HOST, -1), (bcm.BC_LOOP_HOST, 64),
                                      (bcm.BC_LOOP_DEVICE, 64)],
                         ids=["host-scan", "host-sparse", "device"])
def test_dense_and_sparse_groups_in_one_run(loop, div):
    """Batches whose level steps mix 64-vertex groups with dense hit masks (the
    clique: parent and child rows read arc by arc) and sparse ones (the grid's
    deep levels: the transposed, source-by-source walk): BC, dist and sigma
    equal the oracle's whichever walk a group takes, and repeat bit for bit."""
    g = _clique_and_grid()
    rng = np.random.default_rng(40)
    src = np.concatenate([rng.choice(48, 30, replace=False),
                          48 + rng.choice(g.n - 48, 70, replace=False)]).astype(np.int32)
    rng.shuffle(src)
    opt = bcm.make_options(bcm.BC_MODE_BATCHED, level_loop=loop, sparse_div=div)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        got = batched(G, src, level_loop=loop, sparse_div=div)
        again = batched(G, src, level_loop=loop, sparse_div=div)
        _, dist, sigma = G.run_detail(src, opt)
    check_bc(got, oracle_bc(g, src))
    assert np.array_equal(got, again)
    for i in (0, 17, 63, 64, 99):
        od, osg, _, st = oracle.single_source(g.row_ptr, g.col_idx, int(src[i]), with_delta=False)
        assert st == oracle.OK
        assert np.array_equal(dist[i], od), f"dist differs for lane {i} (source {src[i]})"
        check_sigma(sigma[i], osg)


def _hub_past_2_53(m=1100):
    """Source 0 reaches vertex A through 60 diamonds in series (sigma 2^60, level
    120) and vertices u_b, b < 11, through a path then b + 8 diamonds (sigma
    2^(b+8), level 120).  Parent p_j (j = 1..m) is joined to A and to u_b for
    every bit b of j, so sigma(p_j) = 2^60 + 256 j: distinct, exact in double
    and beyond 2^53.  Hub H is joined to every p_j: degree m > 1024, so it is
    split into chunks of 512 arcs (A too), and sigma(H), a sum of m values near
    2^60, rounds.  Returns (graph, A, H, [u_b])."""
    src, dst = [], []
    nxt = [1]

    def new():
        v = nxt[0]
        nxt[0] += 1
        return v

    def diamonds(start, count):
        v = start
        for _ in range(count):
            a, b, e = new(), new(), new()
            src.extend([v, v, a, b])
            dst.extend([a, b, e, e])
            v = e
        return v

    A = diamonds(0, 60)
    us = []
    for b in range(11):
        v = 0
        for _ in range(120 - 2 * (b + 8)):
            w = new()
            src.append(v)
            dst.append(w)
            v = w
        us.append(diamonds(v, b + 8))
    parents = [new() for _ in range(m)]
    H = new()
    for j, p in enumerate(parents, start=1):
        src.extend([p, p])
        dst.extend([A, H])
        for b in range(11):
            if (j >> b) & 1:
                src.append(p)
                dst.append(us[b])
    g = gg.csr_from_edges(nxt[0], np.array(src), np.array(dst), name=f"hub-past-2^53-{m}")
    return g, A, H, us


@pytest.mark.parametrize("loop", [bcm.BC_LOOP_HOST, bcm.BC_LOOP_DEVICE], ids=["host", "device"])
def test_split_hub_sums_past_2_53_repeat_bit_for_bit(loop):
    """Split vertices add their chunks' parent counts in chunk order, so a hub
    whose parents carry distinct counts beyond 2^53 (sums that round) gets the
    same bits on every run and whatever else shares its batch; sigma within
    1e-12 and BC within 1e-9 of the oracle."""
    import torch
    g, A, H, us = _hub_past_2_53()
    srcs = np.array([0, A, H, us[3], 5, 77], np.int32)
    od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, 0, with_delta=False)
    assert od[H] == 122 and osg[H] > 2.0 ** 63
    want = oracle_bc(g, srcs)
    opt = bcm.make_options(bcm.BC_MODE_BATCHED, level_loop=loop)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        runs = [batched(G, srcs, level_loop=loop) for _ in range(6)]
        _, dist, sigma = G.run_detail(srcs, opt)
        other = gg.sample_sources(g, 40, seed=3)
        outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for _ in range(3)]
        G.run_multi([other[:20], srcs, other[20:]], outs)
        alone = torch.empty(g.n, dtype=torch.float64, device="cuda")
        G.run_multi([srcs], [alone])
        torch.cuda.synchronize()
    check_bc(runs[0], want)
    for r in runs[1:]:
        assert np.array_equal(r, runs[0])
    assert np.array_equal(outs[1].cpu().numpy(), alone.cpu().numpy())
    check_bc(alone.cpu().numpy(), want)
    for i, s in enumerate(srcs):
        od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, int(s), with_delta=False)
        assert np.array_equal(dist[i], od)
        check_sigma(sigma[i], osg)


# ---- batches of up to 128 sources (two lane words per vertex) ----------------

WIDE_GRAPHS = [gg.rmat(13, 16, seed=51), gg.grid_road(80, 80, seed=52), gg.star(5000),
               gg.complete(150), gg.erdos_renyi(6000, 12, seed=53)]


@pytest.mark.parametrize("g", WIDE_GRAPHS, ids=lambda g: g.name)
@pytest.mark.parametrize("k", [128, 100, 200, 257], ids=lambda k: f"k{k}")
def test_width_128_batches(g, k):
    """Batches of up to 128 sources (a full one, a short one, 128 + 72 and
    128 + 128 + 1): BC against the oracle, and dist / sigma of lanes in both
    halves of the first batch (sources 0, 63, 64, last)."""
    src = gg.sample_sources(g, min(k, g.n), seed=54 + k)
    check_bc(batched(G_of(g), src, batch_width=128, level_loop=bcm.BC_LOOP_HOST),
             oracle_bc(g, src))
    lanes = sorted({0, 63, min(64, src.size - 1), min(127, src.size - 1), src.size - 1})
    opt = bcm.make_options(bcm.BC_MODE_BATCHED, batch_width=128, level_loop=bcm.BC_LOOP_HOST)
    _, dist, sigma = G_of(g).run_detail(src, opt)
    for i in lanes:
        od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, int(src[i]), with_delta=False)
        assert np.array_equal(dist[i], od), f"dist of lane {i}"
        check_sigma(sigma[i], osg)


_GRAPHS = {}


def G_of(g):
    """One resident graph per test graph (module lifetime)."""
    if id(g) not in _GRAPHS:
        _GRAPHS[id(g)] = bcm.Graph(g.n, g.row_ptr, g.col_idx)
    return _GRAPHS[id(g)]


@pytest.mark.parametrize("div", [-1, 16, 4096], ids=lambda d: f"div{d}")
def test_width_128_sparse_steps_and_parts(div):
    """Width 128 with the scan-all step only, the frontier-driven step often,
    and nearly always; two concurrent parts; results repeat bit for bit."""
    g = gg.rmat(14, 16, seed=55)
    src = gg.sample_sources(g, 256, seed=56)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        a = batched(G, src, batch_width=128, sparse_div=div, concurrency=2,
                    level_loop=bcm.BC_LOOP_HOST)
        b = batched(G, src, batch_width=128, sparse_div=div, concurrency=2,
                    level_loop=bcm.BC_LOOP_HOST)
    assert np.array_equal(a, b)
    check_bc(a, oracle_bc(g, src))


def test_width_128_wide_rows_and_extended_range():
    """Counts past 2^32 (the batch reruns with double rows) and past double's
    range (level-scaled counts) with 128-source batches."""
    lat = gg.grid_full(60, 60)
    src = gg.sample_sources(lat, 120, seed=57)
    with bcm.Graph(lat.n, lat.row_ptr, lat.col_idx) as G:
        check_bc(batched(G, src, batch_width=128, level_loop=bcm.BC_LOOP_HOST),
                 oracle_bc(lat, src))
    ch = gg.diamond_chain(520, 4)
    src_ch = gg.sample_sources(ch, 100, seed=58)
    with bcm.Graph(ch.n, ch.row_ptr, ch.col_idx) as G:
        check_bc(batched(G, src_ch, batch_width=128, level_loop=bcm.BC_LOOP_HOST),
                 oracle_bc_ext(ch, src_ch))


def test_width_128_directed_and_device_loop_request():
    """A directed graph at width 128, and a device-loop request at width 128
    (run on the host loop: the device loop keeps one lane word)."""
    g = gg.rmat(12, 16, seed=59, directed=True)
    src = gg.sample_sources(g, 150, seed=60)
    want, st = oracle.bc(g.row_ptr, g.col_idx, src, directed=True)
    assert st == oracle.OK
    with bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=bcm.BC_GRAPH_DIRECTED) as G:
        check_bc(batched(G, src, batch_width=128, level_loop=bcm.BC_LOOP_HOST), want)
    u = gg.rmat(12, 8, seed=61)
    src_u = gg.sample_sources(u, 130, seed=62)
    with bcm.Graph(u.n, u.row_ptr, u.col_idx) as G:
        check_bc(batched(G, src_u, batch_width=128, level_loop=bcm.BC_LOOP_DEVICE),
                 oracle_bc(u, src_u))


@pytest.mark.parametrize("cut,chunk", [(32, 256), (128, 1024), (64, 64), (16, 2048)],
                         ids=lambda v: str(v))
def test_work_item_thresholds(cut, chunk, tmp_path, monkeypatch):
    """Other degree thresholds for the batched work items (taken from a tuning
    cache line): a lower or higher cut between group and chunk items, chunks
    of 64 to 2048 arcs (hubs split into many chunks, or into few).  BC against
    the oracle on the host loop at widths 64 and 128, on the device loop, and
    on a directed graph."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("BC_MI355X_TUNE_CACHE", str(path))
    seed = 80 + cut + chunk
    g = gg.rmat(13, 16, seed=seed)
    dg = gg.rmat(12, 16, seed=seed, directed=True)
    path.write_text(_shape_line(g, 64, 16, 2, cut=cut, chunk=chunk) +
                    _shape_line(dg, 64, 16, 2, cut=cut, chunk=chunk))
    src = gg.sample_sources(g, 150, seed=seed + 1)
    want = oracle_bc(g, src)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        t = G.autotune(src)
        assert t["cached"] and (t["group_cut"], t["chunk"]) == (cut, chunk)
        for width in (64, 128):
            check_bc(batched(G, src, batch_width=width, level_loop=bcm.BC_LOOP_HOST), want)
        check_bc(batched(G, src, level_loop=bcm.BC_LOOP_DEVICE), want)
        _, dist, sigma = G.run_detail(src[:2], bcm.make_options(bcm.BC_MODE_BATCHED))
    for i in range(2):
        od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, int(src[i]), with_delta=False)
        assert np.array_equal(dist[i], od)
        check_sigma(sigma[i], osg)
    dsrc = gg.sample_sources(dg, 70, seed=seed + 2)
    dwant, st = oracle.bc(dg.row_ptr, dg.col_idx, dsrc, directed=True)
    assert st == oracle.OK
    with bcm.Graph(dg.n, dg.row_ptr, dg.col_idx, flags=bcm.BC_GRAPH_DIRECTED) as G:
        t = G.autotune(dsrc)
        assert t["cached"] and (t["group_cut"], t["chunk"]) == (cut, chunk)
        check_bc(batched(G, dsrc, level_loop=bcm.BC_LOOP_HOST), dwant)


def test_set_work_items_explicit():
    """bc_set_work_items: other thresholds give the oracle's BC; invalid ones
    are rejected and leave the previous ones in place."""
    g = gg.rmat(13, 16, seed=91)
    src = gg.sample_sources(g, 80, seed=92)
    want = oracle_bc(g, src)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        for cut, chunk in [(128, 256), (40, 1024), (64, 512)]:
            G.set_work_items(cut, chunk)
            check_bc(batched(G, src, level_loop=bcm.BC_LOOP_HOST), want)
        G.set_work_items(100, 128)
        for bad in [(0, 512), (64, 100), (64, 8192), (600, 512)]:
            with pytest.raises(bcm.BCError) as ei:
                G.set_work_items(*bad)
            assert ei.value.status == bcm.BC_ERR_INVALID_ARG
        check_bc(batched(G, src, level_loop=bcm.BC_LOOP_HOST), want)
        check_bc(batched(G, src, level_loop=bcm.BC_LOOP_DEVICE), want)


@pytest.mark.parametrize("g", [gg.rmat(13, 16, seed=93), gg.erdos_renyi(6000, 16, seed=94),
                               gg.star(700)], ids=lambda g: g.name)
def test_small_graph_default_items_both_loops(g):
    """A small graph's host loop runs on the finer default work items (cut 8,
    chunks of 128 arcs: hubs split into many chunks), the device-resident loop
    on the creation-time ones (64 / 512): both give the oracle's BC, each
    repeats bit for bit, and so do the 64 / 512 items on the host loop."""
    src = gg.sample_sources(g, 100, seed=95)
    want = oracle_bc(g, src)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        host = batched(G, src, level_loop=bcm.BC_LOOP_HOST)
        check_bc(host, want)
        assert np.array_equal(host, batched(G, src, level_loop=bcm.BC_LOOP_HOST))
        dev = batched(G, src, level_loop=bcm.BC_LOOP_DEVICE)
        check_bc(dev, want)
        assert np.array_equal(dev, batched(G, src, level_loop=bcm.BC_LOOP_DEVICE))
        G.set_work_items(64, 512)
        coarse = batched(G, src, level_loop=bcm.BC_LOOP_HOST)
        check_bc(coarse, want)
        # the device loop does not depend on the host loop's items
        assert np.array_equal(dev, batched(G, src, level_loop=bcm.BC_LOOP_DEVICE))


def _graph_cases():
    return [
        # several batches (ragged last one) in two concurrent parts
        ("rmat13", gg.rmat(13, 16, seed=96), 150, 2, False),
        # ~100 levels: chunks of two levels on the first run (no depth hint
        # yet), one chunk once the hint is known
        ("road64", gg.grid_road(64, 64, seed=97), 64, 1, False),
        # path counts pass 2^32 on the way: the batch reruns with double rows
        ("lattice40", gg.grid_full(40, 40), 40, 1, False),
        # counts beyond double's range: level-scaled (extended-range) counts
        ("diamonds", gg.diamond_chain(520, 4), 3, 1, True),
        ("directed", gg.gnp_directed(900, 0.01, 98), 80, 1, False),
    ]


@pytest.mark.parametrize("name,g,k,conc,ext", [pytest.param(*c, id=c[0]) for c in _graph_cases()])
def test_graph_loop_replays_match_host_loop(name, g, k, conc, ext):
    """BC_LOOP_GRAPH replays captured chunks of level steps (HIP graphs whose
    kernels take the chunk's base level from the device): each replay, with
    eager host-loop runs and other sources in between, gives exactly the host
    loop's BC, which matches the oracle."""
    src = gg.sample_sources(g, min(k, g.n), seed=99)
    if name == "diamonds":
        src = np.array([0, g.n - 1, 7], np.int32)
    other = gg.sample_sources(g, min(k, g.n) // 2 + 1, seed=100)
    directed = name == "directed"
    if directed:
        want, st = oracle.bc(g.row_ptr, g.col_idx, np.asarray(src, np.int32), directed=True)
        assert st == oracle.OK
    else:
        want = oracle_bc_ext(g, src) if ext else oracle_bc(g, src)
    flags = bcm.BC_GRAPH_DIRECTED if directed else 0
    with bcm.Graph(g.n, g.row_ptr, g.col_idx, flags=flags) as G:
        host = batched(G, src, level_loop=bcm.BC_LOOP_HOST, concurrency=conc)
        check_bc(host, want)
        host_other = batched(G, other, level_loop=bcm.BC_LOOP_HOST, concurrency=conc)
        for rep in range(3):
            got = batched(G, src, level_loop=bcm.BC_LOOP_GRAPH, concurrency=conc)
            assert np.array_equal(got, host), f"replay {rep}"
            # eager work and another source set (another lane count) between replays
            assert np.array_equal(batched(G, src, level_loop=bcm.BC_LOOP_HOST, concurrency=conc),
                                  host)
            got_o = batched(G, other, level_loop=bcm.BC_LOOP_GRAPH, concurrency=conc)
            assert np.array_equal(got_o, host_other), f"replay {rep}, other sources"


def test_graph_loop_exports_per_source_state():
    """bc_run_detail on the graph-replayed loop: dist and sigma of every source
    and BC equal the host loop's, bit for bit, and match the oracle."""
    g = gg.rmat(12, 16, seed=101)
    src = gg.sample_sources(g, 70, seed=102)       # two batches, the second ragged
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        host = G.run_detail(src, bcm.make_options(bcm.BC_MODE_BATCHED,
                                                  level_loop=bcm.BC_LOOP_HOST))
        for _ in range(2):
            rep = G.run_detail(src, bcm.make_options(bcm.BC_MODE_BATCHED,
                                                     level_loop=bcm.BC_LOOP_GRAPH))
            for a, b in zip(host, rep):
                assert np.array_equal(a, b)
    bc_h, dist_h, sigma_h = host[0], host[1], host[2]
    check_bc(bc_h, oracle_bc(g, src))
    for i in (0, 69):
        od, osg, _, _ = oracle.single_source(g.row_ptr, g.col_idx, int(src[i]), with_delta=False)
        assert np.array_equal(dist_h[i], od)
        check_sigma(sigma_h[i], osg)


def _disjoint_union(a, b):
    ra = np.repeat(np.arange(a.n), np.diff(a.row_ptr))
    rb = np.repeat(np.arange(b.n), np.diff(b.row_ptr)) + a.n
    src = np.concatenate([ra, rb])
    dst = np.concatenate([a.col_idx, b.col_idx + a.n])
    keep = src < dst
    return gg.csr_from_edges(a.n + b.n, src[keep], dst[keep])


@pytest.mark.parametrize("conc", [1, 2])
def test_uint32_sized_workspaces_widen_when_counts_pass_32_bits(conc):
    """Workspaces start with uint32-sized sigma rows; when a batch's counts
    pass 32 bits the graph switches to double rows and every workspace that
    runs a later batch (of this call, of another part, or pooled for the next
    call) is widened first.  Sources on an R-MAT component (counts fit) and on
    a 40 x 40 lattice (they do not), in separate batches."""
    g = _disjoint_union(gg.rmat(10, 8, seed=31), gg.grid_full(40, 40))
    rng = np.random.default_rng(32)
    src = np.concatenate([rng.choice(1024, 130, replace=False),
                          1024 + rng.choice(1600, 60, replace=False)]).astype(np.int32)
    want = oracle_bc(g, src)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        first = batched(G, src, concurrency=conc, level_loop=bcm.BC_LOOP_HOST)
        check_bc(first, want)
        # the pooled workspaces (some built narrow) serve the next calls
        again = batched(G, src, concurrency=conc, level_loop=bcm.BC_LOOP_HOST)
        check_bc(again, want)
        check_bc(batched(G, src[:64], level_loop=bcm.BC_LOOP_HOST), oracle_bc(g, src[:64]))
