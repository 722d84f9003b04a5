"""Pins for the CPU oracle: facts fixed independently of it.

Each check is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign, a wrong level offset, a transposed ratio, counting the source's own
dependency, a missing reset between sources) breaks at least one of them;
tests/test_oracle_mutants.py plants such slips in a copy of the oracle and
checks that these pins catch them.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import graphgen as gg
import oracle
from tests.bruteforce import (adjacency, bc_by_definition, csr_from_adjacency, parse_golden,
                              walk_dist_sigma)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_worked.txt")


def all_bc(g, sources=None):
    src = np.arange(g.n, dtype=np.int32) if sources is None else np.asarray(sources, np.int32)
    bc, st = oracle.bc(g.row_ptr, g.col_idx, src)
    assert st == oracle.OK
    return bc


def hop_distances(g, s):
    """Unweighted hop distances by scipy's shortest_path (independent BFS)."""
    m = sp.csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    d = shortest_path(m, method="D", unweighted=True, indices=[s])[0]
    return np.where(np.isinf(d), -1, d).astype(np.int64)


# ---------------------------------------------------------------------------
# Hand-worked examples (tests/golden/hand_worked.txt)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", parse_golden(GOLDEN), ids=lambda c: c["name"])
def test_hand_worked(case):
    e = np.asarray(case["edges"], dtype=np.int32).reshape(-1, 2)
    g = gg.csr_from_edges(case["n"], e[:, 0], e[:, 1])
    bc = all_bc(g, case["sources"])
    np.testing.assert_allclose(bc, case["bc"], rtol=1e-15, atol=1e-15)
    for s, d in case["dist"].items():
        dist, sigma, _, st = oracle.single_source(g.row_ptr, g.col_idx, s)
        assert st == oracle.OK
        assert dist.tolist() == d
        assert sigma.tolist() == case["sigma"][s]


# ---------------------------------------------------------------------------
# Brute force: walk counts + the definition
# ---------------------------------------------------------------------------

def _graphs_from_bits(n, bits_batch):
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    A = np.zeros((len(bits_batch), n, n), dtype=np.int64)
    for k, (i, j) in enumerate(pairs):
        on = ((bits_batch >> k) & 1).astype(bool)
        A[on, i, j] = 1
        A[on, j, i] = 1
    return A


@pytest.mark.parametrize("n", [4, 5, 6])
def test_exhaustive_small_graphs(n):
    """Every labelled simple graph on n <= 6 vertices (2**15 graphs at n=6)."""
    n_pairs = n * (n - 1) // 2
    total = 1 << n_pairs
    chunk = 2048
    for lo in range(0, total, chunk):
        bits = np.arange(lo, min(total, lo + chunk), dtype=np.int64)
        A = _graphs_from_bits(n, bits)
        want = bc_by_definition(A)
        for gi in range(A.shape[0]):
            rp, ci = csr_from_adjacency(A[gi])
            got, st = oracle.bc(rp, ci, np.arange(n, dtype=np.int32))
            assert st == oracle.OK
            np.testing.assert_allclose(got, want[gi], rtol=1e-12, atol=1e-12,
                                       err_msg=f"graph bits {bits[gi]}")


def test_random_graphs_definition_and_subsets():
    """G(n,p) up to 14 vertices, all sources and random source multisets."""
    rng = np.random.default_rng(7)
    for trial in range(120):
        n = int(rng.integers(2, 15))
        p = float(rng.uniform(0.1, 0.7))
        g = gg.gnp(n, p, seed=trial)
        A = adjacency(g.row_ptr, g.col_idx)
        np.testing.assert_allclose(all_bc(g), bc_by_definition(A), rtol=1e-12, atol=1e-12)
        srcs = rng.integers(0, n, size=int(rng.integers(1, 2 * n)))
        np.testing.assert_allclose(all_bc(g, srcs), bc_by_definition(A, srcs), rtol=1e-12,
                                   atol=1e-12)


def test_multigraph_and_self_loops():
    """Parallel arcs count as distinct paths; self-loops change nothing."""
    rng = np.random.default_rng(11)
    for trial in range(60):
        n = int(rng.integers(3, 10))
        m = int(rng.integers(n, 3 * n))
        u = rng.integers(0, n, size=m)
        v = rng.integers(0, n, size=m)
        g = gg.csr_from_edges(n, u, v, dedup=False, drop_loops=False)
        A = adjacency(g.row_ptr, g.col_idx)
        np.testing.assert_allclose(all_bc(g), bc_by_definition(A), rtol=1e-12, atol=1e-12)
        # dropping the loops leaves BC unchanged
        g2 = gg.csr_from_edges(n, u, v, dedup=False, drop_loops=True)
        np.testing.assert_allclose(all_bc(g2), all_bc(g), rtol=1e-12, atol=1e-12)


def test_dist_sigma_walk_counts():
    rng = np.random.default_rng(3)
    for trial in range(60):
        n = int(rng.integers(2, 16))
        g = gg.gnp(n, float(rng.uniform(0.1, 0.6)), seed=100 + trial)
        A = adjacency(g.row_ptr, g.col_idx)
        D, S = walk_dist_sigma(A)
        for s in range(n):
            dist, sigma, _, st = oracle.single_source(g.row_ptr, g.col_idx, s)
            assert st == oracle.OK
            assert dist.tolist() == D[s].tolist()
            assert sigma.tolist() == S[s].astype(np.float64).tolist()


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 7, 50, 301])
def test_path_closed_form(n):
    i = np.arange(n)
    np.testing.assert_array_equal(all_bc(gg.path(n)), 2.0 * i * (n - 1 - i))


@pytest.mark.parametrize("n", [2, 3, 10, 257])
def test_star_closed_form(n):
    want = np.zeros(n)
    want[0] = (n - 1) * (n - 2)
    np.testing.assert_array_equal(all_bc(gg.star(n)), want)


@pytest.mark.parametrize("n", [3, 4, 5, 6, 11, 12, 101, 128])
def test_cycle_closed_form(n):
    k = n // 2
    val = k * (k - 1) if n % 2 else (k - 1) ** 2
    np.testing.assert_allclose(all_bc(gg.cycle(n)), np.full(n, float(val)), rtol=1e-13)


def test_cycle_sigma_antipode():
    for n in (4, 10, 64):
        dist, sigma, _, _ = oracle.single_source(gg.cycle(n).row_ptr, gg.cycle(n).col_idx, 0)
        assert dist[n // 2] == n // 2 and sigma[n // 2] == 2.0
        assert np.all(sigma[np.arange(n) != n // 2] == 1.0)


@pytest.mark.parametrize("seed", range(8))
def test_tree_closed_form(seed):
    """BC(v) = (n-1)**2 - sum of squared component sizes of T - v; sigma = 1."""
    n = 40 + 7 * seed
    g = gg.random_tree(n, seed)
    want = np.empty(n)
    for v in range(n):
        seen = np.zeros(n, bool)
        seen[v] = True
        sizes = []
        for r in g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]:
            stack, size = [r], 0
            seen[r] = True
            while stack:
                x = stack.pop()
                size += 1
                for y in g.col_idx[g.row_ptr[x]:g.row_ptr[x + 1]]:
                    if not seen[y]:
                        seen[y] = True
                        stack.append(y)
            sizes.append(size)
        want[v] = (n - 1) ** 2 - sum(s * s for s in sizes)
    np.testing.assert_array_equal(all_bc(g), want)
    _, sigma, _, _ = oracle.single_source(g.row_ptr, g.col_idx, seed % n)
    assert np.all(sigma == 1.0)


@pytest.mark.parametrize("a,b", [(1, 1), (1, 5), (2, 3), (3, 7), (6, 6)])
def test_complete_bipartite_closed_form(a, b):
    g = gg.complete_bipartite(a, b)
    want = np.concatenate([np.full(a, b * (b - 1) / a), np.full(b, a * (a - 1) / b)])
    np.testing.assert_allclose(all_bc(g), want, rtol=1e-14)
    if a > 1:
        _, sigma, _, _ = oracle.single_source(g.row_ptr, g.col_idx, 0)
        assert np.all(sigma[1:a] == b)          # same side: one path through each of b


@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_complete_graph_zero(n):
    np.testing.assert_array_equal(all_bc(gg.complete(n)), np.zeros(n))


@pytest.mark.parametrize("d", [1, 2, 3, 5, 8])
def test_hypercube_closed_form(d):
    g = gg.hypercube(d)
    val = d * 2 ** (d - 1) - 2 ** d + 1
    np.testing.assert_allclose(all_bc(g), np.full(1 << d, float(val)), rtol=1e-12)


def test_hypercube_sigma_factorial():
    """From vertex 0 of Q_18, sigma(t) = popcount(t)! (all below 2**53: 18! < 2**53)."""
    d = 18
    g = gg.hypercube(d)
    dist, sigma, _, st = oracle.single_source(g.row_ptr, g.col_idx, 0)
    assert st == oracle.OK
    pc = np.array([bin(t).count("1") for t in range(1 << d)])
    assert np.array_equal(dist, pc)
    fact = np.array([float(math.factorial(k)) for k in range(d + 1)])
    assert np.array_equal(sigma, fact[pc])


def test_lattice_sigma_binomial():
    """From the corner of a full lattice, sigma(x, y) = C(x+y, x): exact below
    2**53, within 1e-15 relative above (the 60x60 lattice crosses at x+y=57)."""
    rows = cols = 60
    g = gg.grid_full(rows, cols)
    dist, sigma, _, st = oracle.single_source(g.row_ptr, g.col_idx, 0)
    assert st == oracle.OK
    for r in range(rows):
        for c in range(cols):
            v = r * cols + c
            want = math.comb(r + c, r)
            assert dist[v] == r + c
            if want < 2 ** 53:
                assert sigma[v] == float(want)
            else:
                assert abs(sigma[v] - want) <= 1e-15 * want * (r + c)


def test_lattice_overflow_reports_range():
    """sigma from a corner of a 600x600 lattice reaches C(1198, 599) > DBL_MAX."""
    g = gg.grid_full(600, 600)
    _, sigma, _, st = oracle.single_source(g.row_ptr, g.col_idx, 0, with_delta=False)
    assert st == oracle.RANGE and np.isinf(sigma).any()
    _, st2 = oracle.bc(g.row_ptr, g.col_idx, np.array([0], np.int32))
    assert st2 == oracle.RANGE


# ---------------------------------------------------------------------------
# Invariants on the benchmark-shaped R-MAT scale 12 graph
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def rmat12():
    return gg.rmat(12, 8, seed=1)


def test_distances_match_scipy(rmat12):
    for s in gg.sample_sources(rmat12, 12, seed=5):
        dist, _, _, _ = oracle.single_source(rmat12.row_ptr, rmat12.col_idx, s, False)
        assert np.array_equal(dist, hop_distances(rmat12, s))


def test_sum_invariant_all_sources(rmat12):
    """sum_v BC(v) = sum over s, reachable t != s of (d(s,t) - 1), with d from scipy."""
    g = rmat12
    bc = all_bc(g)
    m = sp.csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    D = shortest_path(m, method="D", unweighted=True)
    fin = np.isfinite(D) & (D > 0)
    want = float((D[fin] - 1).sum())
    assert abs(bc.sum() - want) <= 1e-9 * want
    assert np.all(bc >= 0)


def test_per_source_delta_sum(rmat12):
    """sum over v != s of delta_s(v) = sum over reachable t != s of (d(s,t) - 1)."""
    for s in gg.sample_sources(rmat12, 16, seed=6):
        dist, sigma, delta, _ = oracle.single_source(rmat12.row_ptr, rmat12.col_idx, s)
        d = hop_distances(rmat12, s)
        want = float((d[d > 0] - 1).sum())
        got = float(delta.sum() - delta[s])
        assert abs(got - want) <= 1e-10 * max(1.0, want)


def test_additivity_and_duplicates(rmat12):
    s = gg.sample_sources(rmat12, 40, seed=8)
    a, b = s[:17], s[17:]
    np.testing.assert_allclose(all_bc(rmat12, s), all_bc(rmat12, a) + all_bc(rmat12, b),
                               rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(all_bc(rmat12, np.concatenate([a, a])), 2 * all_bc(rmat12, a),
                               rtol=1e-12, atol=1e-9)


def test_thread_count_does_not_change_result(rmat12):
    s = gg.sample_sources(rmat12, 64, seed=9)
    b1, _ = oracle.bc(rmat12.row_ptr, rmat12.col_idx, s, threads=1)
    b4, _ = oracle.bc(rmat12.row_ptr, rmat12.col_idx, s, threads=4)
    np.testing.assert_allclose(b1, b4, rtol=1e-13, atol=1e-9)


# ---------------------------------------------------------------------------
# NetworkX (independent library)
# ---------------------------------------------------------------------------

def test_networkx_cross_check():
    nx = pytest.importorskip("networkx")
    graphs = [gg.gnp(n, 0.3, seed=n) for n in range(5, 30, 3)] + [gg.rmat(8, 8, seed=2)]
    for g in graphs:
        G = nx.Graph()
        G.add_nodes_from(range(g.n))
        for u in range(g.n):
            for v in g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]:
                G.add_edge(u, int(v))
        ref = nx.betweenness_centrality(G, normalized=False)
        want = np.array([2.0 * ref[v] for v in range(g.n)])
        np.testing.assert_allclose(all_bc(g), want, rtol=1e-10, atol=1e-10)


# ---------------------------------------------------------------------------
# Edge cases and argument checks
# ---------------------------------------------------------------------------

def test_edge_cases():
    g = gg.path(5)
    bc, st = oracle.bc(g.row_ptr, g.col_idx, np.zeros(0, np.int32))
    assert st == oracle.OK and np.all(bc == 0)
    single = gg.csr_from_edges(1, [], [])
    bc, st = oracle.bc(single.row_ptr, single.col_idx, np.array([0], np.int32))
    assert st == oracle.OK and bc.tolist() == [0.0]
    empty = gg.csr_from_edges(6, [], [])
    assert np.all(all_bc(empty) == 0)
    with pytest.raises(oracle.OracleError):
        oracle.bc(g.row_ptr, g.col_idx, np.array([5], np.int32))
    with pytest.raises(oracle.OracleError):
        oracle.single_source(g.row_ptr, g.col_idx, -1)


# ---------------------------------------------------------------------------
# Extended range (long double): counts beyond double's range
# ---------------------------------------------------------------------------

def as_fraction(m, e):
    """Exact value m * 2**e of the extended oracle's (mantissa, exponent) pair.
    The mantissa comes back rounded to double (53 bits) from the oracle's
    64-bit long double, so comparisons allow 2**-53 for that rounding."""
    from fractions import Fraction
    return Fraction(float(m)) * (Fraction(2) ** int(e))


def test_ext_oracle_computes_in_extended_precision():
    assert oracle.long_double_digits() >= 64


@pytest.mark.parametrize("k,width", [(1100, 2), (700, 3)])
def test_ext_diamond_chain_closed_form(k, width):
    """Chain of k diamonds of `width` middles, from hub 0: hub i has
    sigma = width**i (past 2**1024 here) and dependency (width+1)*(k-i); a
    middle vertex of diamond i carries 1/width of every path to hub i and
    beyond, so delta = (1 + (width+1)*(k-i)) / width.  The double oracle
    overflows on the same graph."""
    from fractions import Fraction
    g = gg.diamond_chain(k, width)
    step = width + 1
    dist, sm, se, delta, st = oracle.single_source_ext(g.row_ptr, g.col_idx, 0)
    assert st == oracle.OK
    _, _, _, st64 = oracle.single_source(g.row_ptr, g.col_idx, 0)
    assert st64 == oracle.RANGE
    for i in range(1, k + 1):
        hub = i * step
        assert dist[hub] == 2 * i
        want = Fraction(width) ** i
        got = as_fraction(sm[hub], se[hub])
        assert abs(got - want) <= want * (Fraction(1, 2 ** 53) + Fraction(i, 2 ** 62))
        assert delta[hub] == pytest.approx((width + 1) * (k - i), rel=1e-15, abs=0)
        for j in range(1, width + 1):
            mid = hub - step + j
            assert dist[mid] == 2 * i - 1
            want_m = Fraction(width) ** (i - 1)
            assert (abs(as_fraction(sm[mid], se[mid]) - want_m)
                    <= want_m * (Fraction(1, 2 ** 53) + Fraction(i, 2 ** 62)))
            assert delta[mid] == pytest.approx((1 + (width + 1) * (k - i)) / width, rel=1e-15)
    bc, st2 = oracle.bc_ext(g.row_ptr, g.col_idx, np.array([0], np.int32))
    assert st2 == oracle.OK
    want_bc = delta.copy()
    want_bc[0] = 0.0
    assert np.array_equal(bc, want_bc)


def test_ext_lattice_sigma_binomial():
    """From the corner of a 600x600 lattice sigma(r, c) = C(r+c, r), up to
    C(1198, 599) ~ 2**1194: the extended oracle's counts against exact big
    integers on a sample of vertices."""
    from fractions import Fraction
    rows = cols = 600
    g = gg.grid_full(rows, cols)
    dist, sm, se, _, st = oracle.single_source_ext(g.row_ptr, g.col_idx, 0, with_delta=False)
    assert st == oracle.OK
    rng = np.random.default_rng(3)
    for v in list(rng.integers(0, g.n, 300)) + [g.n - 1, cols - 1, (rows - 1) * cols]:
        r, c = divmod(int(v), cols)
        assert dist[v] == r + c
        want = Fraction(math.comb(r + c, r))
        assert (abs(as_fraction(sm[v], se[v]) - want)
                <= want * (Fraction(1, 2 ** 53) + Fraction(r + c + 1, 2 ** 62)))


def test_ext_matches_double_oracle_when_counts_fit():
    """Where every count fits double, the extended oracle gives the double
    oracle's results (to rounding)."""
    for g in (gg.rmat(11, 8, seed=21), gg.grid_road(40, 40, seed=22), gg.hypercube(8)):
        src = gg.sample_sources(g, 50, seed=23)
        a, st = oracle.bc(g.row_ptr, g.col_idx, src)
        b, st2 = oracle.bc_ext(g.row_ptr, g.col_idx, src)
        assert st == st2 == oracle.OK
        nz = a != 0
        assert np.array_equal(nz, b != 0)
        assert np.max(np.abs(a[nz] - b[nz]) / a[nz]) < 1e-12
        for s in src[:3]:
            d0, s0, dl0, _ = oracle.single_source(g.row_ptr, g.col_idx, int(s))
            d1, sm, se, dl1, _ = oracle.single_source_ext(g.row_ptr, g.col_idx, int(s))
            assert np.array_equal(d0, d1)
            assert np.array_equal(np.ldexp(sm, se), s0)  # integers below 2**53: exact
            assert np.allclose(dl1, dl0, rtol=1e-13, atol=0)


def test_ext_sum_invariant_deep_road_grid():
    """Road-like 1024x1024 grid without shortcuts (~1,700 levels, counts past
    double's range): sum_v BC(v) = sum over sources of sum_t (d(s,t) - 1)."""
    g = gg.grid_road(1024, 1024, 0.05, 0.0, seed=2)
    src = gg.sample_sources(g, 2, seed=102)
    bc, st = oracle.bc_ext(g.row_ptr, g.col_idx, src)
    assert st == oracle.OK
    want = 0
    for s in src:
        d = hop_distances(g, int(s))
        r = d[d > 0]
        assert r.max() > 1000
        want += int((r - 1).sum())
    assert abs(bc.sum() - want) <= 1e-12 * want


# ---------------------------------------------------------------------------
# Directed graphs (the CSR lists out-arcs)
# ---------------------------------------------------------------------------

def dir_bc(g, sources=None):
    src = np.arange(g.n, dtype=np.int32) if sources is None else np.asarray(sources, np.int32)
    bc, st = oracle.bc(g.row_ptr, g.col_idx, src, directed=True)
    assert st == oracle.OK
    return bc


@pytest.mark.parametrize("n", [2, 7, 50])
def test_directed_path_closed_form(n):
    """0 -> 1 -> ... -> n-1: vertex i lies on the paths from the i vertices before
    it to the n-1-i after it."""
    g = gg.directed(n, [(i, i + 1) for i in range(n - 1)], f"dpath-{n}")
    want = np.array([i * (n - 1 - i) for i in range(n)], dtype=np.float64)
    assert np.array_equal(dir_bc(g), want)


@pytest.mark.parametrize("n", [3, 9, 12])
def test_directed_cycle_closed_form(n):
    """Directed n-cycle: the unique path of length d has d-1 interior vertices, n
    paths of each length 1..n-1, spread evenly: BC = (n-1)(n-2)/2 everywhere."""
    g = gg.directed(n, [(i, (i + 1) % n) for i in range(n)], f"dcycle-{n}")
    assert np.array_equal(dir_bc(g), np.full(n, (n - 1) * (n - 2) / 2))


def test_directed_stars_and_diamond():
    """Out-star and in-star: no path has an interior vertex.  Diamond DAG
    0 -> {1, 2} -> 3: 1 and 2 each carry half of the one pair (0, 3)."""
    n = 9
    out_star = gg.directed(n, [(0, i) for i in range(1, n)], "out-star")
    in_star = gg.directed(n, [(i, 0) for i in range(1, n)], "in-star")
    assert not dir_bc(out_star).any() and not dir_bc(in_star).any()
    both = gg.directed(n, [(0, i) for i in range(1, n)] + [(i, 0) for i in range(1, n)], "star")
    want = np.zeros(n)
    want[0] = (n - 1) * (n - 2)
    assert np.array_equal(dir_bc(both), want)
    dia = gg.directed(4, [(0, 1), (0, 2), (1, 3), (2, 3)], "diamond-dag")
    assert np.array_equal(dir_bc(dia), [0.0, 0.5, 0.5, 0.0])
    d, sg, dl, st = oracle.single_source(dia.row_ptr, dia.col_idx, 0, directed=True)
    assert list(d) == [0, 1, 1, 2] and list(sg) == [1, 1, 1, 2] and list(dl) == [0, 0.5, 0.5, 0]
    d, sg, _, _ = oracle.single_source(dia.row_ptr, dia.col_idx, 3, directed=True)
    assert list(d) == [-1, -1, -1, 0] and list(sg) == [0, 0, 0, 1]


def test_directed_random_definition():
    """Random digraphs up to 12 vertices: BC from the definition (walk counting
    on the directed adjacency), all sources and random multisets; dist and sigma
    of single sources against the walk counts."""
    rng = np.random.default_rng(17)
    for trial in range(80):
        n = int(rng.integers(2, 13))
        g = gg.gnp_directed(n, float(rng.uniform(0.05, 0.5)), seed=trial)
        A = adjacency(g.row_ptr, g.col_idx)
        np.testing.assert_allclose(dir_bc(g), bc_by_definition(A), rtol=1e-12, atol=1e-12)
        srcs = rng.integers(0, n, size=int(rng.integers(1, 2 * n)))
        np.testing.assert_allclose(dir_bc(g, srcs), bc_by_definition(A, srcs), rtol=1e-12,
                                   atol=1e-12)
        dist, sigma = walk_dist_sigma(A)
        for s in range(min(n, 3)):
            d, sg, _, st = oracle.single_source(g.row_ptr, g.col_idx, s, directed=True)
            assert st == oracle.OK
            assert np.array_equal(d, dist[s]) and np.array_equal(sg, sigma[s])


def test_directed_networkx_cross_check():
    nx = pytest.importorskip("networkx")
    graphs = [gg.gnp_directed(n, 0.2, seed=n) for n in range(5, 26, 5)]
    graphs.append(gg.rmat(8, 8, seed=2, directed=True))
    for g in graphs:
        G = nx.DiGraph()
        G.add_nodes_from(range(g.n))
        for u in range(g.n):
            for v in g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]:
                G.add_edge(u, int(v))
        ref = nx.betweenness_centrality(G, normalized=False)  # ordered pairs for digraphs
        want = np.array([ref[v] for v in range(g.n)])
        np.testing.assert_allclose(dir_bc(g), want, rtol=1e-10, atol=1e-10)


def test_directed_on_symmetric_graph_equals_undirected(rmat12):
    src = gg.sample_sources(rmat12, 60, seed=5)
    a = all_bc(rmat12, src)
    b = dir_bc(rmat12, src)
    assert np.max(np.abs(a - b) / np.maximum(a, 1)) < 1e-12


def test_directed_sum_invariant():
    """Directed R-MAT scale 12: sum_v BC(v) = sum_s sum_{t reachable} (d(s,t) - 1),
    with directed distances from scipy."""
    g = gg.rmat(12, 8, seed=9, directed=True)
    src = gg.sample_sources(g, 40, seed=10)
    m = sp.csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    d = shortest_path(m, method="D", directed=True, unweighted=True, indices=src)
    want = float(np.where(np.isfinite(d) & (d > 0), d - 1, 0).sum())
    got = dir_bc(g, src).sum()
    assert abs(got - want) <= 1e-10 * want


# ---------------------------------------------------------------------------
# Single-source shortest paths (weighted)
# ---------------------------------------------------------------------------

def dijkstra(g, w, s):
    """scipy's Dijkstra on the weighted CSR (an independent method); -1 unreachable."""
    from scipy.sparse.csgraph import dijkstra as sp_dijkstra
    # csr_matrix would add parallel arcs' weights: keep the lightest arc of each pair
    u = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    order = np.lexsort((w, g.col_idx, u))
    u, v, ww = u[order], g.col_idx[order], w[order]
    first = np.ones(len(u), bool)
    first[1:] = (u[1:] != u[:-1]) | (v[1:] != v[:-1])
    m = sp.csr_matrix((ww[first].astype(np.float64), (u[first], v[first])), shape=(g.n, g.n))
    d = sp_dijkstra(m, directed=True, indices=[s])[0]
    return np.where(np.isinf(d), -1, d).astype(np.int64)


@pytest.mark.parametrize("g", [gg.rmat(12, 8, seed=1), gg.grid_road(64, 64, seed=2),
                               gg.rmat(11, 8, seed=4, directed=True),
                               gg.gnp_directed(80, 0.03, seed=5)], ids=lambda g: g.name)
def test_sssp_matches_dijkstra(g):
    w = gg.edge_weights(g, seed=7)
    for s in gg.sample_sources(g, 6, seed=8):
        d, passes = oracle.sssp(g.row_ptr, g.col_idx, w, int(s))
        assert np.array_equal(d, dijkstra(g, w, int(s)))
        assert passes >= 1


def test_sssp_unit_weights_are_hop_distances():
    g = gg.rmat(12, 8, seed=2)
    w = np.ones(g.nnz, dtype=np.int32)
    for s in gg.sample_sources(g, 4, seed=3):
        d, _ = oracle.sssp(g.row_ptr, g.col_idx, w, int(s))
        assert np.array_equal(d, hop_distances(g, int(s)))


def test_sssp_path_prefix_sums_and_zero_weights():
    """Weighted path: dist(i) = sum of the first i weights; zero weights allowed;
    an unreachable vertex gives -1; a directed path is one-way."""
    n = 40
    rng = np.random.default_rng(1)
    wts = rng.integers(0, 100, n - 1).astype(np.int32)
    g = gg.path(n)
    w = np.empty(g.nnz, np.int32)
    for u in range(n):
        for e in range(g.row_ptr[u], g.row_ptr[u + 1]):
            w[e] = wts[min(u, g.col_idx[e])]
    d, _ = oracle.sssp(g.row_ptr, g.col_idx, w, 0)
    assert np.array_equal(d, np.concatenate([[0], np.cumsum(wts)]))
    dp = gg.directed(n + 1, [(i, i + 1) for i in range(n - 1)], "dpath")
    d, _ = oracle.sssp(dp.row_ptr, dp.col_idx, wts, 5)
    assert np.all(d[:5] == -1) and d[n] == -1
    assert np.array_equal(d[5:n], np.concatenate([[0], np.cumsum(wts[5:n - 1])]))


def test_sssp_rejects_negative_weights():
    g = gg.path(3)
    with pytest.raises(oracle.OracleError):
        oracle.sssp(g.row_ptr, g.col_idx, np.array([1, -1, 1, 1], np.int32), 0)


# ---------------------------------------------------------------------------
# PageRank
# ---------------------------------------------------------------------------

def pr_fixed_point(g, damping):
    """Solution of x = (1 - d)/n + d * P x with P[v, u] = 1/outdeg(u) per arc u->v,
    by scipy's sparse direct solver (an independent method)."""
    import scipy.sparse.linalg as sla
    n = g.n
    deg = np.diff(g.row_ptr).astype(np.float64)
    u = np.repeat(np.arange(n), np.diff(g.row_ptr))
    P = sp.csr_matrix((1.0 / deg[u], (g.col_idx, u)), shape=(n, n))
    A = (sp.identity(n, format="csr") - damping * P).tocsc()
    return sla.spsolve(A, np.full(n, (1.0 - damping) / n))


@pytest.mark.parametrize("g", [gg.cycle(12), gg.complete(9), gg.hypercube(6),
                               gg.torus(6, 7)], ids=lambda g: g.name)
def test_pagerank_regular_graphs_uniform(g):
    pr, it, _ = oracle.pagerank(g.row_ptr, g.col_idx, 0.85, 1e-14, 50)
    np.testing.assert_allclose(pr, np.full(g.n, 1.0 / g.n), rtol=1e-14)


@pytest.mark.parametrize("g", [gg.rmat(10, 8, seed=1), gg.rmat(10, 8, seed=2, directed=True),
                               gg.gnp_directed(60, 0.08, seed=3), gg.grid_road(30, 30, seed=4)],
                         ids=lambda g: g.name)
def test_pagerank_converges_to_fixed_point(g):
    """Iterated to a tight tolerance, the ranks are the linear system's solution
    (dangling vertices leak their rank, as in the paper's formula)."""
    for d in (0.85, 0.5):
        pr, it, last = oracle.pagerank(g.row_ptr, g.col_idx, d, 1e-13, 2000)
        assert last <= 1e-13 and it < 2000
        np.testing.assert_allclose(pr, pr_fixed_point(g, d), rtol=1e-9, atol=1e-15)


def test_pagerank_star_one_iteration():
    """Leaves -> centre (n = 9): after one iteration from 1/n the centre has
    (1-d)/n + d (n-1)/n, the leaves (1-d)/n; the next L1 change follows."""
    n, d = 9, 0.85
    g = gg.directed(n, [(i, 0) for i in range(1, n)], "in-star")
    pr, it, last = oracle.pagerank(g.row_ptr, g.col_idx, d, 0.0, 1)
    assert it == 1
    want = np.full(n, (1 - d) / n)
    want[0] += d * (n - 1) / n
    np.testing.assert_allclose(pr, want, rtol=1e-15)
    np.testing.assert_allclose(last, abs(want[0] - 1 / n) + (n - 1) * abs(want[1] - 1 / n),
                               rtol=1e-14)


def test_pagerank_stopping_rule():
    g = gg.rmat(9, 8, seed=5)
    _, it_cap, _ = oracle.pagerank(g.row_ptr, g.col_idx, 0.85, 0.0, 7)
    assert it_cap == 7
    pr, it, last = oracle.pagerank(g.row_ptr, g.col_idx, 0.85, 1e-6, 1000)
    assert last <= 1e-6
    _, _, prev = oracle.pagerank(g.row_ptr, g.col_idx, 0.85, 0.0, it - 1)
    assert prev > 1e-6


def test_pagerank_networkx_cross_check():
    nx = pytest.importorskip("networkx")
    for g in (gg.rmat(9, 8, seed=6), gg.cycle(40), gg.gnp(50, 0.2, seed=7)):
        if (np.diff(g.row_ptr) == 0).any():
            continue   # NetworkX spreads dangling rank; the paper's formula does not
        G = nx.DiGraph()
        G.add_nodes_from(range(g.n))
        for u in range(g.n):
            for v in g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]:
                G.add_edge(u, int(v))
        ref = nx.pagerank(G, alpha=0.85, tol=1e-14, max_iter=10000)
        pr, _, _ = oracle.pagerank(g.row_ptr, g.col_idx, 0.85, 1e-15, 10000)
        np.testing.assert_allclose(pr, [ref[v] for v in range(g.n)], rtol=1e-8)
