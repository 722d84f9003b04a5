"""Plant plausible slips in a copy of the oracle and check that the pins catch them.

Each mutant is a textual edit of oracle/bc_oracle.c compiled into a temporary
library; the committed oracle is never touched.  A mutant survives only if no
pin in tests/test_oracle_pins.py notices it, which would mean the pins leave
that part of the oracle unchecked.
"""
import os
import subprocess

import pytest

import graphgen as gg
import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "bc_oracle.c")

MUTANTS = {
    "drop-one-plus": ("(1.0 + delta[w])", "(delta[w])"),
    "transposed-ratio": ("(sigma[v] / sigma[w])", "(sigma[w] / sigma[v])"),
    "forward-siblings": ("if (dist[w] == dist[v] - 1) acc = acc + sigma[w];",
                         "if (dist[w] == dist[v]) acc = acc + sigma[w];"),
    "backward-siblings-too": ("if (dist[w] == dist[v] + 1) acc",
                              "if (dist[w] >= dist[v] && w != v) acc"),
    "source-counts-itself": ("for (int32_t i = reached - 1; i >= 1; --i)",
                             "for (int32_t i = reached - 1; i >= 0; --i)"),
    "sigma-src-two": ("sigma[s] = 1.0;", "sigma[s] = 2.0;"),
    "bc-overwrite": ("if (bc) bc[v] = bc[v] + delta[v];", "if (bc) bc[v] = delta[v];"),
    "bfs-level-plus-two": ("dist[w] = dist[v] + 1;", "dist[w] = dist[v] + (w == 1 ? 2 : 1);"),
    "no-range-flag": ("if (!isfinite(acc)) status = OR_RANGE;", ""),
}


def _pin_suite():
    """Run a quick subset of the pins against whatever library `oracle` has loaded."""
    for case in pins.parse_golden(pins.GOLDEN):
        pins.test_hand_worked(case)
    pins.test_exhaustive_small_graphs(5)
    pins.test_random_graphs_definition_and_subsets()
    pins.test_multigraph_and_self_loops()
    pins.test_dist_sigma_walk_counts()
    for n in (7, 50):
        pins.test_path_closed_form(n)
    pins.test_star_closed_form(10)
    for n in (11, 12):
        pins.test_cycle_closed_form(n)
    pins.test_tree_closed_form(0)
    pins.test_complete_bipartite_closed_form(3, 7)
    pins.test_hypercube_closed_form(5)
    pins.test_lattice_sigma_binomial()
    pins.test_lattice_overflow_reports_range()


@pytest.fixture()
def swap_oracle(tmp_path):
    saved = (oracle._LIB_PATH, oracle._lib)

    def load(text):
        c = tmp_path / "mutant.c"
        so = tmp_path / f"mutant{len(os.listdir(tmp_path))}.so"
        c.write_text(text)
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", str(c), "-o",
                        str(so), "-lm"], check=True)
        oracle._LIB_PATH, oracle._lib = str(so), None

    yield load
    oracle._LIB_PATH, oracle._lib = saved


def test_unmutated_copy_passes(swap_oracle):
    swap_oracle(open(SRC).read())
    _pin_suite()


# The extended-range (long double) copy of the algorithm sits after this
# marker; the double oracle's mutants edit the text before it, the extended
# ones the text after it.
EXT_MARK = "/* ---- extended range"

EXT_MUTANTS = {
    "drop-one-plus": ("(1.0L + delta[w])", "(delta[w])"),
    "transposed-ratio": ("(sigma[v] / sigma[w])", "(sigma[w] / sigma[v])"),
    "forward-siblings": ("if (dist[w] == dist[v] - 1) acc = acc + sigma[w];",
                         "if (dist[w] == dist[v]) acc = acc + sigma[w];"),
    "backward-siblings-too": ("if (dist[w] == dist[v] + 1) acc",
                              "if (dist[w] >= dist[v] && w != v) acc"),
    "source-counts-itself": ("for (int32_t i = reached - 1; i >= 1; --i)",
                             "for (int32_t i = reached - 1; i >= 0; --i)"),
    "sigma-src-two": ("sigma[s] = 1.0L;", "sigma[s] = 2.0L;"),
    "bc-overwrite": ("if (bc) bc[v] = bc[v] + delta[v];", "if (bc) bc[v] = delta[v];"),
    "double-precision": ("long double acc = 0.0L;\n        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {\n            int32_t w = col_idx[e];\n            if (dist[w] == dist[v] - 1)",
                         "double acc = 0.0;\n        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {\n            int32_t w = col_idx[e];\n            if (dist[w] == dist[v] - 1)"),
}


# Slips in the directed forward pass (the reverse pass is shared with the
# undirected case and covered above).
DIR_MUTANTS = {
    "directed-pulls-like-undirected": ("    if (directed) {", "    if (0) {"),
    "push-without-level-test": ("if (dist[w] == dist[v] + 1) sigma[w] = sigma[w] + sigma[v];",
                                "if (dist[w] >= dist[v] && w != v) sigma[w] = sigma[w] + sigma[v];"),
    "push-skips-source": ("        for (int32_t i = 0; i < reached; ++i) {\n            int32_t v = order[i];\n            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {\n                int32_t w = col_idx[e];\n                if (dist[w] == dist[v] + 1) sigma[w]",
                          "        for (int32_t i = 1; i < reached; ++i) {\n            int32_t v = order[i];\n            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {\n                int32_t w = col_idx[e];\n                if (dist[w] == dist[v] + 1) sigma[w]"),
    "push-overwrites": ("if (dist[w] == dist[v] + 1) sigma[w] = sigma[w] + sigma[v];",
                        "if (dist[w] == dist[v] + 1) sigma[w] = sigma[v];"),
}


def _directed_pin_suite():
    for n in (7, 50):
        pins.test_directed_path_closed_form(n)
    pins.test_directed_cycle_closed_form(9)
    pins.test_directed_stars_and_diamond()
    pins.test_directed_random_definition()


def test_unmutated_copy_passes_directed_pins(swap_oracle):
    swap_oracle(open(SRC).read())
    _directed_pin_suite()


@pytest.mark.parametrize("name", sorted(DIR_MUTANTS))
def test_directed_mutant_is_caught(name, swap_oracle):
    before, after = DIR_MUTANTS[name]
    swap_oracle(_mutate(open(SRC).read(), before, after, ext=False))
    with pytest.raises(AssertionError):
        _directed_pin_suite()


SSSP_MUTANTS = {
    "sssp-unit-weights": ("int64_t dist_new = dist[v] + weight[e];",
                          "int64_t dist_new = dist[v] + 1;"),
    "sssp-single-pass": ("                    finished = 0;\n", ""),
    "sssp-forgets-next": ("                    modified_next[nbr] = 1;\n", ""),
}


def _sssp_pin_suite():
    for g in (gg.rmat(12, 8, seed=1), gg.grid_road(64, 64, seed=2)):
        pins.test_sssp_matches_dijkstra(g)
    pins.test_sssp_path_prefix_sums_and_zero_weights()


def test_unmutated_copy_passes_sssp_pins(swap_oracle):
    swap_oracle(open(SRC).read())
    _sssp_pin_suite()


@pytest.mark.parametrize("name", sorted(SSSP_MUTANTS))
def test_sssp_mutant_is_caught(name, swap_oracle):
    before, after = SSSP_MUTANTS[name]
    swap_oracle(_mutate(open(SRC).read(), before, after, ext=False))
    with pytest.raises(AssertionError):
        _sssp_pin_suite()


PR_MUTANTS = {
    "pr-signed-diff": ("diff = diff + fabs(val - pr[v]);", "diff = diff + (val - pr[v]);"),
    "pr-no-teleport": ("double val = (1.0 - damping) / (double)n + damping * sum;",
                       "double val = damping * sum;"),
    "pr-own-outdeg": ("sum = sum + pr[u] / (double)(row_ptr[u + 1] - row_ptr[u]);",
                      "sum = sum + pr[u] / (double)(row_ptr[v + 1] - row_ptr[v] + 1);"),
}


def _pr_pin_suite():
    for g in (gg.rmat(10, 8, seed=1), gg.rmat(10, 8, seed=2, directed=True)):
        pins.test_pagerank_converges_to_fixed_point(g)
    pins.test_pagerank_star_one_iteration()


def test_unmutated_copy_passes_pagerank_pins(swap_oracle):
    swap_oracle(open(SRC).read())
    _pr_pin_suite()


@pytest.mark.parametrize("name", sorted(PR_MUTANTS))
def test_pagerank_mutant_is_caught(name, swap_oracle):
    before, after = PR_MUTANTS[name]
    swap_oracle(_mutate(open(SRC).read(), before, after, ext=False))
    with pytest.raises(AssertionError):
        _pr_pin_suite()


def _ext_pin_suite():
    """The extended-range pins (quick ones) against the loaded library."""
    pins.test_ext_diamond_chain_closed_form(1100, 2)
    pins.test_ext_diamond_chain_closed_form(700, 3)
    pins.test_ext_lattice_sigma_binomial()
    pins.test_ext_matches_double_oracle_when_counts_fit()


def _mutate(text, before, after, ext):
    head, mark, tail = text.partition(EXT_MARK)
    assert mark, "extended-range section not found"
    part = tail if ext else head
    assert part.count(before) == 1, f"mutation site {before!r} not unique"
    part = part.replace(before, after)
    return head + mark + part if ext else part + mark + tail


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, swap_oracle):
    before, after = MUTANTS[name]
    swap_oracle(_mutate(open(SRC).read(), before, after, ext=False))
    with pytest.raises(AssertionError):
        _pin_suite()


def test_unmutated_copy_passes_extended_pins(swap_oracle):
    swap_oracle(open(SRC).read())
    _ext_pin_suite()


@pytest.mark.parametrize("name", sorted(EXT_MUTANTS))
def test_extended_mutant_is_caught(name, swap_oracle):
    before, after = EXT_MUTANTS[name]
    swap_oracle(_mutate(open(SRC).read(), before, after, ext=True))
    with pytest.raises(AssertionError):
        _ext_pin_suite()
