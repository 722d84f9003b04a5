"""Plant plausible slips in a copy of the oracle and check that the pins catch them.

Each mutant is a textual edit of oracle/bc_oracle.c compiled into a temporary
library; the committed oracle is never touched.  A mutant survives only if no
pin in tests/test_oracle_pins.py notices it, which would mean the pins leave
that part of the oracle unchecked.
"""
import os
import subprocess

import numpy as np
import pytest

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


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, swap_oracle):
    before, after = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(before) == 1, f"mutation site for {name} not unique"
    swap_oracle(text.replace(before, after))
    with pytest.raises(AssertionError):
        _pin_suite()
