"""Independent betweenness computations used to pin the oracle (test code only).

Nothing here follows Brandes' recurrences.  Distances and shortest-path counts
come from walk counting: in a graph, every walk of length d(s,t) from s to t is
a shortest path, so sigma_st is the (s,t) entry of A**d(s,t), where A is the
adjacency matrix with arc multiplicities.  Betweenness then follows from its
definition, BC(v) = sum over s != v != t != s of sigma_sv*sigma_vt/sigma_st
when d(s,v) + d(v,t) = d(s,t).
"""
from __future__ import annotations

import numpy as np


def adjacency(row_ptr, col_idx) -> np.ndarray:
    """Dense arc-multiplicity matrix A[u, v] = number of arcs u->v."""
    n = len(row_ptr) - 1
    A = np.zeros((n, n), dtype=np.int64)
    for u in range(n):
        for e in range(row_ptr[u], row_ptr[u + 1]):
            A[u, col_idx[e]] += 1
    return A


def walk_dist_sigma(A: np.ndarray):
    """All-pairs (dist, sigma) from walk counts; A may be batched [..., n, n].

    dist = -1 when t is unreachable from s; sigma counts shortest paths (exact
    in int64 for the small graphs used here)."""
    A = np.asarray(A, dtype=np.int64)
    n = A.shape[-1]
    dist = np.full(A.shape, -1, dtype=np.int64)
    sigma = np.zeros(A.shape, dtype=np.int64)
    W = np.broadcast_to(np.eye(n, dtype=np.int64), A.shape).copy()
    for k in range(n):
        newly = (W > 0) & (dist < 0)
        dist[newly] = k
        sigma[newly] = W[newly]
        W = W @ A
    return dist, sigma


def bc_by_definition(A: np.ndarray, sources=None) -> np.ndarray:
    """BC_S(v) from the definition (ordered pairs, sources as a multiset).

    A may be batched [G, n, n]; returns [G, n] (or [n])."""
    A = np.asarray(A, dtype=np.int64)
    batched = A.ndim == 3
    if not batched:
        A = A[None]
    G, n, _ = A.shape
    dist, sigma = walk_dist_sigma(A)
    if sources is None:
        weight = np.ones(n)
    else:
        weight = np.bincount(np.asarray(sources, dtype=np.int64), minlength=n).astype(np.float64)
    # index order [g, s, v, t]
    d_sv = dist[:, :, :, None]
    d_vt = dist[:, None, :, :]
    d_st = dist[:, :, None, :]
    on_path = (d_sv >= 0) & (d_vt >= 0) & (d_st >= 0) & (d_sv + d_vt == d_st)
    s_idx = np.arange(n)[:, None, None]
    v_idx = np.arange(n)[None, :, None]
    t_idx = np.arange(n)[None, None, :]
    distinct = (s_idx != v_idx) & (v_idx != t_idx) & (s_idx != t_idx)
    on_path &= distinct[None]
    num = sigma[:, :, :, None].astype(np.float64) * sigma[:, None, :, :].astype(np.float64)
    den = np.where(on_path, sigma[:, :, None, :], 1).astype(np.float64)
    contrib = np.where(on_path, num / den, 0.0)
    bc = np.einsum("gsvt,s->gv", contrib, weight)
    return bc if batched else bc[0]


def csr_from_adjacency(A: np.ndarray):
    """CSR arrays (row_ptr, col_idx) from a multiplicity matrix, neighbours ascending."""
    n = A.shape[0]
    deg = A.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(deg)
    cols = []
    for u in range(n):
        for v in range(n):
            cols.extend([v] * int(A[u, v]))
    return row_ptr, np.asarray(cols, dtype=np.int32)


def parse_golden(path: str):
    """Parse tests/golden/hand_worked.txt into a list of case dicts."""
    cases = []
    cur = None
    with open(path) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            key, *rest = line.split()
            if key == "case":
                cur = {"name": rest[0], "dist": {}, "sigma": {}}
                cases.append(cur)
            elif key == "n":
                cur["n"] = int(rest[0])
            elif key == "edges":
                cur["edges"] = [tuple(int(x) for x in e.split("-")) for e in rest]
            elif key == "sources":
                cur["sources"] = None if rest == ["all"] else [int(x) for x in rest]
            elif key == "bc":
                cur["bc"] = [float(x) for x in rest]
            elif key == "dist":
                cur["dist"][int(rest[0])] = [int(x) for x in rest[1:]]
            elif key == "sigma":
                cur["sigma"][int(rest[0])] = [float(x) for x in rest[1:]]
    return cases
