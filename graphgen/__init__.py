"""Seeded synthetic graph inputs, shared by the CPU oracle tests and the GPU path.

This module holds no centrality arithmetic.  It builds undirected, unweighted
int32 CSR graphs shaped like the paper's input suite (Section "Experimental
Evaluation", input-graph table): R-MAT with a=0.57, b=0.19, c=0.19, d=0.05, a
road-like grid (the stand-in for the large-diameter road networks), a uniform
random graph, and small closed-form families (path, star, cycle, ...) used to
pin the oracle.  Large generators run in ``libgraphgen.so`` (built from
``graphgen.c`` with gcc); every draw is counter-based, so results are identical
for any thread count.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build() -> str:
    """Compile libgraphgen.so with gcc (OpenMP, -O2)."""
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.gg_draw.restype = ctypes.c_uint64
    lib.gg_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    lib.gg_rmat_edges.restype = None
    lib.gg_rmat_edges.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_uint64, i32p, i32p]
    lib.gg_permutation.restype = None
    lib.gg_permutation.argtypes = [ctypes.c_int32, ctypes.c_uint64, i32p]
    lib.gg_relabel.restype = None
    lib.gg_relabel.argtypes = [ctypes.c_int64, i32p, i32p, i32p]
    lib.gg_uniform_edges.restype = None
    lib.gg_uniform_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, i32p, i32p]
    lib.gg_grid_edges.restype = ctypes.c_int64
    lib.gg_grid_edges.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int64,
                                  ctypes.c_uint64, i32p, i32p]
    lib.gg_csr_from_edges.restype = ctypes.c_int64
    lib.gg_csr_from_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, i32p, i32p]
    lib.gg_edge_weights.restype = None
    lib.gg_edge_weights.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_uint64, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int, i32p]
    lib.gg_sample_without_replacement.restype = None
    lib.gg_sample_without_replacement.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                                  i64p]
    _lib = lib
    return lib


def _p32(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


@dataclass
class CSR:
    """Undirected graph as int32 CSR: neighbours of v are col_idx[row_ptr[v]:row_ptr[v+1]]."""

    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    name: str = "graph"
    params: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def csr_from_edges(n: int, src, dst, symmetrize: bool = True, drop_loops: bool = True,
                   dedup: bool = True, name: str = "graph", params: dict | None = None) -> CSR:
    """Build a CSR from an edge list (arrays of endpoints)."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = int(src.shape[0])
    if m and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("edge endpoint out of range")
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    col = np.empty(max(1, 2 * m if symmetrize else m), dtype=np.int32)
    nnz = lib.gg_csr_from_edges(n, m, _p32(src), _p32(dst), int(symmetrize), int(drop_loops),
                                int(dedup), _p32(row_ptr), _p32(col))
    if nnz < 0:
        raise ValueError("arc count exceeds int32")
    col_idx = np.array(col[:nnz], dtype=np.int32, copy=True)
    return CSR(n, row_ptr, col_idx, name, dict(params or {}))


def draw(seed: int, stream: int, i: int) -> int:
    """Draw i of the counter-based generator's stream under a seed (64-bit)."""
    return int(_load().gg_draw(seed, stream, i))


def rmat(scale: int, edgefactor: int, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, relabel: bool = True, directed: bool = False) -> CSR:
    """R-MAT graph with 2**scale vertices and edgefactor*2**scale sampled edges;
    self-loops and duplicates removed, vertex ids randomly relabelled.  Undirected
    (symmetrised) unless `directed`, which keeps each sampled edge as one arc."""
    lib = _load()
    n = 1 << scale
    m = edgefactor * n
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    lib.gg_rmat_edges(scale, m, a, b, c, seed, _p32(src), _p32(dst))
    if relabel:
        perm = np.empty(n, dtype=np.int32)
        lib.gg_permutation(n, seed, _p32(perm))
        lib.gg_relabel(m, _p32(perm), _p32(src), _p32(dst))
    g = csr_from_edges(n, src, dst, symmetrize=not directed,
                       name=f"rmat-s{scale}-ef{edgefactor}" + ("-dir" if directed else ""),
                       params=dict(kind="rmat", scale=scale, edgefactor=edgefactor, a=a, b=b, c=c,
                                   seed=seed, relabel=relabel, directed=directed))
    return g


def erdos_renyi(n: int, avg_degree: int, seed: int = 4) -> CSR:
    """Uniform random graph G(n, m) with m = avg_degree*n/2 sampled edges (loops and
    duplicates removed)."""
    lib = _load()
    m = (avg_degree * n) // 2
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    lib.gg_uniform_edges(n, m, seed, _p32(src), _p32(dst))
    return csr_from_edges(n, src, dst, name=f"er-n{n}-d{avg_degree}",
                          params=dict(kind="er", n=n, avg_degree=avg_degree, seed=seed))


def grid_road(rows: int, cols: int, remove_frac: float = 0.05, shortcut_frac: float = 0.001,
              seed: int = 2) -> CSR:
    """Road-like grid: 4-neighbour rows x cols lattice with each edge removed with
    probability remove_frac, plus round(shortcut_frac * kept edges) uniform random
    long-range edges."""
    lib = _load()
    n = rows * cols
    cap = 2 * n + int(shortcut_frac * 2 * n) + 16
    src = np.empty(cap, dtype=np.int32)
    dst = np.empty(cap, dtype=np.int32)
    kept = lib.gg_grid_edges(rows, cols, remove_frac, 0, seed, _p32(src), _p32(dst))
    n_short = int(round(shortcut_frac * kept))
    total = lib.gg_grid_edges(rows, cols, remove_frac, n_short, seed, _p32(src), _p32(dst))
    return csr_from_edges(n, src[:total], dst[:total],
                          name=f"grid-{rows}x{cols}",
                          params=dict(kind="grid", rows=rows, cols=cols, remove_frac=remove_frac,
                                      shortcut_frac=shortcut_frac, shortcuts=n_short, seed=seed))


def edge_weights(g: CSR, seed: int, lo: int = 1, hi: int = 100) -> np.ndarray:
    """int32 weights in [lo, hi] for g's arcs (CSR order), uniform per edge: the two
    arcs of an undirected edge get the same weight; a directed graph's arcs are
    drawn independently."""
    lib = _load()
    w = np.empty(max(g.nnz, 1), dtype=np.int32)
    lib.gg_edge_weights(g.n, _p32(g.row_ptr), _p32(g.col_idx), seed, lo, hi,
                        0 if g.params.get("directed") else 1, _p32(w))
    return w[:g.nnz]


def sample_sources(g: CSR, k: int, seed: int, min_degree: int = 1) -> np.ndarray:
    """k distinct sources drawn uniformly without replacement from the vertices of
    degree >= min_degree (seeded)."""
    cand = np.nonzero(g.degrees() >= min_degree)[0].astype(np.int64)
    if k > cand.size:
        raise ValueError(f"asked for {k} sources but only {cand.size} candidates")
    out = np.empty(k, dtype=np.int64)
    _load().gg_sample_without_replacement(cand.size, k, seed,
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return cand[out].astype(np.int32)


# ---------------------------------------------------------------------------
# Small closed-form families (numpy edge lists).
# ---------------------------------------------------------------------------

def _from_pairs(n_vertices, pairs, name, **params) -> CSR:
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return csr_from_edges(n_vertices, pairs[:, 0], pairs[:, 1], name=name, params=params)


def path(n: int) -> CSR:
    return _from_pairs(n, [(i, i + 1) for i in range(n - 1)], f"path-{n}", kind="path", n=n)


def star(n: int) -> CSR:
    """Vertex 0 is the centre, 1..n-1 are leaves."""
    return _from_pairs(n, [(0, i) for i in range(1, n)], f"star-{n}", kind="star", n=n)


def cycle(n: int) -> CSR:
    return _from_pairs(n, [(i, (i + 1) % n) for i in range(n)], f"cycle-{n}", kind="cycle", n=n)


def complete(n: int) -> CSR:
    return _from_pairs(n, [(i, j) for i in range(n) for j in range(i + 1, n)], f"K{n}",
                       kind="complete", n=n)


def complete_bipartite(a: int, b: int) -> CSR:
    """Side A = 0..a-1, side B = a..a+b-1."""
    return _from_pairs(a + b, [(i, a + j) for i in range(a) for j in range(b)], f"K{a},{b}",
                       kind="complete_bipartite", a=a, b=b)


def hypercube(d: int) -> CSR:
    n = 1 << d
    pairs = [(v, v ^ (1 << i)) for v in range(n) for i in range(d) if v < v ^ (1 << i)]
    return _from_pairs(n, pairs, f"Q{d}", kind="hypercube", d=d)


def grid_full(rows: int, cols: int) -> CSR:
    """Complete 4-neighbour lattice, vertex id r*cols+c."""
    pairs = []
    for r in range(rows):
        for c in range(cols):
            v = r * cols + c
            if c + 1 < cols:
                pairs.append((v, v + 1))
            if r + 1 < rows:
                pairs.append((v, v + cols))
    return _from_pairs(rows * cols, pairs, f"lattice-{rows}x{cols}", kind="lattice",
                       rows=rows, cols=cols)


def diamond_chain(k: int, width: int = 2) -> CSR:
    """k diamonds in series: hub 0, `width` middle vertices joined to hub 0 and
    to hub 1, then the next diamond from hub 1, and so on.  Hub i
    has id i * (width + 1); the middles of diamond i (between hubs i-1 and
    i) are the ids just below hub i's."""
    step = width + 1
    pairs = []
    for i in range(k):
        a = i * step
        for j in range(1, width + 1):
            pairs.append((a, a + j))
            pairs.append((a + j, a + step))
    return _from_pairs(k * step + 1, pairs, f"diamonds-{k}x{width}", kind="diamond_chain",
                       k=k, width=width)


def torus(rows: int, cols: int) -> CSR:
    pairs = []
    for r in range(rows):
        for c in range(cols):
            v = r * cols + c
            pairs.append((v, r * cols + (c + 1) % cols))
            pairs.append((v, ((r + 1) % rows) * cols + c))
    return _from_pairs(rows * cols, pairs, f"torus-{rows}x{cols}", kind="torus",
                       rows=rows, cols=cols)


def random_tree(n: int, seed: int) -> CSR:
    """Random recursive tree: vertex i>0 attaches to a uniform earlier vertex (stream 11)."""
    pairs = [(i, draw(seed, 11, i) % i) for i in range(1, n)]
    return _from_pairs(n, pairs, f"tree-{n}", kind="tree", n=n, seed=seed)


def gnp(n: int, p: float, seed: int) -> CSR:
    """Erdos-Renyi G(n, p) for small n: each pair kept when its draw (stream 12) < p."""
    pairs = []
    idx = 0
    for i in range(n):
        for j in range(i + 1, n):
            if (draw(seed, 12, idx) >> 11) * 2.0 ** -53 < p:
                pairs.append((i, j))
            idx += 1
    return _from_pairs(n, pairs if pairs else np.zeros((0, 2)), f"gnp-{n}-{p}", kind="gnp",
                       n=n, p=p, seed=seed)


def gnp_directed(n: int, p: float, seed: int) -> CSR:
    """Directed G(n, p) for small n: each ordered pair (i, j), i != j, kept as arc
    i -> j when its draw (stream 13) < p."""
    u, v = [], []
    idx = 0
    for i in range(n):
        for j in range(n):
            if i != j:
                if (draw(seed, 13, idx) >> 11) * 2.0 ** -53 < p:
                    u.append(i)
                    v.append(j)
                idx += 1
    return csr_from_edges(n, np.array(u, np.int64), np.array(v, np.int64), symmetrize=False,
                          name=f"dgnp-{n}-{p}", params=dict(kind="gnp_directed", n=n, p=p,
                                                             seed=seed, directed=True))


def directed(n: int, pairs, name: str) -> CSR:
    """Directed graph from (u, v) arc pairs (duplicates and self-loops removed)."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return csr_from_edges(n, pairs[:, 0], pairs[:, 1], symmetrize=False, name=name,
                          params=dict(kind="directed", n=n, directed=True))


def from_adjacency_bits(n: int, bits: int) -> CSR:
    """Labelled simple graph on n vertices whose edge (i<j), enumerated row-major, is
    present when the corresponding bit of `bits` is set."""
    pairs = []
    idx = 0
    for i in range(n):
        for j in range(i + 1, n):
            if (bits >> idx) & 1:
                pairs.append((i, j))
            idx += 1
    return _from_pairs(n, pairs if pairs else np.zeros((0, 2)), f"bits-{n}-{bits}",
                       kind="bits", n=n, bits=bits)


# ---------------------------------------------------------------------------
# The benchmark workloads (synthetic stand-ins for the paper's input suite).
# ---------------------------------------------------------------------------

WORKLOADS = {
    # name: (builder, source count, source seed)
    "rmat-s12-ef8": (lambda: rmat(12, 8, seed=1), 4096, None),
    "grid-1024x1024": (lambda: grid_road(1024, 1024, 0.05, 0.001, seed=2), 64, 102),
    "rmat-s22-ef16": (lambda: rmat(22, 16, seed=3), 256, 103),
    "er-n8388608-d16": (lambda: erdos_renyi(1 << 23, 16, seed=4), 128, 104),
    # the road-like grid at full diameter (no shortcuts): ~1,700 levels, path
    # counts beyond double's range
    "grid-1024x1024-noshortcut": (lambda: grid_road(1024, 1024, 0.05, 0.0, seed=2), 64, 102),
    # directed R-MAT: each sampled edge kept as one arc (about half the arcs of
    # the undirected graph of the same size)
    "rmat-s22-ef16-dir": (lambda: rmat(22, 16, seed=3, directed=True), 256, 103),
}


def workload(name: str):
    """Return (graph, sources) for a named benchmark workload."""
    builder, k, sseed = WORKLOADS[name]
    g = builder()
    if sseed is None:
        src = np.arange(g.n, dtype=np.int32)[:k]
    else:
        src = sample_sources(g, k, sseed)
    return g, src
