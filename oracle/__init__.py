"""CPU oracle for Brandes betweenness centrality -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never imports, links or calls it, and
the two share no code.  The arithmetic lives in ``bc_oracle.c`` (plain C,
IEEE double, no fast-math), which follows the paper's BC specification
(Section "Background", the ComputeBC listing: forward sigma sums in BFS order,
backward dependency sums in reverse BFS order, BC += delta for v != src), i.e.
Brandes' algorithm for unweighted graphs.  Its readings of the listing are
stated at the top of that file.

Pins (tests/test_oracle_pins.py) tie it to facts fixed independently of it:
brute-force path counting on tiny graphs, closed forms for path, star, cycle,
tree, complete bipartite, complete and hypercube graphs, the distance-sum
invariant, additivity over sources, and NetworkX's betweenness.  The
extended-range functions (``*_ext``, long double) are pinned to closed forms on
chains of diamonds whose path counts pass double's range, to exact big-integer
counts on deep grids, and to the double oracle wherever counts fit double.
The directed entry points (``directed=True``) are pinned to closed forms on
directed paths, cycles and stars, brute force on random digraphs, NetworkX's
directed betweenness and the undirected oracle on symmetric graphs.  ``sssp``
(the paper's weighted single-source shortest paths) is pinned to scipy's
Dijkstra, to hop distances with unit weights and to prefix sums on paths.
``pagerank`` is pinned to the fixed point of its linear system (scipy's direct
solve), to uniform ranks on regular graphs, to a one-iteration closed form on
stars and to NetworkX's PageRank on graphs without dangling vertices.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libbc_oracle.so")
_lib = None

OK = 0
INVALID_ARG = 1
RANGE = 4


class OracleError(RuntimeError):
    pass


def build() -> str:
    """Compile libbc_oracle.so with gcc -O2 (OpenMP over sources; no fast-math)."""
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-march=native", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", _SRC, "-o", tmp, "-lm"]
    try:
        subprocess.run(cmd, check=True)
    except subprocess.CalledProcessError:
        cmd.remove("-march=native")
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
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.oracle_single_source.restype = ctypes.c_int
    lib.oracle_single_source.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, i32p, f64p,
                                         f64p]
    lib.oracle_bc.restype = ctypes.c_int
    lib.oracle_bc.argtypes = [ctypes.c_int32, i32p, i32p, i32p, ctypes.c_int32, ctypes.c_int,
                              f64p]
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_max_threads.argtypes = []
    lib.oracle_single_source_directed.restype = ctypes.c_int
    lib.oracle_single_source_directed.argtypes = lib.oracle_single_source.argtypes
    lib.oracle_bc_directed.restype = ctypes.c_int
    lib.oracle_bc_directed.argtypes = lib.oracle_bc.argtypes
    lib.oracle_sssp.restype = ctypes.c_int64
    lib.oracle_sssp.argtypes = [ctypes.c_int32, i32p, i32p, i32p, ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_pagerank.restype = ctypes.c_int64
    lib.oracle_pagerank.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int32, f64p, f64p]
    lib.oracle_ld_digits.restype = ctypes.c_int
    lib.oracle_ld_digits.argtypes = []
    lib.oracle_single_source_ext.restype = ctypes.c_int
    lib.oracle_single_source_ext.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, i32p,
                                             f64p, i32p, f64p]
    lib.oracle_bc_ext.restype = ctypes.c_int
    lib.oracle_bc_ext.argtypes = [ctypes.c_int32, i32p, i32p, i32p, ctypes.c_int32, ctypes.c_int,
                                  f64p]
    _lib = lib
    return lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def single_source(row_ptr, col_idx, s: int, with_delta: bool = True, directed: bool = False):
    """(dist int32[n], sigma float64[n], delta float64[n] or None, status) from source s
    (directed: the CSR lists out-arcs)."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    ci, cip = _i32(col_idx)
    n = rp.shape[0] - 1
    dist = np.empty(n, dtype=np.int32)
    sigma = np.empty(n, dtype=np.float64)
    delta = np.empty(n, dtype=np.float64) if with_delta else None
    fn = lib.oracle_single_source_directed if directed else lib.oracle_single_source
    st = fn(n, rpp, cip, int(s), dist.ctypes.data_as(ctypes.POINTER(
        ctypes.c_int32)), sigma.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        delta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if with_delta else None)
    if st == INVALID_ARG:
        raise OracleError("invalid argument")
    return dist, sigma, delta, st


def bc(row_ptr, col_idx, sources, threads: int = 0, directed: bool = False):
    """(BC float64[n], status): raw Brandes sum over `sources` (ordered pairs, no scaling;
    directed: the CSR lists out-arcs)."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    ci, cip = _i32(col_idx)
    src, srcp = _i32(sources)
    n = rp.shape[0] - 1
    out = np.empty(n, dtype=np.float64)
    fn = lib.oracle_bc_directed if directed else lib.oracle_bc
    st = fn(n, rpp, cip, srcp if src.size else None, int(src.size), int(threads),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if st == INVALID_ARG:
        raise OracleError("invalid argument")
    return out, st


def long_double_digits() -> int:
    """Significand bits of the C long double the extended oracle computes in."""
    return int(_load().oracle_ld_digits())


def single_source_ext(row_ptr, col_idx, s: int, with_delta: bool = True):
    """Extended range: (dist int32[n], sig_m float64[n], sig_e int32[n], delta float64[n] or
    None, status), sigma = sig_m * 2**sig_e, computed in long double."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    ci, cip = _i32(col_idx)
    n = rp.shape[0] - 1
    dist = np.empty(n, dtype=np.int32)
    sig_m = np.empty(n, dtype=np.float64)
    sig_e = np.empty(n, dtype=np.int32)
    delta = np.empty(n, dtype=np.float64) if with_delta else None
    i32 = ctypes.POINTER(ctypes.c_int32)
    f64 = ctypes.POINTER(ctypes.c_double)
    st = lib.oracle_single_source_ext(n, rpp, cip, int(s), dist.ctypes.data_as(i32),
                                      sig_m.ctypes.data_as(f64), sig_e.ctypes.data_as(i32),
                                      delta.ctypes.data_as(f64) if with_delta else None)
    if st == INVALID_ARG:
        raise OracleError("invalid argument")
    return dist, sig_m, sig_e, delta, st


def bc_ext(row_ptr, col_idx, sources, threads: int = 0):
    """Extended range: (BC float64[n], status), the Brandes sum computed in long double."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    ci, cip = _i32(col_idx)
    src, srcp = _i32(sources)
    n = rp.shape[0] - 1
    out = np.empty(n, dtype=np.float64)
    st = lib.oracle_bc_ext(n, rpp, cip, srcp if src.size else None, int(src.size), int(threads),
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if st == INVALID_ARG:
        raise OracleError("invalid argument")
    return out, st


def sssp(row_ptr, col_idx, weight, s: int):
    """(dist int64[n] with -1 where unreachable, passes): the paper's fixed-point
    SSSP from s over weighted out-arcs (weight[e] for arc e, non-negative)."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    ci, cip = _i32(col_idx)
    w, wp = _i32(weight)
    n = rp.shape[0] - 1
    dist = np.empty(n, dtype=np.int64)
    passes = lib.oracle_sssp(n, rpp, cip, wp if w.size else None, int(s),
                             dist.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if passes < 0:
        raise OracleError("invalid argument")
    return dist, int(passes)


def pagerank(row_ptr, col_idx, damping: float = 0.85, tol: float = 1e-10, max_iter: int = 100):
    """(pr float64[n], iterations, last L1 change): the paper's PageRank (pull over
    in-arcs, start 1/n, stop when the L1 change <= tol or after max_iter)."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    ci, cip = _i32(col_idx)
    n = rp.shape[0] - 1
    pr = np.empty(n, dtype=np.float64)
    last = ctypes.c_double(0.0)
    it = lib.oracle_pagerank(n, rpp, cip, float(damping), float(tol), int(max_iter),
                             pr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(last))
    if it < 0:
        raise OracleError("invalid argument")
    return pr, int(it), float(last.value)
