"""Brandes betweenness centrality on MI355X (gfx950): Python binding.

Thin wrappers with the names of the C ABI in include/bc.h.  They only marshal
arguments (numpy arrays for host memory, torch tensors for device memory and
torch streams for ordering); every step of the computation runs in the HIP
kernels of libbc_mi355x.so.  The library must be present (or buildable with
hipcc): there is no CPU fallback.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _capi
from ._capi import (BC_ERR_DEVICE, BC_ERR_INVALID_ARG, BC_ERR_INVALID_GRAPH,  # noqa: F401
                    BC_ERR_OUT_OF_MEMORY, BC_ERR_RANGE, BC_ERR_TOO_LARGE, BC_ERR_UNSUPPORTED,
                    BC_NOALLOC_SCRATCH_BYTES,
                    BC_GRAPH_DIRECTED, BC_GRAPH_INPUT_ON_DEVICE, BC_GRAPH_TRUST_SYMMETRIC,
                    BC_MODE_AUTO,
                    BC_MODE_BATCHED, BC_MODE_PLAIN, BC_OK, bc_options,
                    BC_LOOP_AUTO, BC_LOOP_HOST, BC_LOOP_DEVICE, BC_LOOP_GRAPH)

__all__ = [
    "BCError", "bc_create_graph", "bc_destroy_graph", "bc_graph_info", "bc_run", "bc_run_async",
    "bc_run_async_noalloc",
    "bc_run_multi", "bc_run_graphs",
    "bc_single_source", "bc_run_detail", "bc_workspace_bytes", "bc_trim_workspaces",
    "bc_workspace_held", "bc_autotune", "bc_set_work_items",
    "bc_profile_enable", "bc_profile_read", "bc_set_weights", "bc_sssp", "bc_pagerank",
    "bc_status_str",
    "make_options", "Graph",
    "load_library",
]


class BCError(RuntimeError):
    """A C-ABI call returned a status other than BC_OK.  `result` holds the
    outputs when the call still wrote them (BC_ERR_RANGE)."""

    def __init__(self, status: int, where: str, result=None):
        super().__init__(f"{where}: {bc_status_str(status)} (status {status})")
        self.status = status
        self.result = result


def load_library():
    return _capi.load()


def bc_status_str(status: int) -> str:
    return _capi.load().bc_status_str(int(status)).decode()


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.int32)


def _device_tensor(t, dtype: str, where: str):
    """Checks that `t` is a contiguous torch tensor of `dtype` ("float64" or
    "int32") in device memory: the library reads or writes it through its
    raw pointer, so a wrong element size or a host buffer would be accessed
    out of bounds on the device."""
    import torch
    want = {"float64": torch.float64, "int32": torch.int32}[dtype]
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{where}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != want:
        raise TypeError(f"{where}: expected a {want} tensor, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{where}: the tensor must be contiguous")
    if not t.is_cuda:
        raise ValueError(f"{where}: the tensor must be in device memory")
    return t


def _fits(t, n: int, where: str):
    """Checks that the device tensor `t` holds at least n entries; returns its pointer."""
    if t.numel() < n:
        raise ValueError(f"{where}: the tensor holds {t.numel()} entries, {n} are written")
    return ctypes.c_void_p(t.data_ptr())


def _graph_n(g) -> int:
    return bc_graph_info(g)[0]


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def make_options(mode: int = BC_MODE_AUTO, batch_width: int = 0, level_chunk: int = 0,
                 sparse_div: int = 0, concurrency: int = 0, level_loop: int = 0):
    o = bc_options()
    o.mode, o.batch_width, o.level_chunk = int(mode), int(batch_width), int(level_chunk)
    o.sparse_div, o.concurrency, o.level_loop = int(sparse_div), int(concurrency), int(level_loop)
    return o


def _check(st: int, where: str, result=None):
    if st != BC_OK:
        raise BCError(st, where, result)


def bc_create_graph(n: int, row_ptr, col_idx, flags: int = 0, stream=None) -> int:
    """Copy a symmetric int32 CSR to the device; returns an opaque handle.

    Host numpy arrays, or device torch tensors together with
    BC_GRAPH_INPUT_ON_DEVICE in `flags`."""
    lib = _capi.load()
    out = ctypes.c_void_p()
    if flags & BC_GRAPH_INPUT_ON_DEVICE:
        _device_tensor(row_ptr, "int32", "bc_create_graph row_ptr")
        _device_tensor(col_idx, "int32", "bc_create_graph col_idx")
        if n >= 0:
            _fits(row_ptr, n + 1, "bc_create_graph row_ptr")
            import torch
            torch.cuda.synchronize(row_ptr.device)
            _fits(col_idx, max(int(row_ptr[n].item()), 0), "bc_create_graph col_idx")
        rp_p, ci_p = ctypes.c_void_p(row_ptr.data_ptr()), ctypes.c_void_p(col_idx.data_ptr())
        keep = None
        st_h = _stream_handle(stream)
    else:
        rp, ci = _i32(row_ptr), _i32(col_idx)
        # the library reads n + 1 offsets and row_ptr[n] column ids
        if n >= 0 and rp.size < n + 1:
            raise ValueError(f"bc_create_graph: row_ptr holds {rp.size} offsets, {n + 1} needed")
        if n >= 0 and ci.size < max(int(rp[n]), 0):
            raise ValueError(f"bc_create_graph: col_idx holds {ci.size} ids, row_ptr[n] = {int(rp[n])}")
        keep = (rp, ci)
        rp_p, ci_p = ctypes.c_void_p(rp.ctypes.data), ctypes.c_void_p(ci.ctypes.data)
        st_h = ctypes.c_void_p(0) if stream is None else _stream_handle(stream)
    st = lib.bc_create_graph(int(n), rp_p, ci_p, int(flags), st_h, ctypes.byref(out))
    del keep
    _check(st, "bc_create_graph")
    return out.value


def bc_destroy_graph(g: int) -> None:
    _check(_capi.load().bc_destroy_graph(ctypes.c_void_p(g)), "bc_destroy_graph")


def bc_graph_info(g: int):
    n, nnz, b = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_size_t()
    _check(_capi.load().bc_graph_info(ctypes.c_void_p(g), ctypes.byref(n), ctypes.byref(nnz),
                                      ctypes.byref(b)), "bc_graph_info")
    return n.value, nnz.value, b.value


def bc_run(g: int, sources) -> np.ndarray:
    """BC over the source multiset (host in, host out)."""
    n, _, _ = bc_graph_info(g)
    src = _i32(sources)
    out = np.empty(max(n, 0), dtype=np.float64)
    st = _capi.load().bc_run(ctypes.c_void_p(g), _ptr(src, ctypes.c_int32), int(src.size),
                             _ptr(out, ctypes.c_double))
    _check(st, "bc_run", out)
    return out


def bc_run_async(g: int, sources, bc_out, options=None, stream=None) -> None:
    """BC into `bc_out` (a float64 device tensor of n entries), ordered on `stream`
    (default: torch's current stream)."""
    src = _i32(sources)
    _device_tensor(bc_out, "float64", "bc_run_async bc_out")
    out_p = _fits(bc_out, _graph_n(g), "bc_run_async bc_out")
    opt = ctypes.byref(options) if options is not None else None
    st = _capi.load().bc_run_async(ctypes.c_void_p(g), _ptr(src, ctypes.c_int32), int(src.size),
                                   out_p, opt, _stream_handle(stream))
    _check(st, "bc_run_async", bc_out)


def bc_run_async_noalloc(g: int, sources, bc_out, stream=None) -> None:
    """bc_run_async without any allocation: the run's device buffers come from
    the library's fixed per-device array (BC_NOALLOC_SCRATCH_BYTES)."""
    src = _i32(sources)
    _device_tensor(bc_out, "float64", "bc_run_async_noalloc bc_out")
    out_p = _fits(bc_out, _graph_n(g), "bc_run_async_noalloc bc_out")
    st = _capi.load().bc_run_async_noalloc(ctypes.c_void_p(g), _ptr(src, ctypes.c_int32),
                                           int(src.size), out_p, _stream_handle(stream))
    _check(st, "bc_run_async_noalloc", bc_out)


def bc_run_multi(g: int, requests, outs, stream=None) -> None:
    """Several requests (a list of source arrays) in one call; outs[r] is a float64
    device tensor of n entries that receives request r's BC."""
    srcs = [_i32(r) for r in requests]
    if len(outs) != len(srcs):
        raise ValueError("bc_run_multi: requests and outs differ in length")
    for o in outs:
        _device_tensor(o, "float64", "bc_run_multi outs")
    n = _graph_n(g) if outs else 0
    ptrs = (ctypes.c_void_p * max(len(srcs), 1))(*[_fits(o, n, "bc_run_multi outs")
                                                   for o in outs])
    start = np.zeros(len(srcs) + 1, dtype=np.int32)
    start[1:] = np.cumsum([s.size for s in srcs])
    flat = np.concatenate(srcs) if srcs else np.zeros(0, np.int32)
    flat = np.ascontiguousarray(flat, dtype=np.int32)
    st = _capi.load().bc_run_multi(ctypes.c_void_p(g), _ptr(flat, ctypes.c_int32),
                                   _ptr(start, ctypes.c_int32), len(srcs), ptrs,
                                   _stream_handle(stream))
    _check(st, "bc_run_multi", outs)


def bc_run_graphs(graphs, sources, outs, level_loop: int = BC_LOOP_AUTO, stream=None) -> list:
    """BC of several graphs in one call (the batches of the graphs that join in
    one device-resident launch): graphs are Graph objects or handles,
    sources[i] the source array of graph i, outs[i] a float64 device tensor of
    n_i entries.  Returns the loop each graph ran on (BC_LOOP_DEVICE or
    BC_LOOP_HOST)."""
    handles = [g.handle if isinstance(g, Graph) else int(g) for g in graphs]
    srcs = [_i32(s) for s in sources]
    if not (len(handles) == len(srcs) == len(outs)):
        raise ValueError("graphs, sources and outs differ in length")
    for o in outs:
        _device_tensor(o, "float64", "bc_run_graphs outs")
    m = max(len(handles), 1)
    h_arr = (ctypes.c_void_p * m)(*handles)
    s_arr = (ctypes.c_void_p * m)(*[s.ctypes.data if s.size else None for s in srcs])
    ks = np.ascontiguousarray([s.size for s in srcs] or [0], dtype=np.int32)
    o_arr = (ctypes.c_void_p * m)(*[_fits(o, _graph_n(h), "bc_run_graphs outs")
                                    for h, o in zip(handles, outs)])
    loops = np.zeros(m, dtype=np.int32)
    st = _capi.load().bc_run_graphs(h_arr, len(handles), s_arr, _ptr(ks, ctypes.c_int32), o_arr,
                                    int(level_loop), _ptr(loops, ctypes.c_int32),
                                    _stream_handle(stream))
    _check(st, "bc_run_graphs", outs)
    return [int(x) for x in loops[:len(handles)]]


def bc_set_weights(g: int, weight) -> None:
    """Arc weights for SSSP (int32 >= 0, in the order of the graph's col_idx)."""
    w = _i32(weight)
    nnz = bc_graph_info(g)[1]
    if w.size != nnz:  # the library reads one weight per arc
        raise ValueError(f"bc_set_weights: {w.size} weights for {nnz} arcs")
    _check(_capi.load().bc_set_weights(ctypes.c_void_p(g), _ptr(w, ctypes.c_int32)),
           "bc_set_weights")


def bc_sssp(g: int, source: int, dist_out, stream=None) -> None:
    """Shortest-path distances from `source` into dist_out (int32 device tensor of
    n entries; -1 where unreachable)."""
    _device_tensor(dist_out, "int32", "bc_sssp dist_out")
    out_p = _fits(dist_out, _graph_n(g), "bc_sssp dist_out")
    st = _capi.load().bc_sssp(ctypes.c_void_p(g), int(source), out_p, _stream_handle(stream))
    _check(st, "bc_sssp", dist_out)


def bc_pagerank(g: int, pr_out, damping: float = 0.85, tol: float = 1e-10, max_iter: int = 100,
                stream=None) -> int:
    """PageRank into pr_out (float64 device tensor of n entries); returns the
    iterations run."""
    _device_tensor(pr_out, "float64", "bc_pagerank pr_out")
    out_p = _fits(pr_out, _graph_n(g), "bc_pagerank pr_out")
    it = ctypes.c_int32(0)
    st = _capi.load().bc_pagerank(ctypes.c_void_p(g), float(damping), float(tol), int(max_iter),
                                  out_p, ctypes.byref(it), _stream_handle(stream))
    _check(st, "bc_pagerank", pr_out)
    return int(it.value)


def bc_single_source(g: int, s: int):
    """(dist int32[n], sigma float64[n], delta float64[n]) for one source."""
    n, _, _ = bc_graph_info(g)
    dist = np.empty(n, dtype=np.int32)
    sigma = np.empty(n, dtype=np.float64)
    delta = np.empty(n, dtype=np.float64)
    st = _capi.load().bc_single_source(ctypes.c_void_p(g), int(s), _ptr(dist, ctypes.c_int32),
                                       _ptr(sigma, ctypes.c_double),
                                       _ptr(delta, ctypes.c_double))
    _check(st, "bc_single_source", (dist, sigma, delta))
    return dist, sigma, delta


def bc_run_detail(g: int, sources, options=None, want_dist: bool = True,
                  want_sigma: bool = True):
    """(bc[n], dist[k][n] or None, sigma[k][n] or None) from the path `options` selects."""
    n, _, _ = bc_graph_info(g)
    src = _i32(sources)
    k = int(src.size)
    bc = np.empty(n, dtype=np.float64)
    dist = np.empty((k, n), dtype=np.int32) if want_dist else None
    sigma = np.empty((k, n), dtype=np.float64) if want_sigma else None
    opt = ctypes.byref(options) if options is not None else None
    st = _capi.load().bc_run_detail(ctypes.c_void_p(g), _ptr(src, ctypes.c_int32), k, opt,
                                    _ptr(bc, ctypes.c_double),
                                    _ptr(dist, ctypes.c_int32) if want_dist else None,
                                    _ptr(sigma, ctypes.c_double) if want_sigma else None)
    _check(st, "bc_run_detail", (bc, dist, sigma))
    return bc, dist, sigma


def bc_autotune(g: int, sources, stream=None) -> dict:
    """Time the library's execution settings on a sample of `sources` and keep
    the fastest for BC_MODE_AUTO on this graph; returns the choice."""
    src = _i32(sources)
    t = _capi.bc_tuning()
    _check(_capi.load().bc_autotune(ctypes.c_void_p(g), _ptr(src, ctypes.c_int32), int(src.size),
                                    _stream_handle(stream), ctypes.byref(t)), "bc_autotune")
    return {"batch_width": t.batch_width, "sparse_div": t.sparse_div,
            "min_batched": t.min_batched, "sample": t.sample,
            "plain_ms_per_source": t.plain_ms_per_source, "batch_ms": t.batch_ms,
            "cached": bool(t.cached), "group_cut": t.group_cut, "chunk": t.chunk}


def bc_set_work_items(g: int, group_cut: int, chunk: int) -> None:
    """Degree thresholds of the batched path's work items (defaults 64, 512)."""
    _check(_capi.load().bc_set_work_items(ctypes.c_void_p(g), int(group_cut), int(chunk)),
           "bc_set_work_items")


def bc_workspace_bytes(g: int, k: int, options=None) -> int:
    out = ctypes.c_size_t()
    opt = ctypes.byref(options) if options is not None else None
    _check(_capi.load().bc_workspace_bytes(ctypes.c_void_p(g), int(k), opt, ctypes.byref(out)),
           "bc_workspace_bytes")
    return out.value


def bc_trim_workspaces(g: int) -> None:
    _check(_capi.load().bc_trim_workspaces(ctypes.c_void_p(g)), "bc_trim_workspaces")


def bc_workspace_held(g: int) -> int:
    """Device bytes the graph's BC workspace pools hold now."""
    out = ctypes.c_size_t()
    _check(_capi.load().bc_workspace_held(ctypes.c_void_p(g), ctypes.byref(out)),
           "bc_workspace_held")
    return out.value


def bc_profile_enable(g: int, on=True) -> None:
    """Measurement off (False / 0) or on (True / 1, or a sampling period P > 1)."""
    _check(_capi.load().bc_profile_enable(ctypes.c_void_p(g), int(on)), "bc_profile_enable")


def bc_profile_read(g: int, reset: bool = False) -> dict:
    """Accumulated per-kernel-class timing and work counters of profiled runs."""
    p = _capi.bc_profile()
    _check(_capi.load().bc_profile_read(ctypes.c_void_p(g), ctypes.byref(p), int(bool(reset))),
           "bc_profile_read")
    out = {"runs": int(p.runs), "levels": int(p.levels)}
    for i, name in enumerate(_capi.PROF_CLASS_NAMES):
        out[name] = {"launches": int(p.launches[i]), "ms": float(p.ms[i]),
                     "owners": int(p.owners[i]), "arcs": int(p.arcs[i]), "hits": int(p.hits[i]),
                     "vertices": int(p.vertices[i])}
    return out


class Graph:
    """Owning wrapper of a bc_graph_t handle."""

    def __init__(self, n: int, row_ptr, col_idx, flags: int = 0, stream=None):
        self.handle = bc_create_graph(n, row_ptr, col_idx, flags, stream)
        self.n, self.nnz, self.device_bytes = bc_graph_info(self.handle)

    def close(self):
        if self.handle:
            bc_destroy_graph(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, sources) -> np.ndarray:
        return bc_run(self.handle, sources)

    def run_async(self, sources, bc_out, options=None, stream=None) -> None:
        bc_run_async(self.handle, sources, bc_out, options, stream)

    def run_async_noalloc(self, sources, bc_out, stream=None) -> None:
        bc_run_async_noalloc(self.handle, sources, bc_out, stream)

    def single_source(self, s: int):
        return bc_single_source(self.handle, s)

    def run_multi(self, requests, outs, stream=None) -> None:
        bc_run_multi(self.handle, requests, outs, stream)

    def run_detail(self, sources, options=None, want_dist=True, want_sigma=True):
        return bc_run_detail(self.handle, sources, options, want_dist, want_sigma)

    def autotune(self, sources, stream=None) -> dict:
        return bc_autotune(self.handle, sources, stream)

    def workspace_bytes(self, k: int, options=None) -> int:
        return bc_workspace_bytes(self.handle, k, options)

    def set_work_items(self, group_cut: int, chunk: int) -> None:
        bc_set_work_items(self.handle, group_cut, chunk)

    def workspace_held(self) -> int:
        return bc_workspace_held(self.handle)

    def trim_workspaces(self) -> None:
        bc_trim_workspaces(self.handle)

    def profile_enable(self, on=True) -> None:
        bc_profile_enable(self.handle, on)

    def profile_read(self, reset: bool = False) -> dict:
        return bc_profile_read(self.handle, reset)

    def pagerank(self, damping: float = 0.85, tol: float = 1e-10, max_iter: int = 100,
                 pr_out=None, stream=None):
        """(ranks as a float64 device tensor, iterations run)."""
        if pr_out is None:
            import torch
            pr_out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        it = bc_pagerank(self.handle, pr_out, damping, tol, max_iter, stream)
        return pr_out, it

    def set_weights(self, weight) -> None:
        bc_set_weights(self.handle, weight)

    def sssp(self, source: int, dist_out=None, stream=None):
        """Distances from `source` (int32 device tensor; allocated when not given)."""
        if dist_out is None:
            import torch
            dist_out = torch.empty(self.n, dtype=torch.int32, device="cuda")
        bc_sssp(self.handle, source, dist_out, stream)
        return dist_out
