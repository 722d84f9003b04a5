"""Host-side checks of the C-ABI library (no GPU needed).

The library must load and export every function include/bc.h declares; the
argument and graph checks that run before any device call return the
documented status codes.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2401_02472_amd as bcm
from paper_2401_02472_amd import _capi

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "bc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_surface():
    assert declared_functions() == sorted(_capi.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = _capi.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    assert bcm.bc_status_str(bcm.BC_OK) == "ok"
    assert "range" in bcm.bc_status_str(bcm.BC_ERR_RANGE)
    assert bcm.bc_status_str(99) == "unknown status"


def _create(n, rp, ci, flags=0):
    lib = _capi.load()
    out = ctypes.c_void_p()
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    st = lib.bc_create_graph(n, ctypes.c_void_p(rp.ctypes.data), ctypes.c_void_p(ci.ctypes.data),
                             flags, None, ctypes.byref(out))
    return st, out


@pytest.mark.parametrize("rp,ci", [
    ([1, 1, 2], [0, 1]),            # row_ptr[0] != 0
    ([0, 2, 1], [1, 0]),            # decreasing offsets
    ([0, 1, 2], [1, 2]),            # neighbour out of range
    ([0, 1, 1], [1]),               # arc 0->1 without 1->0
    ([0, 2, 3], [1, 1, 0]),         # parallel arcs one way only
])
def test_invalid_graphs_rejected(rp, ci):
    st, _ = _create(2, rp, ci)
    assert st == bcm.BC_ERR_INVALID_GRAPH


def test_invalid_arguments_rejected():
    lib = _capi.load()
    rp = np.array([0, 1, 2], dtype=np.int32)
    ci = np.array([1, 0], dtype=np.int32)
    assert lib.bc_create_graph(2, ctypes.c_void_p(rp.ctypes.data),
                               ctypes.c_void_p(ci.ctypes.data), 0, None, None) == \
        bcm.BC_ERR_INVALID_ARG
    out = ctypes.c_void_p()
    assert lib.bc_create_graph(-1, ctypes.c_void_p(rp.ctypes.data),
                               ctypes.c_void_p(ci.ctypes.data), 0, None, ctypes.byref(out)) == \
        bcm.BC_ERR_INVALID_ARG
    assert lib.bc_create_graph(2, ctypes.c_void_p(rp.ctypes.data),
                               ctypes.c_void_p(ci.ctypes.data), 1 << 7, None,
                               ctypes.byref(out)) == bcm.BC_ERR_INVALID_ARG
    assert lib.bc_run(None, None, 0, None) == bcm.BC_ERR_INVALID_ARG
    assert lib.bc_graph_info(None, None, None, None) == bcm.BC_ERR_INVALID_ARG
    assert lib.bc_autotune(None, None, 1, None, None) == bcm.BC_ERR_INVALID_ARG
    assert lib.bc_set_work_items(None, 64, 512) == bcm.BC_ERR_INVALID_ARG
    assert lib.bc_set_weights(None, None) == bcm.BC_ERR_INVALID_ARG
    assert lib.bc_sssp(None, 0, None, None) == bcm.BC_ERR_INVALID_ARG
    assert lib.bc_pagerank(None, 0.85, 0.0, 10, None, None, None) == bcm.BC_ERR_INVALID_ARG
    # several graphs: a negative count, NULL arrays, a NULL graph, another loop
    assert lib.bc_run_graphs(None, -1, None, None, None, 0, None, None) == bcm.BC_ERR_INVALID_ARG
    assert lib.bc_run_graphs(None, 1, None, None, None, 0, None, None) == bcm.BC_ERR_INVALID_ARG
    one = (ctypes.c_void_p * 1)(None)
    k = np.zeros(1, np.int32)
    assert lib.bc_run_graphs(one, 1, one, k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), one,
                             0, None, None) == bcm.BC_ERR_INVALID_ARG
    assert lib.bc_run_graphs(None, 0, None, None, None, bcm.BC_LOOP_GRAPH, None, None) == \
        bcm.BC_ERR_INVALID_ARG
    assert lib.bc_run_graphs(None, 0, None, None, None, 0, None, None) == bcm.BC_OK
    assert lib.bc_destroy_graph(None) == bcm.BC_OK


def test_options_layout_matches_header():
    # eight int32 fields: mode, batch_width, level_chunk, sparse_div, concurrency,
    # level_loop, reserved[2]
    assert ctypes.sizeof(_capi.bc_options) == 32
    assert [f[0] for f in _capi.bc_options._fields_] == ["mode", "batch_width", "level_chunk",
                                                        "sparse_div", "concurrency", "level_loop",
                                                        "reserved"]
    # width, sparse_div, min_batched, sample, two doubles, cached, group_cut,
    # chunk, reserved
    assert ctypes.sizeof(_capi.bc_tuning) == 48
    o = bcm.make_options(bcm.BC_MODE_BATCHED, 32, 0, sparse_div=-1, concurrency=3,
                         level_loop=bcm.BC_LOOP_DEVICE)
    assert (o.mode, o.batch_width, o.sparse_div, o.concurrency, o.level_loop,
            list(o.reserved)) == (2, 32, -1, 3, 2, [0] * 2)


def test_trusted_flag_skips_symmetry_only():
    # an asymmetric CSR passes with the trust flag only if the structure is sound;
    # structural errors are still caught before any device call
    st, _ = _create(2, [0, 1, 2], [1, 5], flags=bcm.BC_GRAPH_TRUST_SYMMETRIC)
    assert st == bcm.BC_ERR_INVALID_GRAPH


LLVM_BIN = "/opt/rocm/llvm/bin"


@pytest.mark.skipif(not os.path.exists(os.path.join(LLVM_BIN, "clang-offload-bundler")),
                    reason="ROCm LLVM tools not installed")
def test_device_code_makes_no_calls(tmp_path):
    """Every device step is inlined into its kernels: the gfx950 code objects
    of the library hold kernels only, no call or return instructions."""
    import subprocess
    _capi.load()
    fat = tmp_path / "fat.bin"
    subprocess.run([os.path.join(LLVM_BIN, "llvm-objcopy"), "--dump-section=.hip_fatbin=" + str(fat),
                    _capi.LIB_PATH, str(tmp_path / "lib.copy")], check=True)
    data = fat.read_bytes()
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    starts = [m.start() for m in re.finditer(re.escape(magic), data)]
    assert starts, "no offload bundle in the library"
    kernels = 0
    for i, a in enumerate(starts):
        b = starts[i + 1] if i + 1 < len(starts) else len(data)
        part = tmp_path / f"b{i}.bin"
        part.write_bytes(data[a:b])
        co = tmp_path / f"co{i}.o"
        subprocess.run([os.path.join(LLVM_BIN, "clang-offload-bundler"), "--unbundle", "--type=o",
                        "--input=" + str(part), "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
                        "--output=" + str(co)], check=True)
        asm = subprocess.run([os.path.join(LLVM_BIN, "llvm-objdump"), "-d", str(co)],
                             capture_output=True, text=True, check=True).stdout
        assert "s_swappc" not in asm and "s_setpc" not in asm
        kernels += asm.count("s_endpgm")
    assert kernels > 0


def test_directed_flag_keeps_structure_checks():
    # a directed CSR need not be symmetric, but its structure is still checked
    # before any device call
    st, _ = _create(2, [0, 1, 2], [1, 5], flags=bcm.BC_GRAPH_DIRECTED)
    assert st == bcm.BC_ERR_INVALID_GRAPH
    st, _ = _create(2, [0, 2, 1], [1, 0], flags=bcm.BC_GRAPH_DIRECTED)
    assert st == bcm.BC_ERR_INVALID_GRAPH


def test_binding_checks_device_tensors_before_any_call():
    # the wrappers pass raw pointers, so an output of the wrong element size or
    # in host memory is refused before the library is reached (handle 0 is never
    # looked up: these checks come first)
    import torch
    cases = [
        (lambda t: bcm.bc_run_async(0, [0], t), "float64"),
        (lambda t: bcm.bc_run_async_noalloc(0, [0], t), "float64"),
        (lambda t: bcm.bc_run_multi(0, [[0]], [t]), "float64"),
        (lambda t: bcm.bc_run_graphs([0], [[0]], [t]), "float64"),
        (lambda t: bcm.bc_sssp(0, 0, t), "int32"),
        (lambda t: bcm.bc_pagerank(0, t), "float64"),
    ]
    for call, dtype in cases:
        other = torch.float32 if dtype == "float64" else torch.int64
        good = getattr(torch, dtype)
        with pytest.raises(TypeError):
            call(np.zeros(8))                                   # not a tensor
        with pytest.raises(TypeError):
            call(torch.zeros(8, dtype=other))                   # wrong element size
        with pytest.raises(ValueError, match="contiguous"):
            call(torch.zeros(16, dtype=good)[::2])
        with pytest.raises(ValueError, match="device memory"):
            call(torch.zeros(8, dtype=good))                    # host tensor
    with pytest.raises(ValueError, match="differ in length"):
        bcm.bc_run_multi(0, [[0], [1]], [])


def test_binding_checks_host_csr_extents():
    # the library reads n + 1 offsets and row_ptr[n] column ids from host memory
    with pytest.raises(ValueError, match="row_ptr"):
        bcm.bc_create_graph(3, np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32))
    with pytest.raises(ValueError, match="col_idx"):
        bcm.bc_create_graph(2, np.array([0, 1, 3], np.int32), np.array([1, 0], np.int32))
    # a CSR of the right extents still reaches the library's own checks
    st, _ = _create(2, [0, 1, 2], [1, 5])
    assert st == bcm.BC_ERR_INVALID_GRAPH
