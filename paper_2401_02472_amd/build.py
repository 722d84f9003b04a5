"""Compile the gfx950 HIP library libbc_mi355x.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "libbc_mi355x.so")
# the same library with the cross-lane exec checks compiled in (BC_CHECK_EXEC)
CHECK_LIB_PATH = os.path.join(HERE, "libbc_mi355x_check.so")
SOURCES = ["bc_graph.hip", "bc_plain.hip", "bc_batched.hip", "bc_sssp.hip", "bc_pagerank.hip",
           "bc_rt_graph.hip", "bc_rt_plain.hip", "bc_rt_batched.hip", "bc_rt_algos.hip", "bc_tune.hip",
           "bc_capi.hip", "bc_noalloc.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no packed FP32 instructions (v_pk_*_f32) in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def build(verbose: bool = False, check_exec: bool = False) -> str:
    """Compile the library; with check_exec, the check build (every cross-lane
    helper counts calls made with part of a wave inactive)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = CHECK_LIB_PATH if check_exec else LIB_PATH
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, *(["-DBC_CHECK_EXEC"] if check_exec else []),
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    import sys
    print(build(verbose=True, check_exec="--check-exec" in sys.argv))
