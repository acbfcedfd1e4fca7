"""Build libhpmap.so (HIP for gfx950) in-tree with hipcc.

Each source is compiled to an object in parallel, then linked.
Usage: python -m paper_2008_05612_amd.build [-v]
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libhpmap.so")
SOURCES = ["structures.cpp", "capi.cpp", "capi_static.hip", "runtime.cpp", "kernels_popcount.hip",
           "gemm_kb1_4.hip", "gemm_kb5.hip", "gemm_kb6_10.hip", "gemm_kb11_12.hip",
           "gemm_batch.hip", "gemm_blk.hip", "gemm_blk_kb1_3.hip", "gemm_blk_kb4.hip",
           "gemm_blk_kb5.hip", "gemm_blk_kb6_7.hip", "gemm_blk_kb8_9.hip", "gemm_blk_kb10.hip",
           "gemm_blk_kb11_12.hip",
           "kernels_net.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed fp32 VALU ops are kept out of every code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in ordinary VGPRs where register pressure allows, so
    # the epilogue reads them without v_accvgpr_read copies
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-I" + os.path.join(ROOT, "include"),
    "-I" + CSRC,
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-result",
]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link libhpmap.so; always recompiles."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
