"""Build libvx.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libvx.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["vx_runtime.hip", "vx_gen.hip", "vx_wind.hip", "vx_refine.hip", "vx_batch.hip", "vx_mlp.hip",
           "vx_node.hip", "vx_density.hip"]

COMMON = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
    "-fno-fast-math",
    # no packed FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
PER_FILE = {
    # the generators must round every FP64 operation separately
    "vx_gen.hip": ["-ffp-contract=off"],
    # products fused into sums within one expression only, decided at the source level, so that the
    # refinement kernels, which share their arithmetic as inline functions, round alike whatever
    # the surrounding control flow
    "vx_refine.hip": ["-ffp-contract=on"],
    "vx_density.hip": ["-ffp-contract=on"],
}


# host-only C++ (the consumers of the lists: graph, sampling, curves), built with the host compiler
CPP_SOURCES = ["vx_graph.cpp"]
CPP_FLAGS = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-fno-fast-math", "-ffp-contract=off"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()

    def one(src):
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmd = [hipcc, *COMMON, *PER_FILE.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    def one_cpp(src):
        obj = os.path.join(BUILD, src.replace(".cpp", ".o"))
        cmd = [os.environ.get("CXX", "g++"), *CPP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"host compiler failed for {src}:\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES) + len(CPP_SOURCES))) as ex:
        objs = list(ex.map(one, SOURCES)) + list(ex.map(one_cpp, CPP_SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
