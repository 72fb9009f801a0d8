"""Compile libtdh.so for gfx950 with hipcc (in-tree, next to this file).

Each source is compiled to its own object in parallel (the device code of a
translation unit is self-contained: no relocatable device code), then the
objects are linked into one shared library."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtdh.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["tdh_kernels.hip", "tdh_mlp.hip", "tdh_gravity.hip", "tdh_remap.hip", "tdh_runtime.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off: they are generated from scalar code otherwise
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no multiply-add contraction: every stage-kernel form (and the oracle)
    # rounds each product and sum on its own, so the forms agree bit for bit
    "-ffp-contract=off",
    "-Wno-unused-command-line-argument",
]


def _compile(hipcc, src, extra, verbose):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [hipcc] + HIPCC_FLAGS + list(extra) + ["-x", "hip", "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"libtdh build failed ({os.path.basename(src)}):\n" + r.stderr[-6000:])
    return obj


def build(verbose: bool = False, extra=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(lambda s: _compile(hipcc, s, extra, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("libtdh link failed:\n" + r.stderr[-6000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
