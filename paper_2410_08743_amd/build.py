"""Builds libgsp.so (the HIP kernels and the C ABI of include/gsp.h) for
gfx950 with hipcc, in-tree, next to this file.

Every source is compiled for gfx950 only.  Packed FP32 instructions are
disabled (-packed-fp32-ops): the kernels are written against the unpacked
VALU, and the library's throughput figures are stated for it.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgsp.so")
SOURCES = ["api.hip", "preprocess.hip", "sort.hip", "raster_fwd.hip", "raster_bwd.hip", "lists.hip",
           "preprocess_bwd.hip", "misc.hip", "joint.hip",
           "relpose.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(HERE, "..", "include")]


# Per-source options.  The rasterizers branch on a wave-uniform
# condition between two variants of their walk over a batch; leaving uniform
# regions unstructured keeps that a plain scalar branch, without the
# register copies that merged paths need at the join.
EXTRA = {f: ["-mllvm", "-structurizecfg-skip-uniform-regions=true"]
         for f in ("raster_fwd.hip", "raster_bwd.hip")}


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if warn and verbose:
        print(warn, flush=True)
    return obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
