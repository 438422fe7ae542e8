"""Build libfs.so (HIP kernels + C ABI) for gfx950 with hipcc, in tree."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libfs.so")
SOURCES = ["ops3d_f32.hip", "ops3d_f32_strat.hip", "ops3d_f64.hip", "ops3d_f64_strat.hip", "ops3d.hip", "ops2d.hip", "ens2d.hip", "mlp.hip", "closure.hip", "diag.hip", "fs_api.cpp"]
ARCH = os.environ.get("FS_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *FLAGS, "-I", INCLUDE, "-x", "hip", "-c", os.path.join(SRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int | None = None, src: str | None = None,
          out: str | None = None, objdir: str | None = None) -> str:
    """Compile the sources in `src` (default csrc/) into `out` (default libfs.so)."""
    global SRC, BUILD
    if src:
        SRC = src
    if objdir:
        BUILD = objdir
    lib = out or LIB
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = lib + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
