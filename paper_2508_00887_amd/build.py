"""Build libfram.so (HIP kernels + host runtime) for gfx950, in-tree.

Usage: python -m paper_2508_00887_amd.build   (or build() from Python)
Every HIP translation unit is compiled with hipcc for --offload-arch=gfx950
with packed-FP32 instruction selection disabled, then linked into
paper_2508_00887_amd/libfram.so next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import pathlib
import subprocess

HERE = pathlib.Path(__file__).resolve().parent
ROOT = HERE.parent
CSRC = HERE / "csrc"
BUILD = ROOT / "_build"
LIB = HERE / "libfram.so"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", str(ROOT / "include"), "-Wall", "-Wno-unused-function",
]
SOURCES = ["gemm.hip", "sdsn.hip", "sdsn_onchip.hip", "misc.hip", "runtime.hip", "lap.hip", "noalloc.hip"]


def _compile(src: str) -> pathlib.Path:
    out = BUILD / (src + ".o")
    cmd = [HIPCC, *COMMON, "-c", str(CSRC / src), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out


def build(verbose: bool = False) -> pathlib.Path:
    BUILD.mkdir(exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *map(str, objs), "-o", str(tmp)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
