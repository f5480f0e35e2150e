"""Build step of the HIP library libcx.so (gfx950).

Every HIP source is compiled by hipcc for gfx950 only; host-only table code is
compiled without FMA contraction so the FP64 sampling tables are reproducible.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libcx.so")
OBJ = os.path.join(HERE, "_build")

SOURCES = ["cx_kernels.hip", "cx_policy.hip", "cx_api.cpp", "cx_spec.cpp", "cx_state.cpp",
           "cx_tune.cpp", "cx_server.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", f"-I{INC}", f"-I{CSRC}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
          "-Wno-unused-command-line-argument"]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    flags = list(COMMON)
    if src == "cx_spec.cpp":
        flags += ["-ffp-contract=off"]
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = ["hipcc", *flags, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
