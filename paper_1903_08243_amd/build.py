"""Build the HIP library (libmf.so) for gfx950 with hipcc, in-tree.

Every source under csrc/ is compiled to an object under _build/ (in parallel)
and linked into paper_1903_08243_amd/libmf.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", BUILD]


def _gen_tables() -> None:
    """Compile and run the host table generator (g++), writing _build/hex_tables.inc."""
    exe = os.path.join(BUILD, "gen_hex_tables")
    srcs = [os.path.join(CSRC, "gen_hex_tables.cpp"), os.path.join(CSRC, "tables.cpp")]
    r = subprocess.run(["g++", "-O2", "-std=c++17", *srcs, "-o", exe], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("table generator build failed:\n" + r.stderr[-4000:])
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    with open(os.path.join(BUILD, "hex_tables.inc"), "w") as f:
        f.write(out)


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    _gen_tables()
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    srcs = [p for p in srcs if not p.endswith("gen_hex_tables.cpp")]
    jobs = min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-4000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
