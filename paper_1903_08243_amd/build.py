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


# Per-file compiler flags (none at present).
FILE_FLAGS: dict = {}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *FILE_FLAGS.get(os.path.basename(src), []), "-c", src, "-o", obj]
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


SAN_LIB = os.path.join(BUILD, "libmf_hostsan.so")
ASAN_RT = "libclang_rt.asan-x86_64.so"


def build_host_sanitized(verbose: bool = False) -> str:
    """A copy of the library whose host code of the set-up paths (mf_api.cpp: meshes,
    spaces, colouring, numbering, patches, operator set-up; cnn.cpp: network
    validation) is built with AddressSanitizer and UndefinedBehaviorSanitizer, for CPU
    runs of those paths (load it with the ASan runtime preloaded; see asan_runtime()).
    The other objects and all device code are the ordinary build's."""
    if not os.path.exists(LIB):
        build(verbose)
    san = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for name in ("mf_api.cpp", "cnn.cpp"):
        obj = os.path.join(BUILD, name + ".hostsan.o")
        flags = [f for f in FLAGS if f != "-O3"]
        r = subprocess.run([HIPCC, *flags, *san, "-c", os.path.join(CSRC, name), "-o", obj], capture_output=True,
                           text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitized build of {name} failed:\n{r.stderr[-4000:]}")
        objs.append(obj)
    rest = [os.path.join(BUILD, f) for f in sorted(os.listdir(BUILD))
            if f.endswith(".o") and not f.endswith(".hostsan.o") and f not in ("mf_api.cpp.o", "cnn.cpp.o")]
    r = subprocess.run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *rest, *objs, "-Xarch_host",
                        "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-o", SAN_LIB],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitized link failed:\n" + r.stderr[-4000:])
    if verbose:
        print("built", SAN_LIB)
    return SAN_LIB


def asan_runtime() -> str:
    """Path of the compiler's ASan runtime (to preload into an uninstrumented Python)."""
    r = subprocess.run([HIPCC, "-print-file-name=" + ASAN_RT], capture_output=True, text=True, check=True)
    return r.stdout.strip()


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
