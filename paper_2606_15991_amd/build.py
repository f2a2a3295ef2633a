"""Build libtilegemm.so (HIP, gfx950) in-tree.

Every translation unit is compiled with hipcc for gfx950 only, then linked
into paper_2606_15991_amd/libtilegemm.so.  Packed binary32 instructions are
disabled in device code (-packed-fp32-ops).
"""
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libtilegemm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["tilegemm.cpp", "tune.cpp", "gemm_tiled.hip", "gemm_skinny.hip",
           "gemm_simple.hip", "split_norm.hip", "mlp.hip", "elementwise.hip"]

DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature",
                "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I", os.path.join(ROOT, "include")]


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [HIPCC] + COMMON + DEVICE_FLAGS + lang + [
        "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip() and verbose:
        print(err, file=sys.stderr)
    return obj


# Benchmark driver of the execution-mode measurement (a separate program
# linked against the library, not part of it).
EXEC_MODES_SRC = "exec_modes.cpp"
EXEC_MODES_BIN = os.path.join(PKG, "tg_exec_modes")


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o",
           LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    cmd = [HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           os.path.join(CSRC, EXEC_MODES_SRC), "-o", EXEC_MODES_BIN + ".tmp",
           "-L", PKG, "-ltilegemm", "-Wl,-rpath,$ORIGIN"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(EXEC_MODES_BIN + ".tmp", EXEC_MODES_BIN)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
