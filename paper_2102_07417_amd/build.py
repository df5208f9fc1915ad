"""Build libcamg.so (the HIP kernels and the C-ABI) for gfx950 with hipcc.

The library is built in-tree next to this file.  Every HIP source is
compiled with -ffp-contract=off (the set-up reproduces the reference
rounding exactly) and without packed-FP32 instructions.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcamg.so")
SOURCES = ["setup.hip", "spgemm.hip", "solve.hip", "multi.hip", "serve.hip", "batch.hip", "camg.hip"]
ARCH = os.environ.get("CAMG_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _obj(src):
    return os.path.join(CSRC, "_build", os.path.splitext(src)[0] + ".o")


def _compile(src, verbose):
    os.makedirs(os.path.join(CSRC, "_build"), exist_ok=True)
    cmd = ["hipcc", "-c", *FLAGS, os.path.join(CSRC, src), "-o", _obj(src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return r.stderr


def build(verbose: bool = False) -> str:
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        warns = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    if verbose:
        for w in warns:
            if w.strip():
                print(w)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *[_obj(s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
