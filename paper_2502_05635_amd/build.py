"""Compile the HIP library libtdagw.so for gfx950, in-tree.

The library links against the HIP runtime that ships inside the installed
PyTorch wheel (its libamdhip64.so carries the same SONAME as the system
one), so a process that imports torch holds exactly one HIP runtime.
Run:  python -m paper_2502_05635_amd.build
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libtdagw.so")
SOURCES = ["context.cpp", "kbuild.hip", "propagate.hip", "compress.hip", "gemm.hip", "adjoint.hip", "intraband.hip"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off: plain float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def torch_lib_dir() -> str:
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or spec.origin is None:
        raise RuntimeError("torch is required: the library links against its HIP runtime")
    return os.path.join(os.path.dirname(spec.origin), "lib")


def _compile(src: str) -> str:
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [os.path.join(ROCM, "bin", "hipcc"), *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", out]
    if src.endswith(".cpp"):
        cmd = [os.path.join(ROCM, "bin", "hipcc"), *[f for f in HIP_FLAGS if not f.startswith("--offload")],
               "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tl = torch_lib_dir()
    tmp = LIB + ".tmp"
    cmd = [os.path.join(ROCM, "lib", "llvm", "bin", "clang++"), "-shared", "-o", tmp, *objs,
           f"-L{tl}", "-l:libamdhip64.so", "-l:librocsolver.so", "-l:librocblas.so",
           f"-Wl,-rpath,{tl}", "-Wl,--no-undefined"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    shutil.move(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
