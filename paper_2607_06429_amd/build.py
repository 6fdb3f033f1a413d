"""Build libvsie.so (HIP, gfx950) in-tree.

    python paper_2607_06429_amd/build.py

(run by path: importing the package needs the library this script builds).

Each csrc/*.hip file is compiled separately (in parallel) into _build/ and
linked into paper_2607_06429_amd/libvsie.so.  Packed FP32 instructions are
disabled for all device code.
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
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libvsie.so")
ARCH = os.environ.get("VSIE_OFFLOAD_ARCH", "gfx950")

SOURCES = ["pair_kernels.hip", "mfma_kernels.hip", "sym_kernels.hip", "far_field.hip", "dense_kernels.hip",
           "aux_kernels.hip", "gradient.hip", "vsie_api.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


# Per-file device options.  The matrix-core pair kernels keep their MFMA
# accumulators in VGPRs: with the compiler's default register classes the
# loop-carried accumulators were copied between AGPRs and VGPRs on every
# source step (192 v_accvgpr moves per step in the FP64 kernel).
FILE_FLAGS = {"mfma_kernels.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def flags_for(src: str) -> list:
    return FLAGS + FILE_FLAGS.get(src, [])


def _hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *flags_for(src), "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), res.stdout, res.stderr))
    errs = [l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if errs:
        sys.stderr.write("\n".join(errs) + "\n")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-L/opt/rocm/lib", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), res.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
