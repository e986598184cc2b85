"""Builds libvasmg.so in-tree for gfx950.

  * csrc/setup.cpp (host hierarchy setup) with g++ -O2 -fopenmp and no
    floating-point contraction (tree midlines and level-1 weights must be
    reproducible bit for bit);
  * csrc/vasmg.hip (kernels, device driver, C ABI) with hipcc for gfx950, packed
    FP32 instructions disabled;
  * csrc/server.hip (serving engine: host threads and streams over the C ABI);
  * csrc/galerkin.hip (device setup: fine assembly, Galerkin coarse operators,
    level layouts; no floating-point contraction);
  * csrc/tree.hip (device setup: region tree, lattice keys, prolongations; no
    floating-point contraction);
  * linked into paper_2505_09064_amd/libvasmg.so.

Run: python -m paper_2505_09064_amd.build   (or __graft_entry__.build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvasmg.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    f"-I{os.path.join(ROOT, 'include')}",
]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-fopenmp", "-ffp-contract=off", "-Wall",
             "-march=x86-64", f"-I{os.path.join(ROOT, 'include')}"]


def _run(cmd):
    print("[build]", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    setup_o = os.path.join(BUILD, "setup.o")
    hip_o = os.path.join(BUILD, "vasmg.o")
    server_o = os.path.join(BUILD, "server.o")
    galerkin_o = os.path.join(BUILD, "galerkin.o")
    tree_o = os.path.join(BUILD, "tree.o")
    _run(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, "setup.cpp"), "-o", setup_o])
    _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "server.hip"), "-o", server_o])
    # the device setup follows the host arithmetic operation by operation: no
    # floating-point contraction there
    _run([HIPCC, *HIP_FLAGS, "-ffp-contract=off", "-c", os.path.join(CSRC, "galerkin.hip"),
          "-o", galerkin_o])
    _run([HIPCC, *HIP_FLAGS, "-ffp-contract=off", "-c", os.path.join(CSRC, "tree.hip"), "-o", tree_o])
    _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "vasmg.hip"), "-o", hip_o])
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, hip_o, server_o, galerkin_o, tree_o, setup_o,
          "-lgomp", "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    build()
    sys.exit(0)
