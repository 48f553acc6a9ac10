"""Compile the gfx950 library libnpfem.so in-tree with hipcc: one object per source (the
step kernels as two, FP32 and FP64), compiled in parallel, then linked."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnpfem.so")
OBJ = os.path.join(HERE, "_build")

SOURCES = ["npfem_host.cpp", "npfem_kernels.hip", "npfem_net.hip", "npfem_collide.hip", "npfem_factor.hip"]
# (object, source, extra flags): the largest source first, so that it starts first
UNITS = [
    ("kernels64", "npfem_kernels.hip", ["-DNPFEM_PART=2"]),
    ("kernels32", "npfem_kernels.hip", ["-DNPFEM_PART=1"]),
    ("net", "npfem_net.hip", []),
    ("collide", "npfem_collide.hip", []),
    ("factor", "npfem_factor.hip", []),
    ("host", "npfem_host.cpp", []),
]
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 instructions are kept out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
    return r.returncode


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    objs = [os.path.join(OBJ, name + ".o") for name, _, _ in UNITS]
    cmds = [[hipcc, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", o]
            for (name, src, extra), o in zip(UNITS, objs)]
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as pool:
        codes = list(pool.map(lambda c: _run(c, verbose), cmds))
    if any(codes):
        raise RuntimeError("hipcc failed building libnpfem.so")
    if _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", LIB + ".tmp"], verbose):
        raise RuntimeError("hipcc failed linking libnpfem.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
