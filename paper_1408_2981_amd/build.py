"""Builds libtpmg.so in-tree for gfx950.

Host C++ (mesh, assembly) is compiled with g++ with floating-point
contraction off, so the geometry is the same on every machine; the C ABI
and the HIP kernels are compiled with hipcc for gfx950 only. Packed FP32
instructions are disabled in device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OUT = os.path.join(HERE, "libtpmg.so")
BUILD = os.path.join(HERE, "_build")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", "-Wall"]
DEVICE_FLAGS = [
    "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-ffp-contract=fast",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in ("mesh.cpp", "operator.cpp"):
        obj = os.path.join(BUILD, src + ".o")
        jobs.append((["g++", *HOST_FLAGS, "-I", INCLUDE, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    for src in ("tpmg.cpp", "mlp.cpp"):
        obj = os.path.join(BUILD, src + ".o")
        jobs.append(([HIPCC, "-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", "-I", INCLUDE, "-c",
                      os.path.join(CSRC, src), "-o", obj], obj))
    for src in sorted(f for f in os.listdir(CSRC) if f.endswith(".hip")):
        obj = os.path.join(BUILD, src + ".o")
        jobs.append(([HIPCC, *DEVICE_FLAGS, "-I", INCLUDE, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    with ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        list(ex.map(lambda j: _run(j[0]), jobs))
    objs = [obj for _, obj in jobs]
    tmp = OUT + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-Wl,--no-undefined", "-o", tmp, *objs])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
