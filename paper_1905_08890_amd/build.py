"""Build step for the HIP library libgrmg.so (gfx950), in-tree.

Compiles every ``csrc/*.hip`` translation unit with hipcc for gfx950 and
links them into ``paper_1905_08890_amd/libgrmg.so``.  Packed FP32 ALU
operations are disabled (``-packed-fp32-ops``); FP64 atomics in the CIC
deposit use the hardware instructions (``-munsafe-fp-atomics``).  A multiply
and an add are contracted into an FMA only within one source expression
(``-ffp-contract=on``, not the default ``fast``, which also contracts across
statements after inlining and so decides differently in different kernels):
the launch forms of a smoother (fused tile, one launch per colour, batched)
then round the same operations and give the same bits.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libgrmg.so")
INCLUDE = os.path.join(ROOT, "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-munsafe-fp-atomics", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build_library(verbose: bool = False, jobs: int = 8) -> str:
    """Compile each .hip to an object (in parallel), then link the .so."""
    objdir = os.path.join(ROOT, "_build", "obj")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIB + f".tmp{os.getpid()}"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{text}")
    warn = [l for l in text.splitlines() if "warning" in l and "packed-fp32-ops" not in l
            and "target-feature" not in l]
    if warn:
        print(f"{os.path.basename(src)}:\n" + "\n".join(warn), file=sys.stderr)


if __name__ == "__main__":
    print(build_library(verbose=True))
