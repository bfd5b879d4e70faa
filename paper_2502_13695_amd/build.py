"""Build the HIP shared library ``libpic.so`` in-tree for gfx950.

Usage: python -m paper_2502_13695_amd.build   (or call ``build()``)
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libpic.so")
BUILD = os.path.join(HERE, "_build")

ARCH = "gfx950"
COMMON = ["-x", "hip", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC,
          # no packed FP32 instructions (v_pk_*_f32) anywhere in device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]
UNITS = [
    ("pic_kernels.hip", ["-O3", "-munsafe-fp-atomics"]),
    ("pic_collide.hip", ["-O3"]),
    ("pic_runtime.hip", ["-O2"]),
    # canonical coefficients must be bit-reproducible: no FP contraction
    ("host_math.cpp", ["-O2", "-ffp-contract=off"]),
]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False):
    """Compile every HIP unit and link libpic.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    objs = []
    for src, flags in UNITS:
        obj = os.path.join(BUILD, src + ".o")
        cmd = [hipcc] + COMMON + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = OUT + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(OUT)
