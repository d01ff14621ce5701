"""Build the gfx950 tracking library ``libxtm.so`` in-tree with hipcc.

Device code is compiled with ``-ffp-contract=off`` (the rounding contract of
the maps relies on explicit fma() calls only) and with packed-FP32 ops
disabled.  The result lands next to this file so it ships with the tree.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libxtm.so")
BUILD = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", BUILD]
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]

KERNEL_SOURCES = ["xtm_kernels.hip", "xtm_learn.hip"]
HOST_SOURCES = ["xtm_api.cpp", "xtm_jit.cpp", "xtm_photon.cpp", "xtm_normal6.cpp"]


def _embed_maps() -> None:
    """The run-time line compiler needs the element-map header as a string."""
    src = open(os.path.join(CSRC, "xtm_maps.h")).read()
    assert ")XTMMAPS\"" not in src
    with open(os.path.join(BUILD, "xtm_maps_src.inc"), "w") as f:
        f.write('R"XTMMAPS(' + src + ')XTMMAPS"\n')


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("hipcc failed (exit %d)" % r.returncode)
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    _embed_maps()
    objs = []
    for src in KERNEL_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run([HIPCC, *COMMON, *DEVICE, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run([HIPCC, *COMMON, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp, "-lhiprtc"])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def dump_isa(out_dir: str) -> None:
    """Write the gfx950 assembly of the kernels (for register/instruction review)."""
    os.makedirs(out_dir, exist_ok=True)
    for src in KERNEL_SOURCES:
        _run([HIPCC, *COMMON, *DEVICE, "--cuda-device-only", "-S", os.path.join(CSRC, src),
              "-o", os.path.join(out_dir, src + ".s")])


if __name__ == "__main__":
    build(verbose=True)
