"""Build the native libraries in-tree.

  libewahthr.so  -- HIP kernels + host runtime + C ABI (hipcc, gfx950 only)
  datagen/libewahgen.so -- seeded input generators (gcc)

Run `python -m paper_1402_4466_amd.build` or call build_all().
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libewahthr.so")
GENLIB = os.path.join(HERE, "datagen", "libewahgen.so")

HIP_SOURCES = ["thr_tile.hip", "thr_api.cpp", "select.hip", "mlp.hip", "selector.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-x", "hip",
    # packed fp32 instructions stay off: some of their forms have given wrong results on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _run(cmd, cwd=None):
    p = subprocess.run(cmd, cwd=cwd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"command failed ({p.returncode}): {' '.join(cmd)}\n{out}")
    return out


def build_generator() -> str:
    tmp = GENLIB + ".tmp"
    _run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp,
          os.path.join(HERE, "datagen", "ewahgen.c"), "-lm"])
    os.replace(tmp, GENLIB)
    return GENLIB


def build_hip() -> str:
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in HIP_SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(objdir, src + ".o")
        _run([HIPCC, *HIP_FLAGS, "-c", "-o", obj, path])
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


def build_tools() -> str:
    """Measurement tool: streaming-read ceiling of the device (not part of the query path)."""
    os.makedirs(os.path.join(HERE, "bin"), exist_ok=True)
    exe = os.path.join(HERE, "bin", "stream_ceiling")
    _run([HIPCC, "-O3", "--offload-arch=gfx950", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-o", exe + ".tmp", os.path.join(CSRC, "stream_ceiling.hip")])
    os.replace(exe + ".tmp", exe)
    return exe


def build_all() -> None:
    build_generator()
    build_hip()
    build_tools()


if __name__ == "__main__":
    build_all()
    print("built", LIB, GENLIB, file=sys.stderr)
