"""Build libhexsv.so for gfx950 with hipcc (in-tree, no JIT cache).

Each translation unit is compiled to an object in ``_build/`` and linked into
``paper_2406_14933_amd/lib/libhexsv.so``.  The FP64 kernels and the common
kernels are compiled without floating-point contraction; packed FP32
instructions are disabled everywhere.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libhexsv.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", CSRC, "-I", INCLUDE]

# (source, extra flags)
UNITS = [
    ("hexsv_f64.hip", ["-ffp-contract=off"]),
    ("hexsv_f32.hip", ["-ffp-contract=fast-honor-pragmas"]),
    ("hexsv_common.hip", ["-ffp-contract=off"]),
    ("hexsv_capi.hip", ["-ffp-contract=off"]),
    ("hexsv_ens.hip", ["-ffp-contract=off"]),
    ("hexsv_tune.cpp", ["-x", "hip"]),
    ("hexsv_nn.hip", ["-ffp-contract=fast-honor-pragmas"]),
    ("hexsv_sur.hip", ["-ffp-contract=off"]),
]


def _compile(src, extra):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(UNITS))) as ex:
        objs = list(ex.map(lambda u: _compile(*u), UNITS))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
