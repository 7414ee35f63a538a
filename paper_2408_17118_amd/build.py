"""Build liboica.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Usage: python -m paper_2408_17118_amd.build   (or build() from Python).
Every call recompiles; objects go to _build/ inside the package and the
shared library is written next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
ROOT = os.path.dirname(PKG)
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "liboica.so")
BUILD = os.path.join(PKG, "_build")

ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources() -> list[str]:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


# Host code instrumented with AddressSanitizer and UndefinedBehaviorSanitizer
# (device code is built as usual): a separate library for CPU tests of the
# host-side paths, loaded with the ASan runtime preloaded.
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
SAN_OUT = os.path.join(BUILD, "san", "liboica_san.so")


def _compile(src: str, san: bool = False) -> str:
    out_dir = os.path.join(BUILD, "san") if san else BUILD
    obj = os.path.join(out_dir, os.path.basename(src)[:-4] + ".o")
    cmd = [hipcc(), *FLAGS, *(SAN_FLAGS if san else []), "-I", INCLUDE, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, san: bool = False) -> str:
    """Compile every source and link the library; san=True builds the
    sanitizer-instrumented copy (SAN_OUT) instead."""
    out_path = SAN_OUT if san else OUT
    os.makedirs(os.path.dirname(out_path) if san else BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda src: _compile(src, san), srcs))
    tmp = out_path + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out_path)
    if verbose:
        print(f"built {out_path}")
    return out_path


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
