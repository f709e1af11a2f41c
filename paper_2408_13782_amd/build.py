"""Build libfpm.so (the HIP hot path) in-tree for gfx950 with hipcc.

Usage: python -m paper_2408_13782_amd.build   (or call build_library()).
The library is written next to this file; it is loaded by fpm.py.
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libfpm.so")

SOURCES = ["fpm_api.hip", "fpm_serve.hip"]
HEADERS = ["fft_line.hpp", "fpm_kernels.hpp", "fpm_aux.hpp", "fpm_subpixel.hpp", "fpm_fused.hpp"]

# Packed FP32 instructions are disabled on purpose (some of their forms have given
# unreliable results on this target).
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread",
    "-munsafe-fp-atomics",
    # gfx950 preloads the first kernel arguments into SGPRs: one scalar-load
    # round trip less at the start of every kernel
    "-mllvm", "-amdgpu-kernarg-preload-count=16",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def source_tag() -> str:
    """Digest of every source file of the library (csrc/ and include/), in name
    order: the tag that fpm_build_tag() returns for a build of these sources."""
    h = hashlib.sha256()
    for d in (CSRC, INCLUDE):
        for name in sorted(os.listdir(d)):
            if name.endswith((".hip", ".hpp", ".h")):
                h.update(name.encode())
                with open(os.path.join(d, name), "rb") as f:
                    h.update(f.read())
    return h.hexdigest()[:16]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build libfpm")
    return exe


def build_library(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, f'-DFPM_BUILD_TAG="{source_tag()}"', "-I", INCLUDE, "-I", CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature: harmless
    err = "\n".join(line for line in res.stderr.splitlines()
                    if "packed-fp32-ops" not in line)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
