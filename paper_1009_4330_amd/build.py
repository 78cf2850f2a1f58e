"""Build the HIP library libmd_mi355x.so (gfx950) in-tree with hipcc.

Device code is compiled with -ffp-contract=off (every FMA is explicit in the
source) and with packed FP32 instructions disabled.
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
LIB = os.path.join(PKG, "libmd_mi355x.so")
SOURCES = ["md_bin.hip", "md_forces.hip", "md_integrate.hip", "md_api.hip"]
ARCH = os.environ.get("MD_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument", f"-I{INCLUDE}", f"-I{CSRC}"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


SAN_LIB = os.path.join(BUILD, "asan", "libmd_mi355x_san.so")
# host code of md_api.hip (argument checks, layouts, workspace and status
# handling) with AddressSanitizer and UBSan; device code as in build()
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address,undefined",
             "-Xarch_host", "-fno-sanitize-recover=all",
             "-Xarch_host", "-fno-omit-frame-pointer"]


def build_sanitized() -> str:
    """The library with md_api.hip's host code built under ASan and UBSan,
    linked with build()'s objects of the other sources (run build() first).
    A process loading it needs clang's ASan runtime preloaded."""
    os.makedirs(os.path.dirname(SAN_LIB), exist_ok=True)
    objs = [os.path.join(BUILD, os.path.splitext(f)[0] + ".o") for f in SOURCES if f != "md_api.hip"]
    for o in objs:
        if not os.path.exists(o):
            raise RuntimeError(f"{o} is missing: run build() first")
    api = os.path.join(os.path.dirname(SAN_LIB), "md_api_san.o")
    cmd = [HIPCC, *FLAGS, *SAN_FLAGS, "-c", os.path.join(CSRC, "md_api.hip"), "-o", api]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed on md_api.hip (sanitized)")
    res = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-o", SAN_LIB, *objs, api],
                         capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc link failed (sanitized)")
    return SAN_LIB


def build() -> str:
    """Compile every HIP source and link the shared library."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
