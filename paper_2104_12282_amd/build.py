"""Builds libfe_hip.so (the gfx950 HIP library behind include/fe_abi.h) in-tree
with hipcc.  Run as ``python -m paper_2104_12282_amd.build``."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libfe_hip.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["fe_host.cpp", "fe_abi.cpp", "fe_kernels.hip", "fe_kxu.hip", "fe_mg.hip", "fe_onsg.hip"]
# Packed-FP32 instructions are switched off for every device pass.
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-Wall",
         "-Wno-unused-function", "-fvisibility=hidden", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def source_digest() -> str:
    """Hash of the HIP sources and the public header (ties stored profiler
    figures to the kernels they were taken on)."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(CSRC, name), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "fe_abi.h"), "rb").read())
    return h.hexdigest()[:16]


def _compile(src: str, out_dir: str = OUT, defines=()) -> str:
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *[f"-D{d}" for d in defines], "-x", "hip", "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, out_lib: str = LIB, defines=()) -> str:
    """Compiles every source and links out_lib; `defines` are extra -D macros
    (tuning constants), empty for the library the package loads."""
    out_dir = OUT if out_lib == LIB else os.path.splitext(out_lib)[0] + "_obj"
    os.makedirs(out_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, out_dir, defines), SOURCES))
    tmp = out_lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-L/opt/rocm/lib", "-lrocblas", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out_lib)
    if verbose:
        print(f"built {out_lib}")
    return out_lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
