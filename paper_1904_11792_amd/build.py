"""Build liblbm.so (HIP, gfx950) in-tree with hipcc.

Usage: python paper_1904_11792_amd/build.py   (always recompiles; run it by
path -- importing the package loads the library it builds)
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "liblbm.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["lbm_step.hip", "lbm_aux.hip", "lbm_capi.hip"]

# Host-sanitized build (build(sanitize_host=True)): the host code of the
# library instrumented with AddressSanitizer and UndefinedBehaviorSanitizer;
# the runtime is not linked in, so a process must preload clang's shared ASan
# runtime (which carries the UBSan handlers) to load it.  It is for testing
# the host code only: its device code is compiled without optimisation (a
# third of the compile time), and its kernels are not meant to run.
OUT_HOSTSAN = os.path.join(HERE, "liblbm_hostsan.so")
OBJDIR_HOSTSAN = os.path.join(HERE, "_build_hostsan")
HOSTSAN_FLAGS = ["-O1", "-Xarch_device", "-O0", "-Xarch_host", "-g",
                 "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled: only scalar FP32 VALU code is emitted.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def _compile(src: str, objdir: str = OBJDIR, extra=()) -> str:
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False, sanitize_host: bool = False) -> str:
    objdir, out = (OBJDIR_HOSTSAN, OUT_HOSTSAN) if sanitize_host else (OBJDIR, OUT)
    extra = HOSTSAN_FLAGS if sanitize_host else ()
    os.makedirs(objdir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda src: _compile(src, objdir, extra), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("linking liblbm.so failed")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
