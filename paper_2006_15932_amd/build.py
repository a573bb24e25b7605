"""Build libdbm.so (gfx950) in-tree with hipcc.

Every HIP source is compiled with packed-FP32 instruction selection disabled
(-packed-fp32-ops); object files are built in parallel and linked into
paper_2006_15932_amd/libdbm.so next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdbm.so")
BUILD_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("DBM_OFFLOAD_ARCH", "gfx950")

SOURCES = ["dbm_kernels.hip", "dbm_api.cpp", "dbm_model.cpp"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, extra=(), build_dir=None) -> str:
    obj = os.path.join(build_dir or BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), "--offload-arch=" + ARCH, *COMMON, *extra, "-c", os.path.join(CSRC, src),
           "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile and link; `defines` are extra -D options (tuning variants)."""
    extra = tuple("-D" + d for d in defines)
    bdir = BUILD_DIR if not defines else BUILD_DIR + "_" + "_".join(defines).replace("=", "")
    os.makedirs(bdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda src: _compile(src, extra, bdir), SOURCES))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
