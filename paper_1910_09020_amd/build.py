"""Build libss.so (HIP, gfx950) in-tree.

Compiles every source under csrc/ with hipcc for gfx950 and links them into
``paper_1910_09020_amd/libss.so``.  The device assembly of every translation
unit is kept under ``_build/`` and scanned by ``isa_check``: the build fails if
any write through the scalar data cache appears in it.

Usage: python -m paper_1910_09020_amd.build [-j N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libss.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC, "-Wno-unused-command-line-argument"]

try:                                   # assembly scanner (kept out of GPU uploads)
    from . import isa_check
except ImportError:                    # pragma: no cover
    isa_check = None


def _compile(src: str) -> str:
    name = os.path.splitext(os.path.basename(src))[0]
    tmpdir = os.path.join(BUILD, name)
    os.makedirs(tmpdir, exist_ok=True)
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC, *FLAGS, "-save-temps=obj", "-c", src, "-o", obj]
    r = subprocess.run(cmd, cwd=tmpdir, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    # -save-temps=obj writes next to the object
    for s in glob.glob(os.path.join(BUILD, name + "*amdgcn*.s")):
        bad = isa_check.scan(s) if isa_check else []
        if bad:
            raise RuntimeError(f"{src}: forbidden scalar-memory write instructions in device code: {bad}")
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    rocm_lib = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(HIPCC))), "lib")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-L", rocm_lib, "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + rocm_lib]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args()
    build(a.j, verbose=True)
    sys.exit(0)
