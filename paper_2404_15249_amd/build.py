"""Build the KFBI HIP library (libkfbi.so) for gfx950, in tree.

Usage: ``python -m paper_2404_15249_amd.build`` (or ``build()`` from Python).
Every call compiles from source.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libkfbi.so")
SOURCES = ["plan.cpp", "plan3.cpp", "kernels.hip", "batch.hip", "dst.hip", "k3.hip", "api.hip", "api3.hip", "gs.hip", "krylov.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the KFBI library needs ROCm's hipcc")


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            # packed FP32 instructions stay off in every HIP translation unit
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def spilling_kernels(remarks: str) -> list:
    """Kernels whose resource-usage remarks report VGPR spills or any other use
    of scratch (private) memory: a stack object a kernel never touches still
    makes every dispatch reserve scratch."""
    out, name = [], None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        if name is None:
            continue
        m = re.search(r"VGPRs Spill: (\d+)", line)
        if m and int(m.group(1)) > 0:
            out.append((name, "VGPRs Spill", int(m.group(1))))
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and int(m.group(1)) > 0:
            out.append((name, "ScratchSize", int(m.group(1))))
    return out


def _compile(src: str, build_dir: str) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + common_flags() + ["-Rpass-analysis=kernel-resource-usage", "-c",
                                        os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
    # every kernel must keep its registers and use no scratch memory: a build error otherwise
    spills = spilling_kernels(r.stderr)
    if spills:
        raise RuntimeError(f"{src}: kernels use scratch memory: {spills}")
    return obj


def build(verbose: bool = False) -> str:
    build_dir = os.path.join(OUT_DIR, "obj")
    os.makedirs(build_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libkfbi.so failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
