"""Builds ``libfht.so`` (the gfx950 HIP library behind ``include/fht.h``) in-tree.

``python -m paper_2411_07351_amd.build`` or ``build()``: hipcc cross-compiles
for gfx950 without a GPU.  Objects go to ``paper_2411_07351_amd/_build/``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libfht.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are kept out of the generated code.
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include")]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra"]


def _torch_lib_dir() -> str | None:
    """torch's bundled ROCm libraries: the library must share torch's HIP runtime
    (streams and device pointers come from torch), so it is linked to look there first."""
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec and spec.origin:
            d = os.path.join(os.path.dirname(spec.origin), "lib")
            if os.path.exists(os.path.join(d, "libamdhip64.so")):
                return d
    except Exception:
        pass
    return None


SOURCES = [("plan.cpp", "cxx"), ("kernels.hip", "hip"), ("adjoint.hip", "hip"), ("peaks.hip", "hip"), ("api.hip", "hip"), ("planner.hip", "hip")]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("command failed: " + " ".join(cmd))
    # hipcc's host pass does not know the packed-fp32 feature name: drop that note.
    noise = ("packed-fp32-ops", "warning generated", "warnings generated")
    msg = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                    if l.strip() and not any(n in l for n in noise))
    if msg.strip():
        sys.stderr.write(msg + "\n")


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compiles every source (in parallel, ``jobs`` at a time; 0: one per
    source, at most 8) and links the library."""
    os.makedirs(OUT, exist_ok=True)
    cmds, objs = [], []
    for name, kind in SOURCES:
        src = os.path.join(CSRC, name)
        obj = os.path.join(OUT, name + ".o")
        if kind == "cxx":
            cmd = ["g++"] + CXX_FLAGS + ["-c", src, "-o", obj]
        else:
            cmd = [HIPCC] + HIP_FLAGS + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        cmds.append(cmd)
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=jobs or min(8, len(cmds))) as pool:
        for f in [pool.submit(_run, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    tdir = _torch_lib_dir()
    if tdir:
        cmd += ["-Wl,-rpath," + tdir, "-Wl,--disable-new-dtags"]
    if verbose:
        print(" ".join(cmd))
    _run(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
