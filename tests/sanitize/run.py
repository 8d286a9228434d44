"""Builds the library's host code with sanitizers and runs the host driver.

CPU only, no device: the host sources of libfht (the planner, the C ABI and
the planner pool) are compiled for the host only with sanitizers, once with
AddressSanitizer and UndefinedBehaviorSanitizer and once with
ThreadSanitizer; the kernel sources' objects of the regular build (kernels and
their launch wrappers, which the driver never calls) are linked as they are,
with
``driver.cpp`` (plans, queries, host-side batches, the planner pool fed from
several threads, fault injection), and run.  ``python tests/sanitize/run.py
[address|thread]``; exits non-zero on a build failure, a failed check or a
sanitizer report.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2411_07351_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"
HIPCC = "/opt/rocm/bin/hipcc"
SOURCES = ["plan.cpp", "api.hip", "planner.hip"]          # sanitized
KERNEL_OBJECTS = ["kernels.hip.o", "adjoint.hip.o", "peaks.hip.o"]  # from the regular build
KINDS = {"address": ["address", "undefined"], "thread": ["thread"]}


def _host_flags(kind):
    flags = []
    for s in KINDS[kind]:
        flags += ["-Xarch_host", "-fsanitize=" + s]
    return flags + ["-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host",
                    "-fno-omit-frame-pointer"]


def build(kind: str, out_dir: str) -> str:
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include")]
    cmds, objs = [], []
    for name in SOURCES:
        obj = os.path.join(out_dir, name + ".o")
        if name.endswith(".hip"):
            # api.hip holds a device variable (the no-allocation scratch), so its
            # device half is built too; the sanitizers apply to the host half only
            only = [] if name == "api.hip" else ["--offload-host-only"]
            cmd = [HIPCC] + only + ["--offload-arch=gfx950"] + common + \
                  _host_flags(kind) + ["-c", os.path.join(CSRC, name), "-o", obj]
        else:
            cmd = [CLANG] + common + _host_flags(kind) + ["-c", os.path.join(CSRC, name), "-o", obj]
        cmds.append(cmd)
        objs.append(obj)
    drv = os.path.join(out_dir, "driver.o")
    cmds.append([CLANG] + common + _host_flags(kind) + ["-c", os.path.join(HERE, "driver.cpp"),
                                                        "-o", drv])
    with ThreadPoolExecutor(max_workers=8) as pool:
        for res in pool.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds):
            if res.returncode != 0:
                raise RuntimeError(res.stdout + res.stderr)
    bdir = os.path.join(ROOT, "paper_2411_07351_amd", "_build")
    if not all(os.path.exists(os.path.join(bdir, o)) for o in KERNEL_OBJECTS):
        sys.path.insert(0, ROOT)
        from paper_2411_07351_amd import build as B
        B.build()
    objs += [os.path.join(bdir, o) for o in KERNEL_OBJECTS]
    exe = os.path.join(out_dir, "driver_" + kind)
    link = [CLANG] + _host_flags(kind) + ["-o", exe, drv] + objs + \
           ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-lpthread"]
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(res.stdout + res.stderr)
    return exe


def run(kind: str) -> subprocess.CompletedProcess:
    with tempfile.TemporaryDirectory() as d:
        exe = build(kind, d)
        env = dict(os.environ)
        env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=1"
        env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
        env["TSAN_OPTIONS"] = "halt_on_error=1:second_deadlock_stack=1"
        env["HIP_VISIBLE_DEVICES"] = ""
        return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=900)


if __name__ == "__main__":
    kinds = sys.argv[1:] or ["address", "thread"]
    rc = 0
    for k in kinds:
        res = run(k)
        sys.stdout.write(f"[{k}] exit {res.returncode}\n{res.stdout}{res.stderr[-4000:]}\n")
        rc = rc or res.returncode
    sys.exit(rc)
