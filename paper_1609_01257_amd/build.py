"""Build librngx.so (HIP for gfx950) in-tree with hipcc.

Every source under csrc/ is compiled as HIP C++ for gfx950 and linked into
paper_1609_01257_amd/librngx.so; cli/rngx_cli.cpp (host code only) becomes
paper_1609_01257_amd/rngx_cli, linked against it. Run ``python -m paper_1609_01257_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJDIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "librngx.so")
CLI_SRC = os.path.join(PKG, "cli", "rngx_cli.cpp")
CLI = os.path.join(PKG, "rngx_cli")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CXXFLAGS = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Wall", "-Wextra", "-Wno-unused-parameter",
    # Keep the compiler from forming packed-fp32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(src: str, extra) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CXXFLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def build(extra=(), jobs: int = 8) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    # A failed build must not leave the previous library (or program) behind
    # for the tests to load: remove both before compiling.
    for stale in (LIB, CLI):
        if os.path.exists(stale):
            os.remove(stale)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(lambda s: _compile(s, list(extra)), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    # The command-line program, linked against the library next to it.
    tmp = CLI + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-O2", "-std=c++17", "-Wall", "-Wextra", "-I", os.path.join(ROOT, "include"),
           CLI_SRC, "-o", tmp, "-L", PKG, "-lrngx", "-Wl,-rpath,$ORIGIN"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("rngx_cli build failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, CLI)
    return LIB


if __name__ == "__main__":
    print(build(extra=sys.argv[1:]))
