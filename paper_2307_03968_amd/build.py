"""Build libhmps.so for gfx950 in-tree.

    python -m paper_2307_03968_amd.build [--jobs N] [--debug]

Host sources (*.cpp) are compiled with ROCm's clang++ and OpenMP; device
sources (*.hip) with hipcc for gfx950 only.  Objects go to _build/, the
shared library next to this file.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libhmps.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

# -fcx-fortran-rules: complex products without the NaN/infinity recovery
# call (identical results for finite operands), division still range-reduced
HOST_FLAGS = ["-O3", "-fcx-fortran-rules", "-fPIC", "-std=c++17", "-fopenmp", "-Wall",
              "-Wno-unused-function",
              "-I" + os.path.join(ROOT, "include")]
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-fopenmp",
             "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
             # no packed FP32 instructions in device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed:\n  " + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def sources():
    host = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    dev = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    return host, dev


def build(jobs: int = 0, debug: bool = False, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    clangxx = os.path.join(ROCM, "llvm", "bin", "clang++")
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    host, dev = sources()
    extra = ["-g"] if debug else []
    cmds = []
    objs = []
    for f in host:
        o = os.path.join(BUILD, f + ".o")
        cmds.append([clangxx] + HOST_FLAGS + extra + ["-c", os.path.join(CSRC, f), "-o", o])
        objs.append(o)
    for f in dev:
        o = os.path.join(BUILD, f + ".o")
        cmds.append([hipcc] + HIP_FLAGS + extra + ["-c", os.path.join(CSRC, f), "-o", o])
        objs.append(o)
    jobs = jobs or min(8, len(cmds))
    with cf.ThreadPoolExecutor(jobs) as ex:
        outs = list(ex.map(_run, cmds))
    if verbose:
        for c, out in zip(cmds, outs):
            if out.strip():
                print(" ".join(c[:1] + c[-3:]), "\n", out)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fopenmp", "-o", tmp] + objs +
         ["-Wl,-rpath," + os.path.join(ROCM, "llvm", "lib"), "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    shutil.move(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=0)
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.debug, a.verbose))


if __name__ == "__main__":
    sys.exit(main())
