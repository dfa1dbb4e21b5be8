"""Builds the HIP library ``libaidw.so`` (gfx950) in the package directory.

Every source in ``csrc/`` is compiled for gfx950 with hipcc (one process per
file, in parallel) and linked into one shared library that exports the C ABI
of ``include/aidw.h``; ``ubench/issue_rate.hip`` (the VALU / transcendental
issue-rate microbenchmark behind the pair kernel's roofline) becomes
``libaidw_ubench.so``.  Flags:
  -O3 -std=c++17 -fPIC
  -ffp-contract=off   no implicit FMA contraction: the kNN squared distances
                      must be formed exactly as written; the pair kernel uses
                      explicit fmaf where it wants one
  -target-feature -packed-fp32-ops   no packed FP32 instructions
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libaidw.so")
UBENCH_SRC = os.path.join(HERE, "ubench", "issue_rate.hip")
UBENCH_LIB = os.path.join(HERE, "libaidw_ubench.so")
OBJ = os.path.join(ROOT, "_build", "obj")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-Wno-unused-command-line-argument"]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _compile(src):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, msgs))
    return obj, msgs


def build(verbose: bool = False) -> str:
    """Compile all HIP sources and link libaidw.so; returns the library path."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    for obj, msgs in results:
        if verbose and msgs.strip():
            print(msgs)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    build_ubench()
    return LIB


def build_ubench() -> str:
    """The issue-rate microbenchmark (bench.py --issue-rates) as its own small library."""
    tmp = UBENCH_LIB + ".tmp%d" % os.getpid()
    r = subprocess.run([HIPCC] + FLAGS + ["-shared", "-o", tmp, UBENCH_SRC], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (UBENCH_SRC, r.stdout + r.stderr))
    os.replace(tmp, UBENCH_LIB)
    return UBENCH_LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
