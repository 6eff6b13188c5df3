"""Build libsn.so in-tree for gfx950.

Steps: compile the host-only Clebsch-Gordan generator with g++, run it to
write csrc/cg_tables.h, compile every csrc/*.hip with hipcc for gfx950 in
parallel, and link libsn.so next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsn.so")

ARCH = os.environ.get("SN_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed-FP32 instructions are disabled for all device code.
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-result",
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def gen_cg():
    exe = os.path.join(CSRC, "cg_gen")
    _run(["g++", "-O2", "-std=c++17", "-o", exe, os.path.join(CSRC, "cg_gen.cpp")])
    _run([exe, os.path.join(CSRC, "cg_tables.h")])


def build(verbose: bool = False, jobs: int | None = None) -> str:
    gen_cg()
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    objs = [os.path.join(OBJ, s[:-4] + ".o") for s in srcs]
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))

    def one(pair):
        s, o = pair
        cmd = [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, s), "-o", o]
        out = _run(cmd)
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        return out

    with cf.ThreadPoolExecutor(jobs) as ex:
        for out in ex.map(one, zip(srcs, objs)):
            if verbose and out.strip():
                print(out, file=sys.stderr)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
