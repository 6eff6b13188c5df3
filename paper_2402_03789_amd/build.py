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


# Resource limits of the tensor-product kernels, from the compiler's resource-usage remarks.
# The float32-arithmetic kernels of models with edge harmonics up to l = 2 (the FP32 and BF16
# forms of the five-block model) must use no scratch at all.  The others (float64 forms, and
# harmonics up to l = 3) may keep a small private array and spill a few registers; beyond
# these limits the build fails.
TP_MAX_VGPR_SPILL = 12
TP_MAX_SCRATCH = 72  # bytes per lane


def tp_resources(remarks: str) -> list:
    """Per-kernel VGPRs, AGPRs, spilled VGPRs, scratch bytes per lane and occupancy parsed from
    `-Rpass-analysis=kernel-resource-usage` output."""
    import re
    recs, cur = [], None
    keys = {"VGPRs": "vgpr", "AGPRs": "agpr", "VGPRs Spill": "spill",
            "ScratchSize [bytes/lane]": "scratch", "Occupancy [waves/SIMD]": "occupancy"}
    for line in remarks.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = {"name": m.group(1)}
            recs.append(cur)
            continue
        m = re.search(r"remark:\s+([A-Za-z][A-Za-z /\[\]]*?): (\d+) \[", line)
        if m and cur is not None and m.group(1) in keys:
            cur[keys[m.group(1)]] = int(m.group(2))
    return recs


def _tp_kernel_kind(mangled: str):
    """(float32 arithmetic, edge harmonic degree) of a k_tp_fwd/k_tp_bwd instantiation from its
    mangled name (template arguments T, S, L1, LSH, ...)."""
    import re
    m = re.search(r"k_tp_(?:fwd|bwd)I([fd])(?:f|d|NS_6bf16_tE|N2sn6bf16_tE)Li(\d)ELi(\d)E", mangled)
    if not m:
        return None
    return m.group(1) == "f", int(m.group(3))


def check_tp_resources(remarks: str, report_path: str) -> list:
    recs = [r for r in tp_resources(remarks) if "k_tp_" in r["name"]]
    bad = []
    lines = ["kernel\tvgpr\tagpr\tspill\tscratch\toccupancy"]
    for r in recs:
        kind = _tp_kernel_kind(r["name"])
        lines.append(f"{r['name']}\t{r.get('vgpr')}\t{r.get('agpr')}\t{r.get('spill')}\t"
                     f"{r.get('scratch')}\t{r.get('occupancy')}")
        strict = kind is not None and kind[0] and kind[1] <= 2
        if strict and (r.get("scratch", 0) or r.get("spill", 0)):
            bad.append(r)
        elif r.get("spill", 0) > TP_MAX_VGPR_SPILL or r.get("scratch", 0) > TP_MAX_SCRATCH:
            bad.append(r)
    with open(report_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    if not recs:
        raise RuntimeError("no resource-usage remarks for the tensor-product kernels")
    strict_n = sum(1 for r in recs if (_tp_kernel_kind(r["name"]) or (False, 9))[0]
                   and (_tp_kernel_kind(r["name"]) or (False, 9))[1] <= 2)
    print(f"tensor-product kernels: {len(recs)} instantiations ({strict_n} float32 l<=2 with no "
          f"scratch allowed); max VGPRs {max(r.get('vgpr', 0) for r in recs)}, max spilled "
          f"VGPRs {max(r.get('spill', 0) for r in recs)}, max scratch "
          f"{max(r.get('scratch', 0) for r in recs)} B/lane; table in {report_path}",
          file=sys.stderr)
    return bad


def build(verbose: bool = False, jobs: int | None = None) -> str:
    gen_cg()
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    objs = [os.path.join(OBJ, s[:-4] + ".o") for s in srcs]
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))

    # the tensor-product kernels (one translation unit per precision form) report their
    # register and scratch use
    def is_tp(s):
        return s.startswith("k_tp_")

    def one(pair):
        s, o = pair
        extra = ["-Rpass-analysis=kernel-resource-usage"] if is_tp(s) else []
        cmd = [HIPCC, *HIP_FLAGS, *extra, "-c", os.path.join(CSRC, s), "-o", o]
        out = _run(cmd)
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        return s, out

    # the longest compiles first, so that they overlap the rest
    order = sorted(zip(srcs, objs), key=lambda so: (not is_tp(so[0]), so[0]))
    remarks = []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for s, out in ex.map(one, order):
            if is_tp(s):
                remarks.append(out)
            elif verbose and out.strip():
                print(out, file=sys.stderr)
    bad = check_tp_resources("\n".join(remarks), os.path.join(OBJ, "k_tp_resources.tsv"))
    if bad:
        raise RuntimeError("tensor-product kernels over their register/scratch limits: "
                           + ", ".join(f"{r['name']} (spill {r.get('spill')}, scratch "
                                       f"{r.get('scratch')})" for r in bad))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
