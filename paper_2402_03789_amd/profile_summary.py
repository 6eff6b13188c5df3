"""Summaries of rocprofv3 outputs for profiles/ (kernel-trace stats and HBM counters).

Usage:
  python -m paper_2402_03789_amd.profile_summary stats <rocprof_dir> <steps[:blocks]> <out.md> <command...>
  python -m paper_2402_03789_amd.profile_summary traffic <fetch_dir> <write_dir> <kernel> \
        <source.hip> <precision> <out.json> <command...>
  python -m paper_2402_03789_amd.profile_summary utilization <pmc_dir> <out.md> <command...>

The traffic summary scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch) by the
readings of the same counters for the 256 MiB device copy that the benchmark
runs first with --calib-copy (a copy reads and writes exactly 256 MiB; the largest
copy issued before the first library kernel).  A kernel
given as NAME@UNIT is reported per dispatch of UNIT: the bytes of all NAME
dispatches divided by the number of UNIT dispatches (k_tp_bwd@k_mlp_fused_bwd: per
interaction block, since the radial-MLP adjoint runs once per block).

The stats summary also gives, for the tensor-product and radial-MLP kernels, the
GPU time per interaction block (all their dispatches of a step / the model's blocks,
5 unless given as steps:blocks).
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import sys


def _rows(d, pattern):
    files = glob.glob(f"{d}/**/{pattern}", recursive=True)
    if not files:
        raise FileNotFoundError(f"{pattern} under {d}")
    return list(csv.DictReader(open(files[0])))


def stats(d, steps, out, cmd, blocks=5):
    rows = _rows(d, "*kernel_stats.csv")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# Kernel-trace summary", "", f"Command: `{cmd}`", "",
             f"Per step = totals / {steps} profiled steps (plus warm-up launches where noted by calls).",
             "", "| kernel | calls | avg us | total ms/step | % |", "|---|---|---|---|---|"]
    for r in rows[:30]:
        name = r["Name"].split("(")[0].replace("void ", "")
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6 / steps:.3f} | {float(r['Percentage']):.2f} |")
    # device copies: the benchmark's 1 GiB copy-rate measurement and set-up uploads, outside
    # the timed steps, plus a few small position copies of each graph build
    copies = sum(float(r["TotalDurationNs"]) for r in rows if "copyBuffer" in r["Name"])
    lines += ["", f"Total GPU time per step: {total / 1e6 / steps:.3f} ms "
              f"({(total - copies) / 1e6 / steps:.3f} ms without `__amd_rocclr_copyBuffer`, "
              "most of which is the benchmark's copy-rate measurement outside the timed steps)", "",
              f"Per interaction block (sum over the kernel's instantiations per step / {blocks} "
              "blocks):", ""]
    for k in ("k_tp_bwd", "k_tp_fwd", "k_mlp_fused_bwd", "k_mlp_fused_fwd"):
        t = sum(float(r["TotalDurationNs"]) for r in rows if _is_kernel(r["Name"], k))
        lines.append(f"- `{k}`: {t / 1e3 / steps / blocks:.1f} us")
    open(out, "w").write("\n".join(lines) + "\n")


def _is_kernel(name, k):
    """Whether a demangled kernel name is kernel k: any instantiation of the template k, the
    plain function k, or its FP32 split form k_split."""
    return f"::{k}<" in name or f"::{k}(" in name or f"::{k}_split(" in name


def traffic(fetch_dir, write_dir, kernel, source, precision, out, cmd):
    f_rows = _rows(fetch_dir, "*counter_collection.csv")
    w_rows = _rows(write_dir, "*counter_collection.csv")

    def calib(rows, counter):
        # the 256 MiB calibration copy runs before the first library kernel (copies issued
        # later, of other sizes, are not calibration)
        first = min(int(r["Dispatch_Id"]) for r in rows if "sn::" in r["Kernel_Name"])
        vals = [float(r["Counter_Value"]) for r in rows
                if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]
                and int(r["Dispatch_Id"]) < first]
        return max(vals)
    cf = calib(f_rows, "FETCH_SIZE") / (256 * 1024)
    cw = calib(w_rows, "WRITE_SIZE") / (256 * 1024)
    kernel, _, unit = kernel.partition("@")
    fk = [float(r["Counter_Value"]) for r in f_rows if _is_kernel(r["Kernel_Name"], kernel)]
    wk = [float(r["Counter_Value"]) for r in w_rows if _is_kernel(r["Kernel_Name"], kernel)]
    nf = nw = len(fk)
    if unit:
        nf = sum(1 for r in f_rows if _is_kernel(r["Kernel_Name"], unit))
        nw = sum(1 for r in w_rows if _is_kernel(r["Kernel_Name"], unit))
    fetch = sum(fk) / nf / cf * 1024
    write = sum(wk) / nw / cw * 1024
    rec = {"kernel": kernel, "per": f"dispatch of {unit}" if unit else "dispatch",
           "precision": precision, "command": cmd,
           "calibration": {"fetch_KiB_per_copy_KiB": cf, "write_KiB_per_copy_KiB": cw},
           "dispatches": len(fk), "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "bytes_per_launch": fetch + write,
           "source_sha256": hashlib.sha256(open(source, "rb").read()).hexdigest()}
    json.dump(rec, open(out, "w"), indent=1)


def utilization(d, out, cmd, top=24):
    """Per-kernel matrix-core and vector-ALU utilisation from a `--pmc MfmaUtil VALUBusy
    SQ_INSTS_VALU_FLOPS_FP32 SQ_INSTS_VALU_MFMA_MOPS_*` run: the mean over a kernel's
    dispatches of MfmaUtil (matrix-core busy cycles over GPU-active cycles of every SIMD)
    and VALUBusy (vector-ALU instruction cycles over GPU-active cycles of every CU), the
    raw float32 VALU flop counter and the matrix-core MOPs per dispatch (1 MOP = 512
    flops)."""
    rows = _rows(d, "*counter_collection.csv")
    per = {}
    for r in rows:
        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
        k = per.setdefault(name, {})
        k.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    cols = ["MfmaUtil", "VALUBusy", "SQ_INSTS_VALU_FLOPS_FP32", "SQ_INSTS_VALU_MFMA_MOPS_F32",
            "SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F64"]

    def mean(v):
        return sum(v) / len(v) if v else 0.0
    def work(n):  # all flops of the kernel's dispatches
        return sum(per[n].get(cols[2], [0])) + 512 * sum(sum(per[n].get(c, [0])) for c in cols[3:])
    order = sorted(per, key=lambda n: -work(n))
    lines = ["# Matrix-core and vector-ALU utilisation per kernel", "", f"Command: `{cmd}`", "",
             "MfmaUtil and VALUBusy: percent, mean over the kernel's dispatches (rocprofv3 derived "
             "counters: SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE x SIMDs) and "
             "SQ_ACTIVE_INST_VALU / (CUs x GRBM_GUI_ACTIVE)); the float32 VALU flop counter "
             "(SQ_INSTS_VALU_FLOPS_FP32, raw, 1e9 counts) and the matrix-core MOPs (x 512 flops) "
             "per dispatch.", "",
             "| kernel | dispatches | MfmaUtil % | VALUBusy % | FP32 VALU counter (G) | MFMA F32 GFLOP "
             "| MFMA BF16 GFLOP | MFMA F64 GFLOP |", "|---|---|---|---|---|---|---|---|"]
    for n in order[:top]:
        k = per[n]
        nd = max(len(v) for v in k.values())
        lines.append(f"| `{n}` | {nd} | {mean(k.get('MfmaUtil', [])):.1f} | "
                     f"{mean(k.get('VALUBusy', [])):.1f} | "
                     f"{mean(k.get('SQ_INSTS_VALU_FLOPS_FP32', [])) / 1e9:.2f} | "
                     + " | ".join(f"{512 * mean(k.get(c, [])) / 1e9:.2f}" for c in cols[3:]) + " |")
    open(out, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        steps, _, blocks = sys.argv[3].partition(":")
        stats(sys.argv[2], float(steps), sys.argv[4], " ".join(sys.argv[5:]),
              int(blocks) if blocks else 5)
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:8], " ".join(sys.argv[8:]))
    elif sys.argv[1] == "utilization":
        utilization(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
