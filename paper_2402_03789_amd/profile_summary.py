"""Summaries of rocprofv3 outputs for profiles/ (kernel-trace stats and HBM counters).

Usage:
  python -m paper_2402_03789_amd.profile_summary stats <rocprof_dir> <steps[:blocks]> <out.md> <command...>
  python -m paper_2402_03789_amd.profile_summary traffic <fetch_dir> <write_dir> <kernel> \
        <source.hip> <precision> <out.json> <command...>

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
    # (the FP32 form's radial-MLP forward is the non-template k_mlp_fused_fwd_split)
    for k in ("k_tp_bwd", "k_tp_fwd", "k_mlp_fused_bwd", "k_mlp_fused_fwd"):
        t = sum(float(r["TotalDurationNs"]) for r in rows
                if f"::{k}<" in r["Name"] or f"::{k}_split(" in r["Name"])
        lines.append(f"- `{k}`: {t / 1e3 / steps / blocks:.1f} us")
    open(out, "w").write("\n".join(lines) + "\n")


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
    fk = [float(r["Counter_Value"]) for r in f_rows if f"::{kernel}<" in r["Kernel_Name"]]
    wk = [float(r["Counter_Value"]) for r in w_rows if f"::{kernel}<" in r["Kernel_Name"]]
    nf = nw = len(fk)
    if unit:
        nf = sum(1 for r in f_rows if f"::{unit}<" in r["Kernel_Name"])
        nw = sum(1 for r in w_rows if f"::{unit}<" in r["Kernel_Name"])
    fetch = sum(fk) / nf / cf * 1024
    write = sum(wk) / nw / cw * 1024
    rec = {"kernel": kernel, "per": f"dispatch of {unit}" if unit else "dispatch",
           "precision": precision, "command": cmd,
           "calibration": {"fetch_KiB_per_copy_KiB": cf, "write_KiB_per_copy_KiB": cw},
           "dispatches": len(fk), "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "bytes_per_launch": fetch + write,
           "source_sha256": hashlib.sha256(open(source, "rb").read()).hexdigest()}
    json.dump(rec, open(out, "w"), indent=1)


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        steps, _, blocks = sys.argv[3].partition(":")
        stats(sys.argv[2], float(steps), sys.argv[4], " ".join(sys.argv[5:]),
              int(blocks) if blocks else 5)
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:8], " ".join(sys.argv[8:]))
