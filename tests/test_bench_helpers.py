"""Host-side helpers of the benchmark and of the rocprofv3 summaries (no GPU)."""
import csv
import json
import os

import numpy as np
import pytest

from oracle.cg import real_cg
from synth import model_spec_small


def _nnz(l1, l2, l3):
    return int(np.count_nonzero(np.abs(real_cg(l1, l2, l3)) > 1e-12))


def test_tp_adjoint_flops_small_model_by_hand():
    import bench
    spec = model_spec_small()  # 3 blocks, 32x0e + 32x1e, l_sh 1
    got = bench._tp_adjoint_flops(spec, _nnz)
    # CG nonzeros of the l <= 1 couplings: (0,0,0) 1, (0,1,1) 3, (1,0,1) 3, (1,1,0) 3,
    # (1,1,1) 6 (the cross product); 9 flops per nonzero and channel (6 in the first block,
    # which writes no dE/dx), plus 3 (2 l3 + 1) per path and channel
    assert [_nnz(*p) for p in ((0, 0, 0), (0, 1, 1), (1, 0, 1), (1, 1, 0), (1, 1, 1))] == [1, 3, 3, 3, 6]
    first = 32 * (6 * 1 + 3) + 32 * (6 * 3 + 9)                 # paths (0,0,0), (0,1,1)
    middle = (32 * (9 * 1 + 3) + 32 * (9 * 3 + 9)                # l1 = 0
              + 32 * (9 * 3 + 9) + 32 * (9 * 3 + 3) + 32 * (9 * 6 + 9))  # l1 = 1
    last = 32 * (9 * 1 + 3) + 32 * (9 * 3 + 3)                   # scalar outputs only
    assert got == [first, middle, last]


def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    cols = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(cols, r)))


def test_traffic_calibrates_on_the_copy_before_the_library(tmp_path):
    from paper_2402_03789_amd import profile_summary as ps
    MiB = 1024.0  # counters are in KiB
    # the 256 MiB calibration copy reads as 128 MiB fetched and 256 MiB written; a later
    # 1 GiB copy must not be taken as the calibration
    fetch = [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 128 * MiB),
             (2, "void sn::k_tp_bwd<float, float, 1, 2, 2, false, true, 0>(...)", "FETCH_SIZE", 50 * MiB),
             (3, "void sn::k_tp_bwd<float, float, 2, 2, 2, false, true, 0>(...)", "FETCH_SIZE", 30 * MiB),
             (4, "sn::k_mlp_fused_bwd_split(long, int const*)", "FETCH_SIZE", 10 * MiB),
             (5, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 512 * MiB)]
    write = [(d, k, "WRITE_SIZE", v * 2 if "copy" in k else v) for d, k, _, v in fetch]
    _write_counters(tmp_path / "f", fetch)
    _write_counters(tmp_path / "w", write)
    src = tmp_path / "k.hip"
    src.write_text("// source")
    out = tmp_path / "t.json"
    ps.traffic(str(tmp_path / "f"), str(tmp_path / "w"), "k_tp_bwd@k_mlp_fused_bwd", str(src),
               "fp32", str(out), "cmd")
    rec = json.loads(out.read_text())
    assert rec["calibration"]["fetch_KiB_per_copy_KiB"] == pytest.approx(0.5)
    assert rec["calibration"]["write_KiB_per_copy_KiB"] == pytest.approx(1.0)
    # per dispatch of the MLP adjoint (one block): 80 MiB fetched x 2, 80 MiB written x 1
    assert rec["fetch_bytes_per_launch"] == pytest.approx(160 * 2 ** 20)
    assert rec["write_bytes_per_launch"] == pytest.approx(80 * 2 ** 20)


def test_stats_counts_split_and_plain_kernels_per_block(tmp_path):
    from paper_2402_03789_amd import profile_summary as ps
    d = tmp_path / "trace"
    d.mkdir()
    cols = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"]
    rows = [("void sn::k_mlp_fused_fwd_split(long, int const*)", 15, 7.5e6, 5e5, 40.0),
            ("sn::k_mlp_fused_bwd(long, int const*)", 15, 3e6, 2e5, 10.0),
            ("void sn::k_tp_bwd<float, float, 0, 2, 2, false, true, 0>(...)", 15, 1.5e7, 1e6, 60.0)]
    with open(d / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(cols)
        w.writerows(rows)
    out = tmp_path / "s.md"
    ps.stats(str(d), 3.0, str(out), "cmd")
    text = out.read_text()
    assert "- `k_mlp_fused_fwd`: 500.0 us" in text   # 7.5 ms / 3 steps / 5 blocks
    assert "- `k_mlp_fused_bwd`: 200.0 us" in text   # the plain (non-template) kernel
    assert "- `k_tp_bwd`: 1000.0 us" in text


def test_algorithmic_work_small_model_by_hand():
    import bench
    spec = model_spec_small()  # radial weights per edge: 64, 160, 64 over the three blocks
    n, g, e, npairs = 10, 5, 100, 50
    w = bench._algorithmic_work(spec, _nnz, n, g, e, npairs, "fp32")
    # radial MLP once per undirected pair, forward and input-gradient adjoint
    assert w["radial_mlp"]["flops"] == npairs * 2 * 2 * (3 * (8 * 64 + 64 * 64) + 64 * 288)
    # tensor product: forward + adjoint flops per edge
    fwd = bench._tp_forward_flops(spec, _nnz)
    bwd = bench._tp_adjoint_flops(spec, _nnz)
    assert w["tensor_product"]["flops"] == e * (sum(fwd) + sum(bwd))
    # first-block forward by hand: paths (0,0,0), (0,1,1): 3 flops per nonzero + 2 (2 l3 + 1)
    assert fwd[0] == 32 * (3 * 1 + 2) + 32 * (3 * 3 + 6)
    # linears: Lin1 on 15 rows in block 1, Linsc 32 -> 64 gate inputs, Lin2 mid -> outputs...
    C0 = 32
    lin1 = 2 * (n + g) * 32 * 32
    sc1 = 2 * n * 32 * 64
    assert w["linears"]["flops"] > lin1 + sc1
    r = bench._step_roofline(w, 2.0)
    for c in r["classes"].values():
        assert c["bound_ms"] == pytest.approx(max(c["flops"] / (c["peak_TFLOPs"] * 1e12),
                                                  c["bytes"] / 8e12) * 1e3)
    assert r["frac"] == pytest.approx(r["lower_bound_ms"] / 2.0)


def test_algorithmic_work_real_size_matches_the_survey_estimate():
    """At the 24k-atom configuration (818,560 edges, 409,280 pairs, 11,633 ghosts) the
    pair-shared radial MLP is 0.40 TFLOP, the tensor product about 0.22-0.26 TFLOP and the
    linears about 0.095 TFLOP per evaluation."""
    import bench
    from synth import model_spec_real
    w = bench._algorithmic_work(model_spec_real(), _nnz, 24000, 11633, 818560, 409280, "fp32")
    assert w["radial_mlp"]["flops"] / 1e12 == pytest.approx(0.40, rel=0.02)
    assert 0.21 <= w["tensor_product"]["flops"] / 1e12 <= 0.27
    assert w["linears"]["flops"] / 1e12 == pytest.approx(0.095, rel=0.05)


def test_tp_resource_guard_parses_remarks(tmp_path):
    """The build's guard over the tensor-product kernels' compiler resource remarks: float32
    kernels with harmonics up to l = 2 may use no scratch; the others stay within limits."""
    from paper_2402_03789_amd import build as b

    def rec(name, vgpr, spill, scratch):
        return (f"k.hip:1:1: remark: Function Name: {name} [-Rpass-analysis=kernel-resource-usage]\n"
                f"k.hip:1:1: remark:     VGPRs: {vgpr} [-Rpass-analysis=kernel-resource-usage]\n"
                f"k.hip:1:1: remark:     AGPRs: 0 [-Rpass-analysis=kernel-resource-usage]\n"
                f"k.hip:1:1: remark:     ScratchSize [bytes/lane]: {scratch} [-Rpass-analysis=kernel-resource-usage]\n"
                f"k.hip:1:1: remark:     VGPRs Spill: {spill} [-Rpass-analysis=kernel-resource-usage]\n")
    fp32_l2 = "_ZN2sn8k_tp_bwdIffLi1ELi2ELi2ELb0ELb1ELi0EEEvNS_6TPArgsE"
    bf16_l2 = "_ZN2sn8k_tp_fwdIfNS_6bf16_tELi2ELi2ELi2ELb0ELi64EEEvNS_6TPArgsE"
    fp64_l3 = "_ZN2sn8k_tp_fwdIddLi3ELi3ELi3ELb0ELi0EEEvNS_6TPArgsE"
    assert b._tp_kernel_kind(fp32_l2) == (True, 2)
    assert b._tp_kernel_kind(bf16_l2) == (True, 2)
    assert b._tp_kernel_kind(fp64_l3) == (False, 3)
    ok = rec(fp32_l2, 120, 0, 0) + rec(bf16_l2, 90, 0, 0) + rec(fp64_l3, 256, 10, 68)
    assert b.check_tp_resources(ok, str(tmp_path / "r.tsv")) == []
    assert (tmp_path / "r.tsv").read_text().count("\n") == 4
    bad = rec(fp32_l2, 120, 0, 36) + rec(fp64_l3, 256, 40, 200)
    assert [r["name"] for r in b.check_tp_resources(bad, str(tmp_path / "r.tsv"))] == [fp32_l2, fp64_l3]
