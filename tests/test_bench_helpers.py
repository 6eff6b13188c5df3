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
             (4, "void sn::k_mlp_fused_bwd<false>(...)", "FETCH_SIZE", 10 * MiB),
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


def test_stats_counts_the_split_forward_per_block(tmp_path):
    from paper_2402_03789_amd import profile_summary as ps
    d = tmp_path / "trace"
    d.mkdir()
    cols = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"]
    rows = [("void sn::k_mlp_fused_fwd_split(long, int const*)", 15, 7.5e6, 5e5, 40.0),
            ("void sn::k_tp_bwd<float, float, 0, 2, 2, false, true, 0>(...)", 15, 1.5e7, 1e6, 60.0)]
    with open(d / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(cols)
        w.writerows(rows)
    out = tmp_path / "s.md"
    ps.stats(str(d), 3.0, str(out), "cmd")
    text = out.read_text()
    assert "- `k_mlp_fused_fwd`: 500.0 us" in text   # 7.5 ms / 3 steps / 5 blocks
    assert "- `k_tp_bwd`: 1000.0 us" in text


def test_step_roofline_small_model_by_hand():
    import bench
    spec = model_spec_small()  # radial weights per edge: 64, 160, 64 over the three blocks
    n, g, e, npairs = 10, 5, 100, 50
    r = bench._step_roofline(spec, _nnz, n, g, e, npairs, "fp32", 1.0, {})
    k = r["kernels"]
    # forward MLP: 2 (8 64 + 64 64 + 64 P) flops and 4 P + 32 bytes per pair, summed over blocks
    assert k["mlp_fwd"]["flops"] == npairs * 2 * (3 * (8 * 64 + 64 * 64) + 64 * 288)
    assert k["mlp_fwd"]["bytes"] == npairs * (4 * 288 + 3 * 32)
    # each kernel bounded by the slower of its arithmetic and its HBM bytes
    for kind in k.values():
        assert kind["bound_ms"] >= kind["bytes"] / 8e12 * 1e3 - 1e-15
    # dE/dx rows exist from the second block on; sender rows: the first block's are the
    # 32 scalars, then 32 scalars + 32 vectors (128 floats)
    assert k["sender_fold"]["bytes"] == sum(e * D * 4 + 2 * (n + g) * D * 8 + n * D * 8
                                            for D in (128, 128))
    assert r["frac"] == pytest.approx(r["lower_bound_ms"] / 1.0)
    assert r["modelled_share"] is None
