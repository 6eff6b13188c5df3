"""Benchmark: atom-steps/s of the E + F + virial evaluation on one MI355X.

One step = one full pass of the hot path on device-resident inputs: graph
build (cell list, ghost shell, CSRs), edge basis, 5 interaction blocks,
readout and energy sum, the hand-written adjoint through every block, edge
gradients, forces with the ghost fold, and the virial.

Workload: 24,000-atom SiO2 (8,000 Si + 16,000 O) in a periodic cubic box at
2.2 g/cm^3, seeded random sequential addition with 1.4 A minimum distance;
5-layer model with 128x0e+64x1e+32x2e features, l <= 2, 8 Bessel functions,
r_c = 5 A, radial MLP 8-64-64, seeded N(0, 1/fan_in) weights.

Prints one JSON line (rank 0).  --gpus above 1 exits: the library evaluates the
subdomains of one GPU's share on that GPU; the multi-GPU decomposition is not
implemented.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

def _traffic(kernel, source, precision):
    """Measured HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when absent or when the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{precision}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(source, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()
    if rec.get("source_sha256") != h:
        return None
    return rec.get("bytes_per_launch")


def _tp_blocks(spec):
    """(P, Dx, Dm, writes dE/dx) of every interaction block's tensor product: radial weights
    per edge, sender feature width, message width, and whether the adjoint writes per-edge
    sender gradients (not for the first block, whose inputs are the species embedding)."""
    out = []
    for t in range(spec.n_layers):
        paths = spec._paths(t)
        P = sum(spec.muls[l1] for (l1, _, _) in paths)
        Dm = sum(spec.muls[l1] * (2 * l3 + 1) for (l1, _, l3) in paths)
        Dx = sum(spec.muls[l] * (2 * l + 1) for l in spec._in_ls(t))
        out.append((P, Dx, Dm, t > 0))
    return out


def _tp_adjoint_flops(spec, cg_nnz):
    """Algorithmic arithmetic of the tensor-product adjoint per edge of each block: per path
    (l1, l2, l3) and channel, t = C x Y (3 flops per CG nonzero), dE/dw = G . t (2 (2 l3 + 1)),
    gg = w G (2 l3 + 1), dE/dx += C Y gg and dE/dY += C x gg (3 flops per nonzero each; no
    dE/dx in the first block)."""
    out = []
    for t in range(spec.n_layers):
        f = 0
        for (l1, l2, l3) in spec._paths(t):
            per_nz = 9 if t > 0 else 6
            f += spec.muls[l1] * (per_nz * cg_nnz(l1, l2, l3) + 3 * (2 * l3 + 1))
        out.append(f)
    return out


def _tp_forward_flops(spec, cg_nnz):
    """Algorithmic arithmetic of the tensor-product forward per edge of each block: per path
    (l1, l2, l3) and channel, t = C x Y (3 flops per CG nonzero) and m += w t (2 (2 l3 + 1))."""
    return [sum(spec.muls[l1] * (3 * cg_nnz(l1, l2, l3) + 2 * (2 * l3 + 1))
                for (l1, l2, l3) in spec._paths(t)) for t in range(spec.n_layers)]


def _linear_flops(spec, n, g):
    """Channel-mixing GEMM flops of one evaluation (forward and the adjoint's input
    gradients): Lin1 (block 1 also on the ghost rows), Linsc and Lin2 per degree, rows =
    atoms x (2l + 1); the adjoint repeats Lin2 in every block and Lin1, Linsc in blocks
    after the first (the first block's inputs are the species embedding); readout."""
    f = 0
    for t in range(spec.n_layers):
        paths = spec._paths(t)
        rows1 = (n + g) if t == 0 else n
        for l in spec._in_ls(t):
            m = spec.muls[l]
            fl1 = 2 * rows1 * (2 * l + 1) * m * m
            fsc = 2 * n * (2 * l + 1) * m * spec._gate_mul(t, l)
            f += fl1 + fsc + ((2 * n * (2 * l + 1) * m * m + fsc) if t > 0 else 0)
        for l in spec._out_ls(t):
            mid = sum(spec.muls[l1] for (l1, _, l3) in paths if l3 == l)
            f += 2 * 2 * n * (2 * l + 1) * mid * spec._gate_mul(t, l)
    C0 = spec.muls[0]
    return f + 2 * 2 * n * C0 * (C0 // 2)


def _algorithmic_work(spec, cg_nnz, n, g, e, npairs, precision):
    """Algorithmic flops F and minimum HBM bytes B of one E + F evaluation by work class,
    as the hot-path measurement section prices them:
      radial MLP  -- 8 -> 64 -> 64 -> P_t per undirected pair (w depends on |d| only), forward
                     and input-gradient adjoint: 2 x 2 (8 64 + 64 64 + 64 P_t) flops per pair
                     and block; bytes: the radial basis of every edge read once;
      tensor product -- per edge and block, forward 3 flops per CG nonzero and channel plus
                     2 (2 l3 + 1) per path and channel, adjoint 9 per nonzero and channel plus
                     3 (2 l3 + 1) (6 per nonzero in the first block, which has no dE/dx);
                     bytes: every sender feature row read, every message row written and its
                     adjoint read (float32), every sender's dE/dx row written (float64);
      linears     -- the channel-mixing GEMMs (forward and adjoint); bytes: node state read
                     and written once per block in each direction (float64).
    Peaks: radial MLP and linears on the matrix cores of the form's operand type (float32
    157.3 TFLOP/s; bfloat16 2,500), the tensor product on the float32 vector units (157.3),
    float64 78.6; HBM 8 TB/s."""
    b = {"fp32": 4, "bf16": 2, "fp64": 8}[precision]
    tb = 8 if precision == "fp64" else 4
    mm_peak = {"fp32": 157.3, "bf16": 2500.0, "fp64": 78.6}[precision] * 1e12
    alu_peak = (78.6 if precision == "fp64" else 157.3) * 1e12
    fwd_f = _tp_forward_flops(spec, cg_nnz)
    bwd_f = _tp_adjoint_flops(spec, cg_nnz)
    mlp_f = tp_f = tp_b = lin_b = 0
    for t, (P, Dx, Dm, wdx) in enumerate(_tp_blocks(spec)):
        mlp_f += npairs * 2 * 2 * (8 * 64 + 64 * 64 + 64 * P)
        tp_f += e * (fwd_f[t] + bwd_f[t])
        tp_b += (n + g) * Dx * b + 2 * n * Dm * tb + ((n + g) * Dx * 8 if wdx else 0)
        hin = sum(spec.muls[l] * (2 * l + 1) for l in spec._in_ls(t))
        yw = sum(spec._gate_mul(t, l) * (2 * l + 1) for l in spec._out_ls(t))
        lin_b += 2 * n * (hin + 2 * yw) * 8
    return {
        "radial_mlp": {"flops": mlp_f, "bytes": e * 8 * tb, "peak_flops": mm_peak},
        "tensor_product": {"flops": tp_f, "bytes": tp_b, "peak_flops": alu_peak},
        "linears": {"flops": _linear_flops(spec, n, g), "bytes": lin_b, "peak_flops": mm_peak},
    }


def _step_roofline(work, ms):
    """Whole-step fraction of roofline: sum over work classes of max(F/P, B/BW) against the
    measured step time (inputs resident in HBM, graph build included in the step)."""
    hbm = 8000e9
    kinds = {}
    bound = 0.0
    for k, w in work.items():
        t = max(w["flops"] / w["peak_flops"], w["bytes"] / hbm) * 1e3
        kinds[k] = {"flops": w["flops"], "bytes": w["bytes"], "peak_TFLOPs": w["peak_flops"] / 1e12,
                    "bound_ms": t}
        bound += t
    return {"bound": "sum over work classes of max(flops/peak, bytes/8 TB/s)",
            "lower_bound_ms": bound, "ms_per_step": ms, "frac": bound / ms if ms > 0 else None,
            "classes": kinds}


def _impl_traffic_entry(kernel, nbytes, ms, traffic):
    """The dominant kernel against HBM with the bytes this implementation's data layout
    makes it move (per-edge weight, dE/dw and dE/dx rows): how close the kernel runs to the
    bandwidth its own traffic needs, not an algorithmic bound."""
    achieved = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else None
    return {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
            "frac": (achieved / 8000.0) if achieved else None, "traffic": traffic,
            "launch_ms": ms, "implementation_bytes_per_launch": nbytes}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the BF16-form steps timed beside the FP32 headline")
    ap.add_argument("--no-isolated", action="store_true",
                    help="skip the evaluations after the timed steps (the single-stream context "
                         "that times the roofline kernels in isolation, the kept-list steps, "
                         "the host-buffer entry point), for kernel traces of the overlapped "
                         "steps alone")
    ap.add_argument("--cpu-sample-si", type=int, default=800,
                    help="Si count of the SiO2 sample box timed with the CPU oracle")
    ap.add_argument("--host-steps", type=int, default=5,
                    help="evaluations timed through the host-buffer entry point (0 to skip)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device copy first (HBM counter calibration)")
    ap.add_argument("--workload", default="sio2_24k",
                    choices=["sio2_24k", "md", "serving", "fd", "size_sweep", "paper_models",
                             "train"],
                    help="sio2_24k: the headline line (plus a short serving replay); md: molecular "
                         "dynamics (default the 112k-atom Si3N4 Verlet run); serving: the full "
                         "2,000-request stream; fd: the differentiation and precision report; "
                         "size_sweep: throughput against atom count; paper_models: the 20 "
                         "benchmark models (l_max 3) in NVT MD of alpha-quartz-density SiO2")
    ap.add_argument("--models", default=None,
                    help="paper_models: comma-separated CxT list (default all 20, e.g. 32x4)")
    ap.add_argument("--sweep-channels", default=None,
                    help="size_sweep: comma-separated channel counts of benchmark models (l_max 3) "
                         "to sweep instead of the l <= 2 model")
    ap.add_argument("--sweep-layers", type=int, default=4,
                    help="size_sweep: interaction blocks of the benchmark models")
    ap.add_argument("--sweep-sizes", default=None,
                    help="size_sweep: comma-separated atom counts (multiples of 3) instead of the "
                         "default ladder")
    ap.add_argument("--sizes", default="4608,12960",
                    help="paper_models: atom counts (multiples of 3)")
    ap.add_argument("--serve-requests", type=int, default=None,
                    help="requests of the serving stream to replay: default 1,000 beside the "
                         "headline line (0 to skip), 2,000 for --workload serving")
    ap.add_argument("--serve-streams", type=int, default=3)
    ap.add_argument("--serve-high-rate", type=float, default=5000.0,
                    help="second replay of the serving stream at this arrival rate (per s)")
    ap.add_argument("--domains", default="1,1,1",
                    help="nx,ny,nz spatial subdomains of the 24k-atom box, each with its own "
                         "ghost shell (halo refresh and fold in device memory)")
    ap.add_argument("--md-system", default="si3n4_112k", choices=["si3n4_112k", "sio2_24k", "sio2_192"],
                    help="MD box: the 112k-atom Si3N4 workload, or a 192-atom SiO2 box where "
                         "launch overhead matters")
    ap.add_argument("--capture", action="store_true",
                    help="MD: replay the steps between rebuilds from a recorded HIP graph")
    ap.add_argument("--md-steps", type=int, default=100)
    ap.add_argument("--md-warmup", type=int, default=10)
    ap.add_argument("--thermostat", choices=["none", "nh"], default="none",
                    help="MD: none (velocity Verlet) or one Nose-Hoover thermostat (NVT)")
    ap.add_argument("--md-temperature", type=float, default=None,
                    help="MD start (and thermostat) temperature, K; default 1500, or 300 for the "
                         "24k-atom SiO2 box")
    ap.add_argument("--md-tau", type=float, default=100.0, help="Nose-Hoover time constant, fs")
    ap.add_argument("--md-skin", type=float, default=1.0,
                    help="neighbour-list skin, A (0 with --md-rebuild 1: a fresh list every step)")
    ap.add_argument("--md-rebuild", default=None,
                    help="MD: steps between neighbour-list rebuilds (default 10), or 'skin' to "
                         "rebuild when an atom has moved more than half the skin (the default "
                         "with --paper-protocol)")
    ap.add_argument("--paper-protocol", action="store_true",
                    help="MD as in the paper's benchmarks (section 4): NVT Nose-Hoover, 210 steps "
                         "of which the last 100 are timed; the list is rebuilt on the skin trigger")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library evaluates one GPU's share on one GPU; "
                                   "--gpus must be 1"}))
        sys.exit(2)

    if args.workload == "md":
        print(json.dumps(bench_md(args)))
        return
    if args.workload == "fd":
        print(json.dumps(bench_fd(args)))
        return
    if args.workload == "train":
        print(json.dumps(bench_train(args)))
        return
    if args.workload == "size_sweep":
        print(json.dumps(bench_size_sweep(args)))
        return
    if args.workload == "paper_models":
        print(json.dumps(bench_paper_models(args)))
        return
    if args.workload == "serving":
        count = 2000 if args.serve_requests is None else args.serve_requests
        print(json.dumps(bench_serving(args, count, args.precision, full=True)))
        return

    import torch

    import paper_2402_03789_amd as sn
    from synth import model_spec_real, make_weights, write_weights, config_structure

    spec = model_spec_real()
    weights = make_weights(spec, 102)
    s = config_structure("sio2_24k")
    tmp = tempfile.mkdtemp()
    wpath = os.path.join(tmp, "model.snw")
    write_weights(wpath, spec, weights)
    domains = tuple(int(v) for v in args.domains.split(","))

    head = _run_form(args, sn, torch, wpath, spec, s, args.precision, domains, extras=True)
    bf16 = None
    if args.precision == "fp32" and not args.no_bf16:
        torch.cuda.empty_cache()
        r = _run_form(args, sn, torch, wpath, spec, s, "bf16", domains, extras=False)
        bf16 = {k: r[k] for k in ("value", "unit", "ms_per_step", "steps", "roofline",
                                  "roofline_step")}
        bf16["dtype"] = "bf16"

    cpu = None if args.no_cpu_baseline else _cpu_baseline(args, spec, weights)

    serving = None
    count = 1000 if args.serve_requests is None else args.serve_requests
    if count > 0:
        torch.cuda.empty_cache()
        serving = bench_serving(args, count, args.precision, full=False)

    out = {
        "metric": "atom-steps/s (E+F), 5-layer l<=2 model, 24k-atom SiO2",
        "value": head["value"], "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "SiO2 24,000 atoms (8,000 Si + 16,000 O), 2.2 g/cm^3, periodic cubic "
                               "71.32 A; 5 blocks 128x0e+64x1e+32x2e, l<=2, r_c 5 A; E+F+virial "
                               "as one subdomain + r_c ghost shell",
                   "n_atoms": head["n"], "n_ghost": head["g"], "n_edges": head["e"],
                   "precision": args.precision, "subdomains": list(domains)},
        "roofline": head["roofline"],
        "roofline_step": head["roofline_step"],
        "bf16": bf16,
        "cpu_baseline": cpu,
        "implementation_traffic": head.get("implementation_traffic"),
        "roofline_mlp_adjoint": head.get("roofline_mlp_adjoint"),
        "list_reused": head.get("list_reused"),
        "host_buffers": head.get("host_buffers"),
        "phases_ms": head["phases_ms"],
        "serving": serving,
    }
    print(json.dumps(out))


def _run_form(args, sn, torch, wpath, spec, s, precision, domains, extras):
    """Time `args.steps` evaluations (graph build, forward, adjoint, forces, virial) of the
    24k-atom box in one precision form on device-resident inputs, after `args.warmup`
    untimed ones, and price them against the algorithmic roofline.  With `extras`: also
    the kept-list steps, the host-buffer entry point, the single-stream (isolated) kernel
    times and the implementation-traffic figures."""
    import numpy as np

    dev = torch.device("cuda:0")
    ctx = sn.Context(sn.Model(wpath), device=0, precision=precision)
    if domains != (1, 1, 1):
        ctx.set_domains(*domains)
    pos = torch.tensor(s.pos, dtype=torch.float64, device=dev)
    Z = torch.tensor(s.Z, dtype=torch.int32, device=dev)
    energy = torch.zeros(1, dtype=torch.float64, device=dev)
    forces = torch.zeros((s.n, 3), dtype=torch.float64, device=dev)
    virial = torch.zeros(9, dtype=torch.float64, device=dev)

    def step():
        ctx.forward_device(pos, Z, s.cell, energy)
        ctx.backward_device(1.0, forces, virial)

    if args.calib_copy and extras:
        buf = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        buf.fill_(1.0)
        out_buf = buf.clone()
        torch.cuda.synchronize()
        del buf, out_buf
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    phase_ms = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        ctx.synchronize()  # collects the per-phase HIP-event timings of this step
        for k, v in ctx.timings().items():
            phase_ms[k] = phase_ms.get(k, 0.0) + v
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt / args.steps * 1e3
    n, g, e = ctx.graph_size()
    npairs = ctx.n_pairs()
    print(f"bench: {precision} {ms:.3f} ms/step", file=sys.stderr, flush=True)

    def cg_nnz(l1, l2, l3):
        return int(np.count_nonzero(np.abs(sn.cg_table(l1, l2, l3)) > 1e-12))

    # Headline roofline object: the dominant kernel, the tensor-product adjoint (k_tp_bwd).
    # Unit: the adjoint of one interaction block, i.e. its per-degree launches, which form
    # exactly the "bwd.layer<t>.tp" phase timed by HIP events on the context's stream
    # (averaged over the blocks).  Its work is vector-ALU arithmetic: per edge and block,
    # 9 flops per CG nonzero and channel (t = C x Y, dE/dx += C Y gg, dE/dY += C x gg; 6 in
    # the first block, which writes no dE/dx) plus 3 (2 l3 + 1) per path and channel
    # (dE/dw = G . t, gg = w G), nonzeros from the library's own tables, against the
    # published float32 vector peak (157.3 TFLOP/s, which counts packed two-wide FP32
    # instructions; the library builds without them, so 78.6 is what it can reach).
    blocks = _tp_blocks(spec)
    tp_phases = [f"bwd.layer{t}.tp" for t in range(len(blocks))]
    tp_ms = sum(phase_ms.get(k, 0.0) for k in tp_phases) / (len(tp_phases) * args.steps)
    flops_tp = sum(e * f for f in _tp_adjoint_flops(spec, cg_nnz)) / len(blocks)
    alu_peak = 78.6 if precision == "fp64" else 157.3
    alu_tf = flops_tp / (tp_ms * 1e-3) / 1e12 if tp_ms > 0 else None
    tp_src = os.path.join(ROOT, "paper_2402_03789_amd", "csrc", "k_tp.h")
    roofline = {"bound": "alu", "kernel": "k_tp_bwd (tensor-product adjoint; one interaction "
                                          "block = its degree launches)",
                "achieved": alu_tf, "peak": alu_peak, "unit": "TFLOP/s",
                "frac": alu_tf / alu_peak if alu_tf else None,
                "traffic": _traffic("k_tp_bwd", tp_src, precision),
                "launch_ms": tp_ms, "algorithmic_flops_per_launch": flops_tp,
                "attainable_peak_unpacked": 78.6,
                "attainable_frac": alu_tf / 78.6 if alu_tf else None}
    work = _algorithmic_work(spec, cg_nnz, n, g, e, npairs, precision)
    out = {"value": s.n * args.steps / dt, "unit": "atom-steps/s", "ms_per_step": ms,
           "steps": args.steps, "n": n, "g": g, "e": e, "roofline": roofline,
           "roofline_step": _step_roofline(work, ms),
           "phases_ms": {k: v / args.steps for k, v in phase_ms.items()}}
    if not extras:
        del ctx
        return out

    # The same evaluation with the neighbour list kept from the last build (positions
    # unchanged, so the kept graph is exact): every step without the graph build.
    list_reused = host_buffers = None
    if not args.no_isolated:
        f_ref = forces.clone()
        ctx.set_graph_reuse(True)
        step()
        ctx.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            step()
            ctx.synchronize()
        torch.cuda.synchronize()
        rdt = time.perf_counter() - t1
        ctx.set_graph_reuse(False)
        list_reused = {"steps": args.steps, "ms_per_step": rdt / args.steps * 1e3,
                       "value": s.n * args.steps / rdt, "unit": "atom-steps/s",
                       "max_abs_dF_vs_rebuild": float((forces - f_ref).abs().max())}
        del f_ref
    # The host-buffer entry point (positions in, energies, forces and virial out over PCIe,
    # one synchronisation per call): reported beside the device-resident rate, never as it.
    if args.host_steps > 0 and not args.no_isolated:
        ctx.compute(s.pos, s.Z, s.cell)
        t1 = time.perf_counter()
        for _ in range(args.host_steps):
            ctx.compute(s.pos, s.Z, s.cell)
        hdt = time.perf_counter() - t1
        host_buffers = {"entry_point": "sn_compute (host buffers)", "steps": args.host_steps,
                        "ms_per_step": hdt / args.host_steps * 1e3,
                        "value": s.n * args.host_steps / hdt, "unit": "atom-steps/s"}

    # Implementation traffic of the dominant kernel: per edge the pair's w slice read and
    # dE/dw written (2 b P_t), the dE/dx row written (b Dx_t, not in the first block), per
    # degree launch Y read and dE/dY read and written; per receiver its G rows; every
    # sender row once.  b = storage bytes of w, dE/dw, x and dE/dx (4 FP32, 2 BF16, 8 FP64).
    wbytes = {"fp32": 4, "bf16": 2, "fp64": 8}[precision]
    tbytes = 8 if precision == "fp64" else 4
    tp_bytes = [e * (2 * wbytes * P + (wbytes * Dx if wdx else 0) + 3 * 3 * 9 * tbytes)
                + n * Dm * tbytes + (n + g) * Dx * wbytes for (P, Dx, Dm, wdx) in blocks]
    impl = _impl_traffic_entry("k_tp_bwd (same unit)", sum(tp_bytes) / len(tp_bytes), tp_ms,
                               roofline["traffic"])
    # practical streaming ceiling: a 1 GiB device copy timed with events (not in counter runs)
    if not args.calib_copy:
        cbuf = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        cdst = torch.empty_like(cbuf)
        cdst.copy_(cbuf)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(5):
            cdst.copy_(cbuf)
        ev1.record()
        torch.cuda.synchronize()
        impl["copy_GBps"] = 5 * 2 * cbuf.numel() * 4 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
        impl["frac_of_copy"] = impl["achieved"] / impl["copy_GBps"] if impl["achieved"] else None
        del cbuf, cdst

    # The radial-MLP adjoint (one launch per block on the MLP stream): per pair, dE/dw of
    # both edges read (2 b P), rho read and drho written; matrix-core flops of
    # dz2 = dE/dw Wc^T and the two hidden layers' adjoints.
    Ps = [bk[0] for bk in blocks]
    mlp_phases = [f"bwd.layer{t}.mlp" for t in range(len(blocks))]
    mlp_ms = sum(phase_ms.get(k, 0.0) for k in mlp_phases) / (len(mlp_phases) * args.steps)
    P_mean = sum(Ps) / len(Ps)
    bytes_mlp = npairs * (2 * wbytes * P_mean + 64)
    flops_mlp = npairs * (2 * 64 * P_mean + 2 * (8 * 64 + 64 * 64 + 64 * 64 + 64 * 8))
    peak_tf = {"fp32": 157.3, "bf16": 2500.0, "fp64": 78.6}[precision]
    mlp_src = os.path.join(ROOT, "paper_2402_03789_amd", "csrc", "k_mlp.hip")
    roofline_mlp = _impl_traffic_entry("k_mlp_fused_bwd (radial-MLP adjoint over edge pairs)",
                                       bytes_mlp, mlp_ms,
                                       _traffic("k_mlp_fused_bwd", mlp_src, precision))
    roofline_mlp["algorithmic_flops_per_launch"] = flops_mlp
    roofline_mlp["mfma_frac"] = flops_mlp / (mlp_ms * 1e-3) / 1e12 / peak_tf if mlp_ms > 0 else None

    # The same kernels timed in isolation: a second context created with SN_SERIAL=1 runs
    # every launch on one stream (the timed steps overlap the radial MLPs with the
    # node-feature chain, which stretches the launches of both while they share the GPU).
    if not args.no_isolated:
        iso = {}
        prev = os.environ.get("SN_SERIAL")
        os.environ["SN_SERIAL"] = "1"
        sctx = sn.Context(sn.Model(wpath), device=0, precision=precision)
        if prev is None:
            del os.environ["SN_SERIAL"]
        else:
            os.environ["SN_SERIAL"] = prev
        if domains != (1, 1, 1):
            sctx.set_domains(*domains)
        for k in range(3):
            sctx.forward_device(pos, Z, s.cell, energy)
            sctx.backward_device(1.0, forces, virial)
            sctx.synchronize()
            if k > 0:
                for kk, v in sctx.timings().items():
                    iso[kk] = iso.get(kk, 0.0) + v / 2
        del sctx
        iso_tp = sum(iso.get(kk, 0.0) for kk in tp_phases) / len(tp_phases)
        if iso_tp > 0:
            roofline["isolated"] = {"launch_ms": iso_tp,
                                    "achieved": flops_tp / (iso_tp * 1e-3) / 1e12,
                                    "frac": flops_tp / (iso_tp * 1e-3) / 1e12 / alu_peak}
        iso_mlp = sum(iso.get(kk, 0.0) for kk in mlp_phases) / len(mlp_phases)
        if iso_mlp > 0:
            roofline_mlp["isolated"] = {"launch_ms": iso_mlp,
                                        "mfma_frac": flops_mlp / (iso_mlp * 1e-3) / 1e12 / peak_tf,
                                        "hbm_frac": bytes_mlp / (iso_mlp * 1e-3) / 8000e9}
        out["isolated_phases_ms"] = iso
    out.update(implementation_traffic=impl, roofline_mlp_adjoint=roofline_mlp,
               list_reused=list_reused, host_buffers=host_buffers)
    del ctx
    return out


def _cpu_baseline(args, spec, weights):
    """The FP64 oracle on this machine's host cores (every core the process may use): the
    hot path's own model on a bounded sample of the workload (an SiO2 box at the same
    density, one evaluation after a warm-up), plus the small configuration (192-atom SiO2,
    3-block l <= 1 model) timed over 5 runs.  A full 24,000-atom oracle evaluation takes
    about 9 minutes on 8 cores, so the sample keeps the benchmark within minutes."""
    import subprocess

    import torch

    from oracle.model import OracleModel, evaluate
    from synth import sio2_box, model_spec_small, make_weights as mk

    cores = len(os.sched_getaffinity(0))
    torch.set_num_threads(cores)
    model_name = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model_name = line.split(":", 1)[1].strip()
    except Exception:
        pass
    # small configuration: 1 warm-up + 5 timed runs
    sspec = model_spec_small()
    som = OracleModel(sspec.config(), mk(sspec, 101))
    small = sio2_box(64, seed=1)
    evaluate(som, small.pos, small.Z, small.cell)
    t1 = time.perf_counter()
    for _ in range(5):
        evaluate(som, small.pos, small.Z, small.cell)
    sdt = (time.perf_counter() - t1) / 5
    # the workload's model on a bounded sample
    om = OracleModel(spec.config(), weights)
    sample = sio2_box(args.cpu_sample_si, seed=2)
    t1 = time.perf_counter()
    evaluate(om, sample.pos, sample.Z, sample.cell)
    cdt = time.perf_counter() - t1
    return {"value": sample.n / cdt, "unit": "atom-steps/s", "cores": cores, "kind": "oracle",
            "cpu_model": model_name,
            "sample": f"FP64 E+F+virial of a {sample.n}-atom SiO2 box at 2.2 g/cm^3 with the "
                      f"5-block model ({cdt:.1f} s, after the small runs warmed the process); "
                      f"FP64 reference on {cores} host cores, not an optimized CPU code",
            "small_config": {"n_atoms": small.n, "runs": 5, "s_per_run": sdt,
                             "value": small.n / sdt, "unit": "atom-steps/s"}}


def _model_file(species, seed):
    from synth import model_spec_real, make_weights, write_weights
    spec = model_spec_real(species)
    path = os.path.join(tempfile.mkdtemp(), "model.snw")
    write_weights(path, spec, make_weights(spec, seed))
    return path


def bench_serving(args, count, precision, full):
    """Replay the serving stream (Poisson arrivals at 200 requests/s, 8-2,048 atoms,
    1-4 of 89 species, triclinic cells) through the continuous-batching server and
    through the plain single-structure path (one stream, one structure per launch)."""
    import paper_2402_03789_amd as sn
    from paper_2402_03789_amd.serve import Server, replay, latency_summary
    from synth import serving_stream

    t0 = time.perf_counter()
    stream = serving_stream(count=count, seed=6)
    gen_s = time.perf_counter() - t0
    model = sn.Model(_model_file(tuple(range(1, 90)), 106))
    warm = serving_stream(count=24, seed=60)
    out = {"requests": count, "offered_rate_per_s": 200.0, "precision": precision,
           "stream_seed": 6, "generation_s": gen_s}
    # the stream's own arrival rate (200/s), then the same requests arriving 25 times faster
    # (5,000/s, more work than the GPU serves), where continuous batching has to carry the load
    for name, kw in (("batched", dict(n_streams=args.serve_streams, max_batch_atoms=16384,
                                      max_batch_structures=256)),
                     ("single", dict(n_streams=1, max_batch_atoms=1 << 40,
                                     max_batch_structures=1))):
        srv = Server(model, precision=precision, **kw)
        big = max((s for _, s in warm), key=lambda s: s.n)
        srv.warmup(big.pos, big.Z, big.cell)  # every worker: workspace and kernels
        replay(srv, [(0.0, s) for _, s in warm])
        rep = replay(srv, stream)
        summ = latency_summary(rep)
        summ.update(kw)
        out[name] = summ
        rep = replay(srv, stream, time_scale=200.0 / args.serve_high_rate)
        srv.close()
        summ = latency_summary(rep)
        summ["offered_rate_per_s"] = args.serve_high_rate
        out[name + "_high_rate"] = summ
    if not full:
        return out
    atoms = out["batched"]["atoms"]
    return {"metric": "serving stream: p50/p99 latency and atom-steps/s (E+F), 5-layer l<=2 "
                      "model with 89 species",
            "value": out["batched"]["atom_steps_per_s"], "unit": "atom-steps/s", "n_gpus": 1,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": {"fp32": "f32", "bf16": "bf16", "fp64": "f64"}[precision],
            "data": "synthetic",
            "config": {"workload": f"{count} periodic structures, {atoms} atoms, Poisson "
                                   "arrivals at 200/s", "precision": precision},
            "p50_ms": out["batched"]["p50_ms"], "p99_ms": out["batched"]["p99_ms"],
            "serving": out}


def bench_fd(args):
    """Differentiation and precision report on the 24k-atom SiO2 box: forces from the
    hand-written adjoint behind torch.autograd.Function against central differences of the
    FP64 energy (h = 1e-4 A on 32 seeded atoms), and the FP32 and BF16 forms against the
    stored FP64 oracle values of 256 sampled atoms."""
    import numpy as np
    import torch

    import paper_2402_03789_amd as sn
    from synth import config_structure

    s = config_structure("sio2_24k")
    model = sn.Model(_model_file((8, 14), 102))
    dev = torch.device("cuda:0")
    Z = torch.tensor(s.Z, dtype=torch.int32, device=dev)
    ctx = sn.Context(model, precision="fp64")
    pos = torch.tensor(s.pos, dtype=torch.float64, device=dev, requires_grad=True)
    t0 = time.perf_counter()
    E = sn.energy(pos, Z, s.cell, ctx)
    E.backward()
    F = -pos.grad.cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(3))
    atoms = rng.choice(s.n, size=32, replace=False)
    h = 1e-4
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    err = 0.0
    base = torch.tensor(s.pos, dtype=torch.float64, device=dev)
    for i in atoms:
        for a in range(3):
            vals = []
            for sgn in (1.0, -1.0):
                p = base.clone()
                p[i, a] += sgn * h
                ctx.forward_device(p, Z, s.cell, e)
                vals.append(float(e.cpu()[0]))
            fd = -(vals[0] - vals[1]) / (2 * h)
            err = max(err, abs(fd - F[i, a]))
    fd_s = time.perf_counter() - t0
    out = {"metric": "force error of the hand-written adjoint (eV/A)", "workload":
           "SiO2 24,000 atoms; 5 blocks 128x0e+64x1e+32x2e, l<=2, r_c 5 A",
           "fd": {"atoms": 32, "h_A": h, "max_abs_fp64_vs_central_difference": err,
                  "seconds": fd_s}}
    gpath = os.path.join(ROOT, "tests", "golden", "sio2_24k.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            gold = json.load(f)
        idx = np.array(gold["sample_index"])
        ref = np.array(gold["sample_forces"])
        for prec in ("fp64", "fp32", "bf16"):
            c = sn.Context(model, precision=prec)
            r = c.compute(s.pos, s.Z, s.cell)
            d = r["forces"][idx] - ref
            de = np.abs(r["atom_energy"][idx] - np.array(gold["sample_atom_energy"]))
            out[prec] = {"force_max_abs": float(np.abs(d).max()),
                         "force_rms_rel": float(np.sqrt(np.mean(d ** 2)) / gold["force_rms"]),
                         "atom_energy_max_rel": float(de.max() / gold["atom_energy_rms"]),
                         "virial_rel": float(np.linalg.norm(r["virial"].ravel() - np.array(gold["virial"]))
                                             / np.linalg.norm(gold["virial"]))}
            del c
    return out


def bench_train(args):
    """Training steps of the energy term of eq 9 (paper section 5.1: batches of 16): forward in
    training mode, the Huber loss of per-atom energies against labels, and the adjoint with
    every weight gradient, on (a) 16-structure batches from the serving stream's distribution
    with the 89-species model and (b) the 24k-atom SiO2 box.  Labels are the model's own
    energies shifted by a seeded per-atom offset (synthetic: no DFT data)."""
    import numpy as np
    import torch

    import paper_2402_03789_amd as sn
    from paper_2402_03789_amd.train import energy_loss_and_grads
    from synth import config_structure, serving_stream

    out = {"metric": "training steps (energy term of eq 9, weight gradients)", "unit": "steps/s",
           "n_gpus": 1, "dtype": {"fp32": "f32", "bf16": "bf16", "fp64": "f64"}[args.precision],
           "data": "synthetic", "cases": []}
    rng = np.random.Generator(np.random.PCG64(8))
    cases = [("batch of 16 serving-stream structures, 89-species model",
              [s for _, s in serving_stream(count=16 * (args.steps + args.warmup), seed=9)],
              tuple(range(1, 90)), 16),
             ("SiO2 24,000 atoms", [config_structure("sio2_24k")], (8, 14), 1)]
    for label, pool, species, bsz in cases:
        ctx = sn.Context(sn.Model(_model_file(species, 102)), precision=args.precision)
        times, atoms = [], 0
        for k in range(args.warmup + args.steps):
            batch = [(s.pos, s.Z, s.cell) for s in pool[(k * bsz) % len(pool):(k * bsz) % len(pool) + bsz]]
            labels = [0.0] * len(batch)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = energy_loss_and_grads(ctx, batch, labels)
            torch.cuda.synchronize()
            if k >= args.warmup:
                times.append(time.perf_counter() - t0)
                atoms += sum(len(z) for _, z, _ in batch)
            del r
        dt = sum(times)
        out["cases"].append({"workload": label, "steps": len(times), "ms_per_step": dt / len(times) * 1e3,
                             "steps_per_s": len(times) / dt, "atoms_per_s": atoms / dt})
        print(f"train: {label}: {dt / len(times) * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
        del ctx
        torch.cuda.empty_cache()
    out["value"] = out["cases"][0]["steps_per_s"]
    return out


def bench_size_sweep(args):
    """One-GPU throughput against system size (the paper's single-GPU utilisation curve,
    section 4.2 and its supplementary figure): E+F+virial evaluations, graph build included.
    Default: SiO2 boxes at 2.2 g/cm^3 from 192 to 48,000 atoms with the 5-block l <= 2 model.
    With --sweep-channels: the benchmark models (l_max 3, r_c 4 A, --sweep-layers blocks) of
    each channel count on SiO2 at the alpha-quartz density, from 96 to 73,728 atoms."""
    import torch

    import paper_2402_03789_amd as sn
    from synth import model_spec_bench, model_spec_real, make_weights, write_weights, sio2_box

    tmp = tempfile.mkdtemp()
    if args.sweep_channels:
        density = 2.65
        n_si = (32, 128, 512, 1536, 4320, 12288, 24576)
        if args.sweep_sizes:
            n_si = tuple(int(v) // 3 for v in args.sweep_sizes.split(","))
        models = []
        for c in (int(v) for v in args.sweep_channels.split(",")):
            spec = model_spec_bench(c, args.sweep_layers)
            models.append((f"{c} channels, {args.sweep_layers} blocks, l_max 3", spec,
                           make_weights(spec, 300 + 10 * c + args.sweep_layers)))
    else:
        density = 2.2
        n_si = (64, 256, 1024, 4000, 8000, 16000)
        if args.sweep_sizes:
            n_si = tuple(int(v) // 3 for v in args.sweep_sizes.split(","))
        spec = model_spec_real()
        models = [("5 blocks, 128x0e+64x1e+32x2e", spec, make_weights(spec, 102))]
    dev = torch.device("cuda:0")
    boxes = {k: sio2_box(k, density=density, seed=2) for k in n_si}
    curves = []
    for label, spec, w in models:
        wpath = os.path.join(tmp, "model.snw")
        write_weights(wpath, spec, w)
        model = sn.Model(wpath)
        points = []
        for k_si in n_si:
            s = boxes[k_si]
            ctx = sn.Context(model, device=0, precision=args.precision)
            pos = torch.tensor(s.pos, dtype=torch.float64, device=dev)
            Z = torch.tensor(s.Z, dtype=torch.int32, device=dev)
            energy = torch.zeros(1, dtype=torch.float64, device=dev)
            forces = torch.zeros((s.n, 3), dtype=torch.float64, device=dev)
            virial = torch.zeros(9, dtype=torch.float64, device=dev)
            steps = max(5, min(200, int(4e5 / s.n)))
            for k in range(3 + steps):
                if k == 3:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                ctx.forward_device(pos, Z, s.cell, energy)
                ctx.backward_device(1.0, forces, virial)
            ctx.synchronize()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            points.append({"n_atoms": s.n, "steps": steps, "ms_per_step": dt / steps * 1e3,
                           "atom_steps_per_s": s.n * steps / dt, "device_bytes": ctx.memory()})
            print(f"size sweep: {label}: {s.n} atoms {dt / steps * 1e3:.2f} ms/step",
                  file=sys.stderr, flush=True)
            del ctx
        best = max(p["atom_steps_per_s"] for p in points)
        for p in points:  # throughput relative to the largest this model reaches on the sweep
            p["relative_throughput"] = p["atom_steps_per_s"] / best
        curves.append({"model": label, "points": points})
        del model
    return {"metric": "atom-steps/s (E+F) against atom count, SiO2",
            "unit": "atom-steps/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
            "dtype": {"fp32": "f32", "bf16": "bf16", "fp64": "f64"}[args.precision],
            "config": {"workload": f"SiO2 boxes at {density} g/cm^3, {3 * n_si[0]} to "
                                   f"{3 * n_si[-1]:,} atoms; one evaluation = graph build + E + F "
                                   "+ virial",
                       "precision": args.precision},
            "curves": curves, "points": curves[0]["points"]}


def bench_paper_models(args):
    """The paper's benchmark models (section 4): channels C in {4, 8, 16, 32, 64} at every degree
    l <= 3, T in {2, 3, 4, 5} interaction blocks, r_c 4 A, in NVT MD (Nose-Hoover, 300 K, dt 1 fs,
    210 steps of which the last 100 are timed) of SiO2 at the alpha-quartz density 2.65 g/cm^3,
    at the paper's one-GPU sizes of 4,608 atoms (the weak-scaling share) and 12,960 atoms (the
    strong-scaling system).  The graph is built afresh every step.  Random-packed boxes stand in
    for the crystal; each model's energy scale gives RMS forces of 1 eV/A on its start box."""
    import dataclasses

    import numpy as np
    import torch

    import paper_2402_03789_amd as sn
    from paper_2402_03789_amd.md import NoseHoover, VelocityVerlet
    from synth import make_weights, model_spec_bench, sio2_box, write_weights

    if args.models:
        family = [tuple(int(v) for v in m.split("x")) for m in args.models.split(",")]
    else:
        family = [(c, t) for c in (4, 8, 16, 32, 64) for t in (2, 3, 4, 5)]
    sizes = [int(v) for v in args.sizes.split(",")]
    if any(n % 3 for n in sizes):
        raise SystemExit("--sizes: SiO2 atom counts are multiples of 3")
    boxes = {n: sio2_box(n // 3, density=2.65, seed=7) for n in sizes}
    tmp = tempfile.mkdtemp()
    rows = []
    for c, t in family:
        spec = model_spec_bench(c, t)
        w = make_weights(spec, 300 + 10 * c + t)
        path = os.path.join(tmp, f"bench_{c}x{t}.snw")
        write_weights(path, spec, w)
        s0 = boxes[sizes[0]]
        f = sn.Context(sn.Model(path), precision=args.precision).compute(s0.pos, s0.Z, s0.cell)["forces"]
        spec = dataclasses.replace(spec, sigma=1.0 / float(np.sqrt(np.mean(f ** 2))))
        write_weights(path, spec, w)
        model = sn.Model(path)
        n_params = model.info()["n_params"]
        for n in sizes:
            s = boxes[n]
            ctx = sn.Context(model, precision=args.precision, skin=0.0)
            md = VelocityVerlet(ctx, s.pos, s.Z, s.cell, s.masses(), dt=1.0, rebuild_every=1,
                                temperature=300.0, seed=5, thermostat=NoseHoover(300.0, 100.0))
            md.run(110)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            md.run(100)
            ctx.synchronize()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            _, g, e = ctx.graph_size()
            rows.append({"channels": c, "layers": t, "n_atoms": n, "n_params": n_params,
                         "ms_per_step": dt / 100 * 1e3, "atom_steps_per_s": n * 100 / dt,
                         "n_ghost": g, "n_edges": e, "device_bytes": ctx.memory(),
                         "temperature_K": md.temperature()})
            print(f"paper models: C{c} T{t} {n} atoms {dt / 100 * 1e3:.2f} ms/step "
                  f"{ctx.memory() / 2 ** 30:.2f} GiB", file=sys.stderr, flush=True)
            del md, ctx
        del model
    return {"metric": "atom-steps/s (E+F) of NVT MD per benchmark model (l_max 3, r_c 4 A)",
            "unit": "atom-steps/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
            "dtype": {"fp32": "f32", "bf16": "bf16", "fp64": "f64"}[args.precision],
            "config": {"workload": "SiO2 at 2.65 g/cm^3 (random packing, all pairs >= 1.4 A apart), "
                                   "NVT Nose-Hoover 300 K, tau 100 fs, dt 1 fs, 110 warm-up + "
                                   "100 timed steps, graph rebuilt every step",
                       "sizes": sizes, "precision": args.precision},
            "models": rows}


def bench_md(args):
    """Molecular dynamics on device-resident arrays.  Default: 112,000-atom amorphous-density
    Si3N4, velocity Verlet at dt = 1 fs from a 1500 K Maxwell-Boltzmann start, neighbour list
    (skin 1 A) rebuilt every 10 steps.  Options: the 24k-atom SiO2 box or a 192-atom SiO2
    box, a Nose-Hoover thermostat, the skin-triggered rebuild, and the paper's benchmark
    protocol (NVT, 210 steps, the last 100 timed)."""
    import torch

    import paper_2402_03789_amd as sn
    from paper_2402_03789_amd.md import NoseHoover, VelocityVerlet
    from synth import config_structure, sio2_box

    if args.paper_protocol:
        args.thermostat, args.md_warmup, args.md_steps = "nh", 110, 100
    if args.md_rebuild is None:
        args.md_rebuild = "skin" if args.paper_protocol else "10"
    t0 = time.perf_counter()
    system = args.md_system
    if system == "sio2_192":
        s = sio2_box(64, seed=1)
    else:
        s = config_structure(system)
    gen_s = time.perf_counter() - t0
    species = (7, 14) if system == "si3n4_112k" else (8, 14)
    temp = args.md_temperature or (300.0 if system == "sio2_24k" else 1500.0)
    every = None if args.md_rebuild == "skin" else int(args.md_rebuild)
    thermo = NoseHoover(temp, args.md_tau) if args.thermostat == "nh" else None
    ctx = sn.Context(sn.Model(_model_file(species, 102)), precision=args.precision,
                     skin=args.md_skin)
    md = VelocityVerlet(ctx, s.pos, s.Z, s.cell, s.masses(), dt=1.0, rebuild_every=every,
                        temperature=temp, seed=5, capture=args.capture, thermostat=thermo)
    md.run(args.md_warmup)
    e0 = md.conserved_energy()
    r0 = md.rebuilds
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    md.run(args.md_steps)
    ctx.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    e1 = md.conserved_energy()
    n, g, e = ctx.graph_size()
    e_eval, _ = ctx.evaluated_edges()  # the list compacted to the pairs inside r_c
    workload = {"sio2_192": "SiO2 192 atoms, 2.2 g/cm^3, periodic cubic 14.26 A",
                "sio2_24k": "SiO2 24,000 atoms (8,000 Si + 16,000 O), 2.2 g/cm^3, periodic "
                            "cubic 71.32 A",
                "si3n4_112k": "Si3N4 112,000 atoms (48,000 Si + 64,000 N), 3.1 g/cm^3, periodic "
                              "cubic 106.33 A"}[system]
    ens = (f"NVT Nose-Hoover {temp:g} K, tau {args.md_tau:g} fs" if thermo else
           f"NVE from a {temp:g} K start")
    reb = ("rebuild when an atom moved > skin/2" if every is None else
           f"rebuild every {every} steps")
    return {"metric": f"atom-steps/s (E+F), 5-layer l<=2 model, {s.n}-atom MD",
            "value": s.n * args.md_steps / dt, "unit": "atom-steps/s", "n_gpus": 1,
            "steps": args.md_steps, "warmup": args.md_warmup,
            "ms_per_step": dt / args.md_steps * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": {"fp32": "f32", "bf16": "bf16", "fp64": "f64"}[args.precision],
            "data": "synthetic",
            "config": {"workload": f"{workload}; dt 1 fs, {ens}, skin {args.md_skin:g} A, {reb}",
                       "n_atoms": n, "n_ghost": g, "n_edges": e,
                       "n_edges_evaluated_last_step": e_eval, "precision": args.precision,
                       "graph_replay": bool(args.capture), "thermostat": args.thermostat,
                       "rebuild": args.md_rebuild},
            "rebuilds_timed": md.rebuilds - r0, "temperature_K": md.temperature(),
            "conserved_energy_drift_eV_per_atom": (e1 - e0) / s.n, "generation_s": gen_s}


if __name__ == "__main__":
    main()
