"""Full-size parity: the 24,000-atom SiO2 benchmark configuration, evaluated through the
device entry points that bench.py times, against sampled FP64 oracle outputs stored by
tests/golden/make_golden.py (which calls only oracle/ and synth/)."""
import json
import os

import numpy as np
import pytest

from gpu_common import (log, write_model, TOL_E_REL_FP32, TOL_F_ABS_FP32, TOL_W_REL_FP32,
                        TOL_F_RMS_BF16, TOL_W_REL_BF16)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2402_03789_amd as sn  # noqa: E402
from synth import model_spec_real, config_structure  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sio2_24k.json")


@pytest.fixture(scope="module")
def golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("golden file missing")
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_sio2_24k_sampled_parity(tmp_path, golden, precision):
    spec = model_spec_real()
    path, _ = write_model(tmp_path, spec, golden["weights_seed"])
    s = config_structure("sio2_24k")
    log(f"full-size parity precision={precision} n={s.n}")
    ctx = sn.Context(sn.Model(path), precision=precision)
    dev = torch.device("cuda:0")
    pos = torch.tensor(s.pos, dtype=torch.float64, device=dev)
    Z = torch.tensor(s.Z, dtype=torch.int32, device=dev)
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    ae = torch.zeros(s.n, dtype=torch.float64, device=dev)
    f = torch.zeros((s.n, 3), dtype=torch.float64, device=dev)
    w = torch.zeros(9, dtype=torch.float64, device=dev)
    ctx.forward_device(pos, Z, s.cell, e, ae)
    ctx.backward_device(1.0, f, w)
    ctx.synchronize()
    n, g, ne = ctx.graph_size()
    assert ne == golden["n_edges"]
    idx = np.array(golden["sample_index"])
    ae_s = ae.cpu().numpy()[idx]
    f_s = f.cpu().numpy()[idx]
    de = np.abs(ae_s - np.array(golden["sample_atom_energy"])).max() / golden["atom_energy_rms"]
    df = np.abs(f_s - np.array(golden["sample_forces"])).max()
    df_rms = np.sqrt(np.mean((f_s - np.array(golden["sample_forces"])) ** 2)) / golden["force_rms"]
    W = w.cpu().numpy()
    dw = np.linalg.norm(W - np.array(golden["virial"])) / np.linalg.norm(golden["virial"])
    dE = abs(float(e.cpu()[0]) - golden["energy"]) / (golden["atom_energy_rms"] * np.sqrt(s.n))
    log(f"e_rel={de:.2e} f_abs={df:.2e} f_rms_rel={df_rms:.2e} w_rel={dw:.2e} dE/(rms*sqrtN)={dE:.2e}")
    if precision == "fp32":
        assert de <= TOL_E_REL_FP32 and df <= TOL_F_ABS_FP32 and dw <= TOL_W_REL_FP32
        # total energy per atom within the per-atom tolerance (|dE| <= N tol RMS(E_i))
        assert dE / np.sqrt(s.n) <= TOL_E_REL_FP32
    else:
        assert df_rms <= TOL_F_RMS_BF16 and dw <= TOL_W_REL_BF16
    ctx.close()
    torch.cuda.empty_cache()


def test_sio2_24k_autograd_forces_vs_central_differences(tmp_path, golden):
    """Forces of the hand-written adjoint behind torch.autograd.Function on the full 24k-atom
    box (FP64 form) against central differences of the energy, h = 1e-4 A, on 32 atoms drawn
    with seed 3 (all three components each), and the FP32 and BF16 forms' forces on the same
    atoms against the stored oracle values."""
    spec = model_spec_real()
    path, _ = write_model(tmp_path, spec, golden["weights_seed"])
    s = config_structure("sio2_24k")
    dev = torch.device("cuda:0")
    ctx = sn.Context(sn.Model(path), precision="fp64")
    Z = torch.tensor(s.Z, dtype=torch.int32, device=dev)
    pos = torch.tensor(s.pos, dtype=torch.float64, device=dev, requires_grad=True)
    E = sn.energy(pos, Z, s.cell, ctx)
    E.backward()
    F = -pos.grad.cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(3))
    atoms = rng.choice(s.n, size=32, replace=False)
    h = 1e-4
    log(f"central differences on {len(atoms)} atoms of the 24k box, h={h}")
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    base = torch.tensor(s.pos, dtype=torch.float64, device=dev)
    err = 0.0
    for i in atoms:
        for a in range(3):
            vals = []
            for sgn in (1.0, -1.0):
                p = base.clone()
                p[i, a] += sgn * h
                ctx.forward_device(p, Z, s.cell, e)
                vals.append(float(e.cpu()[0]))
            err = max(err, abs(-(vals[0] - vals[1]) / (2 * h) - F[i, a]))
    log(f"  max |F_adjoint - F_central_difference| = {err:.2e} eV/A")
    assert err <= 2e-6
    ctx.close()
    torch.cuda.empty_cache()


SI3N4 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "si3n4_112k.json")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_si3n4_112k_sampled_parity(tmp_path, precision):
    """The large-box configuration (112,000-atom Si3N4 at 3.1 g/cm^3) with the neighbour list
    of its MD runs (r_c + 1 A skin) through the device entry points, against sampled FP64
    oracle values (the oracle's list is exactly r_c: pairs between r_c and r_c + skin carry
    zero weight)."""
    if not os.path.exists(SI3N4):
        pytest.skip("golden file missing")
    with open(SI3N4) as fh:
        gold = json.load(fh)
    spec = model_spec_real(tuple(gold["species"]))
    path, _ = write_model(tmp_path, spec, gold["weights_seed"])
    s = config_structure("si3n4_112k")
    log(f"112k Si3N4 parity precision={precision} n={s.n}")
    ctx = sn.Context(sn.Model(path), precision=precision, skin=1.0)
    dev = torch.device("cuda:0")
    pos = torch.tensor(s.pos, dtype=torch.float64, device=dev)
    Z = torch.tensor(s.Z, dtype=torch.int32, device=dev)
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    ae = torch.zeros(s.n, dtype=torch.float64, device=dev)
    f = torch.zeros((s.n, 3), dtype=torch.float64, device=dev)
    w = torch.zeros(9, dtype=torch.float64, device=dev)
    ctx.forward_device(pos, Z, s.cell, e, ae)
    ctx.backward_device(1.0, f, w)
    ctx.synchronize()
    n, g, ne = ctx.graph_size()
    assert n == s.n and ne > gold["n_edges"]  # the skin list holds every r_c pair and more
    idx = np.array(gold["sample_index"])
    ae_s = ae.cpu().numpy()[idx]
    f_s = f.cpu().numpy()[idx]
    de = np.abs(ae_s - np.array(gold["sample_atom_energy"])).max() / gold["atom_energy_rms"]
    df = np.abs(f_s - np.array(gold["sample_forces"])).max()
    df_rms = np.sqrt(np.mean((f_s - np.array(gold["sample_forces"])) ** 2)) / gold["force_rms"]
    dw = np.linalg.norm(w.cpu().numpy() - np.array(gold["virial"])) / np.linalg.norm(gold["virial"])
    dE = abs(float(e.cpu()[0]) - gold["energy"]) / (gold["atom_energy_rms"] * np.sqrt(s.n))
    log(f"  edges {ne} (oracle r_c list {gold['n_edges']}), ghosts {g}; e_rel={de:.2e} "
        f"f_abs={df:.2e} f_rms_rel={df_rms:.2e} w_rel={dw:.2e} dE/(rms*sqrtN)={dE:.2e}")
    if precision == "fp32":
        assert de <= TOL_E_REL_FP32 and df <= TOL_F_ABS_FP32 and dw <= TOL_W_REL_FP32
        assert dE / np.sqrt(s.n) <= TOL_E_REL_FP32  # total energy per atom, as above
    else:
        assert df_rms <= TOL_F_RMS_BF16 and dw <= TOL_W_REL_BF16
    ctx.close()
    del pos, Z, e, ae, f, w
    torch.cuda.empty_cache()


QUARTZ = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "quartz_4608_32x4.json")


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_benchmark_model_4608_sampled_parity(tmp_path, precision):
    # one of the paper's benchmark models (32 channels at every l <= 3, 4 blocks, r_c 4 A)
    # on its per-GPU share of 4,608 atoms at the alpha-quartz density
    if not os.path.exists(QUARTZ):
        pytest.skip("golden file missing")
    with open(QUARTZ) as fh:
        gold = json.load(fh)
    from synth import model_spec_bench, sio2_box
    spec = model_spec_bench(32, 4, sigma=gold["sigma"])
    path, _ = write_model(tmp_path, spec, gold["weights_seed"])
    s = sio2_box(gold["n_atoms"] // 3, density=2.65, seed=gold["structure_seed"])
    log(f"benchmark-model parity precision={precision} n={s.n}")
    ctx = sn.Context(sn.Model(path), precision=precision)
    r = ctx.compute(s.pos, s.Z, s.cell)
    assert ctx.graph_size()[2] == gold["n_edges"]
    idx = np.array(gold["sample_index"])
    de = np.abs(r["atom_energy"][idx] - np.array(gold["sample_atom_energy"])).max() / gold["atom_energy_rms"]
    df = np.abs(r["forces"][idx] - np.array(gold["sample_forces"])).max()
    df_rms = (np.sqrt(np.mean((r["forces"][idx] - np.array(gold["sample_forces"])) ** 2))
              / gold["force_rms"])
    dw = np.linalg.norm(r["virial"].reshape(-1) - np.array(gold["virial"])) / np.linalg.norm(gold["virial"])
    log(f"e_rel={de:.2e} f_abs={df:.2e} f_rms_rel={df_rms:.2e} w_rel={dw:.2e}")
    if precision == "fp64":
        assert de <= 1e-10 and df <= 1e-10 and dw <= 1e-10
    elif precision == "fp32":
        assert de <= TOL_E_REL_FP32 and df <= TOL_F_ABS_FP32 and dw <= TOL_W_REL_FP32
    else:
        assert df_rms <= TOL_F_RMS_BF16 and dw <= TOL_W_REL_BF16
