"""Full-size parity: the 24,000-atom SiO2 benchmark configuration, evaluated through the
device entry points that bench.py times, against sampled FP64 oracle outputs stored by
tests/golden/make_golden.py (which calls only oracle/ and synth/)."""
import json
import os

import numpy as np
import pytest

from gpu_common import log, write_model, TOL_E_REL_FP32, TOL_F_ABS_FP32, TOL_W_REL_FP32, TOL_F_RMS_BF16

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
    else:
        assert df_rms <= TOL_F_RMS_BF16
