"""Scalar degrees of 65-128 channels take two channels per lane in the tensor-product
kernels: adjacent pairs (2u, 2u + 1) in the FP32 and BF16 forms (channel counts are
multiples of 4, so every row offset is even), u and u + 64 on a 64-lane slot in the FP64
form.  The benchmark model (128 scalar channels) takes the pairs at full occupancy; these
models cover partial slots against the FP64 oracle: 96 and 72 scalar channels (48 and 36
of the 64 lanes active in the paired map)."""
import pytest

from gpu_common import (log, write_model, errors, TOL_E_REL_FP32, TOL_F_ABS_FP32, TOL_W_REL_FP32,
                        TOL_E_REL_FP64, TOL_F_ABS_FP64, TOL_F_RMS_BF16, TOL_W_REL_BF16)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2402_03789_amd as sn  # noqa: E402
from oracle.model import OracleModel, evaluate  # noqa: E402
from synth import ModelSpec, sio2_box  # noqa: E402
from synth.weights import SIGMA_SMALL, _number_density_kavg, _SIO2_NUMBER_DENSITY  # noqa: E402


def _spec(c0):
    return ModelSpec(n_layers=2, muls=(c0, 8), l_sh=1, r_cut=4.0, species=(8, 14),
                     k_avg=_number_density_kavg(192, 192 / _SIO2_NUMBER_DENSITY, 4.0),
                     sigma=SIGMA_SMALL)


_MODELS = {}


def _model(c0, tmp_path_factory):
    if c0 not in _MODELS:
        spec = _spec(c0)
        path, w = write_model(tmp_path_factory.mktemp("m"), spec, 400 + c0)
        _MODELS[c0] = (path, OracleModel(spec.config(), w))
    return _MODELS[c0]


@pytest.mark.parametrize("c0,precision", [(96, "fp64"), (96, "fp32"), (96, "bf16"), (72, "fp32")])
def test_two_channel_lane_maps(c0, precision, tmp_path_factory):
    path, om = _model(c0, tmp_path_factory)
    s = sio2_box(32, seed=21)  # 96 atoms
    log(f"scalar channels={c0} precision={precision} n={s.n}")
    ctx = sn.Context(sn.Model(path), precision=precision)
    got = ctx.compute(s.pos, s.Z, s.cell)
    ref = evaluate(om, s.pos, s.Z, s.cell)
    err = errors(got, ref)
    log(str(err))
    if precision == "fp64":
        assert err["e_rel"] < TOL_E_REL_FP64 and err["f_abs"] < TOL_F_ABS_FP64
        assert err["w_rel"] < 1e-10
    elif precision == "fp32":
        assert err["e_rel"] <= TOL_E_REL_FP32 and err["f_abs"] <= TOL_F_ABS_FP32
        assert err["w_rel"] <= TOL_W_REL_FP32
    else:
        assert err["f_rms_rel"] <= TOL_F_RMS_BF16 and err["w_rel"] <= TOL_W_REL_BF16
