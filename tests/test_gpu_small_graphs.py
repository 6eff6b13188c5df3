"""Graph sizes on both sides of the small-graph launch choices, against the FP64 oracle.

Below 2,048 receivers the tensor-product adjoint spreads each receiver's edges over 2, 4
or 8 waves (switching at 1,024, 512 and 256 receivers); the channel-mixing GEMMs of one
layer share a launch while they span at most 1,024 tiles; the radial-MLP forward splits
its output panels over blocks when there are few pairs.  Each size runs the real-size
model in the FP64 form (bit-level paths, 1e-10) and the FP32 form (FP32 bounds).
"""
import pytest

from gpu_common import (TOL_E_REL_FP32, TOL_E_REL_FP64, TOL_F_ABS_FP32, TOL_F_ABS_FP64,
                        TOL_W_REL_FP32, errors, log, write_model)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2402_03789_amd as sn  # noqa: E402
from oracle.model import OracleModel, evaluate  # noqa: E402
from synth import model_spec_real, sio2_box  # noqa: E402


@pytest.fixture(scope="module")
def real_model(tmp_path_factory):
    spec = model_spec_real()
    path, w = write_model(tmp_path_factory.mktemp("m"), spec, 102)
    return path, OracleModel(spec.config(), w)


# 96 atoms: 8 waves per receiver; 300: 4; 600: 2; 1,200: 1 (and GEMM groups above 1,024 tiles)
@pytest.mark.parametrize("n_si", [32, 100, 200, 400])
def test_small_graph_regimes_match_oracle(real_model, n_si):
    path, om = real_model
    s = sio2_box(n_si, seed=20 + n_si)
    ref = evaluate(om, s.pos, s.Z, s.cell)
    model = sn.Model(path)
    for precision in ("fp64", "fp32"):
        got = sn.Context(model, precision=precision).compute(s.pos, s.Z, s.cell)
        err = errors(got, ref)
        log(f"small graph n={s.n} {precision}: {err}")
        if precision == "fp64":
            assert err["e_rel"] < TOL_E_REL_FP64 and err["f_abs"] < TOL_F_ABS_FP64
        else:
            assert err["e_rel"] < TOL_E_REL_FP32 and err["f_abs"] < TOL_F_ABS_FP32
            assert err["w_rel"] < TOL_W_REL_FP32


@pytest.mark.parametrize("precision,w_asym", [("fp64", 1e-12), ("fp32", 1e-8), ("bf16", 1e-4)])
def test_force_sum_and_virial_symmetry(real_model, precision, w_asym):
    # every edge gradient g_e enters its receiver's force with + and its sender's owner's
    # with -, so the forces sum to zero up to rounding of float64 sums in every form; the
    # virial is symmetric as far as the arithmetic keeps the energy rotation-invariant
    import numpy as np
    path, _ = real_model
    s = sio2_box(200, seed=31)
    got = sn.Context(sn.Model(path), precision=precision).compute(s.pos, s.Z, s.cell)
    f, w = got["forces"], got["virial"]
    f_rms = float(np.sqrt(np.mean(f ** 2)))
    sum_f = np.abs(f.sum(axis=0)).max()
    asym = np.linalg.norm(w - w.T) / np.linalg.norm(w)
    log(f"{precision}: |sum F| {sum_f:.3g} (rms F {f_rms:.3g}), virial asymmetry {asym:.3g}")
    assert sum_f < 1e-9 * f_rms * len(f)
    assert asym < w_asym
