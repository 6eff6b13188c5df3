"""GPU path vs the FP64 oracle, element by element, through the C ABI."""
import numpy as np
import pytest

from gpu_common import (log, write_model, errors, TOL_E_REL_FP32, TOL_F_ABS_FP32, TOL_W_REL_FP32,
                        TOL_E_REL_FP64, TOL_F_ABS_FP64, TOL_F_RMS_BF16, TOL_W_REL_BF16)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2402_03789_amd as sn  # noqa: E402
from oracle.model import OracleModel, evaluate  # noqa: E402
from oracle.graph import periodic_edges, wrap  # noqa: E402
from synth import (model_spec_small, model_spec_real, sio2_box, config_structure, rsa_box,  # noqa: E402
                   si3n4_box)


@pytest.fixture(scope="module")
def small_model(tmp_path_factory):
    spec = model_spec_small()
    path, w = write_model(tmp_path_factory.mktemp("m"), spec, 101)
    return spec, path, w, OracleModel(spec.config(), w)


@pytest.fixture(scope="module")
def real_model(tmp_path_factory):
    spec = model_spec_real()
    path, w = write_model(tmp_path_factory.mktemp("m"), spec, 102)
    return spec, path, w, OracleModel(spec.config(), w)


def _tri(n=24, seed=3):
    cell = np.array([[8.5, 0, 0], [2.0, 7.9, 0], [-1.5, 1.0, 8.2]])
    pos = rsa_box(cell, n, 1.4, np.random.Generator(np.random.PCG64(seed)))
    Z = np.where(np.arange(n) % 3 == 0, 14, 8).astype(np.int32)
    return pos, Z, cell


def _edge_set(recv, send, shift):
    return set(zip(recv.tolist(), send.tolist(), map(tuple, np.asarray(shift).tolist())))


@pytest.mark.parametrize("case", ["small_box", "triclinic", "tiny_cell"])
def test_graph_exact(small_model, case):
    spec, path, w, om = small_model
    if case == "small_box":
        s = config_structure("small")
        pos, Z, cell = s.pos, s.Z, s.cell
    elif case == "triclinic":
        pos, Z, cell = _tri()
    else:
        pos, Z, cell = _tri(n=3, seed=5)
        cell = cell * 0.45  # cell narrower than r_c: self-images and multiple shells
    log(f"graph case={case} n={len(Z)}")
    ctx = sn.Context(sn.Model(path), precision="fp64")
    ctx.compute(pos, Z, cell)
    g = ctx.graph()
    recv, send, shift = periodic_edges(wrap(pos, cell), cell, spec.r_cut)
    assert _edge_set(g["recv"], g["send_owner"], g["shift"]) == _edge_set(recv, send, shift)
    assert len(g["recv"]) == len(recv)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_small_config(small_model, precision):
    spec, path, w, om = small_model
    s = config_structure("small")
    log(f"small config precision={precision}")
    ctx = sn.Context(sn.Model(path), precision=precision)
    got = ctx.compute(s.pos, s.Z, s.cell)
    ref = evaluate(om, s.pos, s.Z, s.cell)
    err = errors(got, ref)
    log(str(err))
    if precision == "fp64":
        assert err["e_rel"] < TOL_E_REL_FP64 and err["f_abs"] < TOL_F_ABS_FP64
        assert err["w_rel"] < 1e-10
    else:
        assert err["e_rel"] <= TOL_E_REL_FP32 and err["f_abs"] <= TOL_F_ABS_FP32
        assert err["w_rel"] <= TOL_W_REL_FP32


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_real_model_medium_box(real_model, precision):
    spec, path, w, om = real_model
    s = sio2_box(100, seed=12)  # 300 atoms: several tiles per kernel and ragged tails
    log(f"real model medium box precision={precision} n={s.n}")
    ctx = sn.Context(sn.Model(path), precision=precision)
    got = ctx.compute(s.pos, s.Z, s.cell)
    ref = evaluate(om, s.pos, s.Z, s.cell)
    err = errors(got, ref)
    log(str(err))
    if precision == "fp64":
        assert err["e_rel"] < TOL_E_REL_FP64 and err["f_abs"] < TOL_F_ABS_FP64
    elif precision == "fp32":
        assert err["e_rel"] <= TOL_E_REL_FP32 and err["f_abs"] <= TOL_F_ABS_FP32
        assert err["w_rel"] <= TOL_W_REL_FP32
    else:
        assert err["f_rms_rel"] <= TOL_F_RMS_BF16 and err["w_rel"] <= TOL_W_REL_BF16


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_si3n4_box_with_skin(tmp_path, precision):
    """The large-box configuration's chemistry and list at a size the oracle evaluates in
    seconds: Si3N4 at 3.1 g/cm^3 (48 Si + 64 N, RSA 1.5 A plus 0.05 A jitter), the real-size
    model with N/Si species, and the r_c + 1 A skin list of the MD runs."""
    spec = model_spec_real((7, 14))
    path, w = write_model(tmp_path, spec, 102)
    om = OracleModel(spec.config(), w)
    s = si3n4_box(48, seed=9)
    log(f"Si3N4 box precision={precision} n={s.n}")
    got = sn.Context(sn.Model(path), precision=precision, skin=1.0).compute(s.pos, s.Z, s.cell)
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
        assert err["f_rms_rel"] <= TOL_F_RMS_BF16


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_real_model_triclinic_small_cell(real_model, precision):
    spec, path, w, om = real_model
    pos, Z, cell = _tri(n=20, seed=8)
    log(f"real model triclinic precision={precision}")
    ctx = sn.Context(sn.Model(path), precision=precision, skin=0.7)
    got = ctx.compute(pos, Z, cell)
    ref = evaluate(om, pos, Z, cell)
    err = errors(got, ref)
    log(str(err))
    if precision == "fp64":
        assert err["e_rel"] < TOL_E_REL_FP64 and err["f_abs"] < TOL_F_ABS_FP64
    else:
        assert err["e_rel"] <= TOL_E_REL_FP32 and err["f_abs"] <= TOL_F_ABS_FP32


def test_isolated_atoms_and_sizes(small_model):
    spec, path, w, om = small_model
    cell = np.eye(3) * 20.0
    pos = np.array([[1.0, 1.0, 1.0], [10.0, 10.0, 10.0], [10.0, 10.0, 12.0]])
    Z = np.array([8, 14, 8], dtype=np.int32)
    log("isolated atoms")
    ctx = sn.Context(sn.Model(path), precision="fp64")
    got = ctx.compute(pos, Z, cell)
    ref = evaluate(om, pos, Z, cell)
    assert np.abs(got["atom_energy"] - ref["atom_energy"]).max() < 1e-12
    np.testing.assert_allclose(got["forces"], ref["forces"], atol=1e-12)
    # one atom alone in a big cell: no edges at all
    got1 = ctx.compute(pos[:1], Z[:1], cell)
    ref1 = evaluate(om, pos[:1], Z[:1], cell)
    assert abs(got1["energy"] - ref1["energy"]) < 1e-12
    assert ctx.graph_size()[2] == 0


def test_context_reuse_growing_and_shrinking(small_model):
    spec, path, w, om = small_model
    ctx = sn.Context(sn.Model(path), precision="fp32")
    for n_si in (4, 40, 8):
        s = sio2_box(n_si, seed=30 + n_si)
        log(f"reuse n={s.n}")
        got = ctx.compute(s.pos, s.Z, s.cell)
        ref = evaluate(om, s.pos, s.Z, s.cell)
        err = errors(got, ref)
        assert err["e_rel"] <= TOL_E_REL_FP32 and err["f_abs"] <= TOL_F_ABS_FP32


def test_bitwise_determinism(real_model):
    spec, path, w, om = real_model
    s = sio2_box(60, seed=4)
    log("determinism")
    ctx = sn.Context(sn.Model(path), precision="fp32")
    a = ctx.compute(s.pos, s.Z, s.cell)
    b = ctx.compute(s.pos, s.Z, s.cell)
    assert a["energy"] == b["energy"]
    assert np.array_equal(a["forces"], b["forces"])
    assert np.array_equal(a["virial"], b["virial"])


def test_finite_differences_fp64(real_model):
    # the hand-written adjoint against central differences of the GPU energy itself
    spec, path, w, om = real_model
    pos, Z, cell = _tri(n=16, seed=11)
    log("finite differences fp64")
    ctx = sn.Context(sn.Model(path), precision="fp64")
    F = ctx.compute(pos, Z, cell)["forces"]
    h = 1e-4
    for i in (0, 5, 11):
        for a in range(3):
            p, q = pos.copy(), pos.copy()
            p[i, a] += h
            q[i, a] -= h
            fd = -(ctx.compute(p, Z, cell, forces=False, virial=False)["energy"]
                   - ctx.compute(q, Z, cell, forces=False, virial=False)["energy"]) / (2 * h)
            assert abs(fd - F[i, a]) < 1e-7 * max(1.0, abs(fd))


def test_virial_finite_strain_fp64(real_model):
    # W = -sum_e d_e (x) dE/dd_e equals -dE/d(strain) for positions and cell strained together
    spec, path, w, om = real_model
    pos, Z, cell = _tri(n=16, seed=12)
    log("virial by finite strain fp64")
    ctx = sn.Context(sn.Model(path), precision="fp64")
    W = ctx.compute(pos, Z, cell)["virial"]
    h = 1e-5
    for a in range(3):
        for b in range(3):
            E = []
            for sgn in (1, -1):
                eps = np.eye(3)
                eps[a, b] += sgn * h
                E.append(ctx.compute(pos @ eps, Z, cell @ eps, forces=False, virial=False)["energy"])
            fd = -(E[0] - E[1]) / (2 * h)
            assert abs(fd - W[a, b]) < 1e-6 * max(1.0, abs(fd)), (a, b, fd, W[a, b])


def test_errors_are_reported(small_model):
    spec, path, w, om = small_model
    ctx = sn.Context(sn.Model(path), precision="fp32")
    s = sio2_box(4, seed=2)
    log("error paths")
    bad = s.Z.copy()
    bad[0] = 79
    with pytest.raises(sn.SNError) as e:
        ctx.compute(s.pos, bad, s.cell)
    assert e.value.status == -1
    p = s.pos.copy()
    p[1] = np.nan
    with pytest.raises(sn.SNError):
        ctx.compute(p, s.Z, s.cell)
    p = s.pos.copy()
    p[1] = p[0]
    with pytest.raises(sn.SNError):
        ctx.compute(p, s.Z, s.cell)
    with pytest.raises(sn.SNError):
        ctx.compute(s.pos, s.Z, np.zeros((3, 3)))
    # the context stays usable after argument errors
    got = ctx.compute(s.pos, s.Z, s.cell)
    assert np.isfinite(got["energy"])
