"""Pins of the oracle model: counts, invariances, finite differences, special cases.

The paper prints no worked numeric example, so absolute energies for given
weights are "parity unpinned"; everything else is pinned here against facts
that do not depend on the oracle's own code.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle.model import OracleModel, evaluate, evaluate_ghost, evaluate_subdomains
from synth import (model_spec_small, model_spec_real, make_weights, sio2_box, rsa_box,
                   ACT_SCALE)


def _small_model(seed=101, **over):
    spec = model_spec_small()
    for k, v in over.items():
        setattr(spec, k, v)
    return OracleModel(spec.config(), make_weights(spec, seed)), spec


def _real_model(seed=102, species=(8, 14)):
    spec = model_spec_real(species)
    return OracleModel(spec.config(), make_weights(spec, seed)), spec


def _tiny_sio2(seed=21, n_si=8):
    return sio2_box(n_si, seed=seed)


def _tri_struct(seed=5, n=16):
    cell = np.array([[7.0, 0, 0], [1.5, 6.5, 0], [-1.0, 2.0, 6.8]])
    pos = rsa_box(cell, n, 1.4, np.random.Generator(np.random.PCG64(seed)))
    Z = np.where(np.arange(n) % 3 == 0, 14, 8).astype(np.int32)
    return pos, Z, cell


def test_parameter_count_matches_paper():
    # section 5.1: 0.84 million parameters for the 89-element model
    m, _ = _real_model(species=tuple(range(1, 90)))
    assert m.n_params() == 842_432
    assert _real_model()[0].n_params() == 831_296
    assert _small_model()[0].n_params() == 56_400


@pytest.mark.parametrize("which", ["small", "real"])
def test_translation_rotation_permutation(which):
    m = _small_model()[0] if which == "small" else _real_model()[0]
    pos, Z, cell = _tri_struct()
    r0 = evaluate(m, pos, Z, cell)
    # translation
    r1 = evaluate(m, pos + np.array([0.3, -1.7, 2.2]), Z, cell)
    assert abs(r1["energy"] - r0["energy"]) < 1e-10
    np.testing.assert_allclose(r1["forces"], r0["forces"], atol=1e-10)
    # proper rotation of positions and cell
    R = Rotation.random(random_state=3).as_matrix()
    r2 = evaluate(m, pos @ R.T, Z, cell @ R.T)
    assert abs(r2["energy"] - r0["energy"]) < 1e-10
    np.testing.assert_allclose(r2["forces"], r0["forces"] @ R.T, atol=1e-10)
    np.testing.assert_allclose(r2["virial"], R @ r0["virial"] @ R.T, atol=1e-9)
    # permutation
    perm = np.random.default_rng(0).permutation(len(Z))
    r3 = evaluate(m, pos[perm], Z[perm], cell)
    assert abs(r3["energy"] - r0["energy"]) < 1e-10
    np.testing.assert_allclose(r3["forces"], r0["forces"][perm], atol=1e-10)
    np.testing.assert_allclose(r3["atom_energy"], r0["atom_energy"][perm], atol=1e-12)


@pytest.mark.parametrize("which", ["small", "real"])
def test_forces_sum_to_zero_and_match_autograd(which):
    m = _small_model()[0] if which == "small" else _real_model()[0]
    pos, Z, cell = _tri_struct(seed=6)
    r = evaluate(m, pos, Z, cell)
    np.testing.assert_allclose(r["forces"].sum(0), 0.0, atol=1e-11)
    # eqs 5-6 (edge-force assembly) equal the direct gradient (eq 2)
    np.testing.assert_allclose(r["forces"], r["forces_autograd"], atol=1e-12)
    np.testing.assert_allclose(r["virial"], r["virial"].T, atol=1e-11)


@pytest.mark.parametrize("which", ["small", "real"])
def test_forces_central_differences(which):
    m = _small_model()[0] if which == "small" else _real_model()[0]
    pos, Z, cell = _tri_struct(seed=7, n=12)
    r = evaluate(m, pos, Z, cell)
    h = 1e-4
    rng = np.random.default_rng(3)
    for i in rng.choice(len(Z), size=4, replace=False):
        for a in range(3):
            p, q = pos.copy(), pos.copy()
            p[i, a] += h
            q[i, a] -= h
            fd = -(evaluate(m, p, Z, cell)["energy"] - evaluate(m, q, Z, cell)["energy"]) / (2 * h)
            assert abs(fd - r["forces"][i, a]) < 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("which", ["small", "real"])
def test_virial_strain_differences(which):
    m = _small_model()[0] if which == "small" else _real_model()[0]
    pos, Z, cell = _tri_struct(seed=8, n=12)
    W = evaluate(m, pos, Z, cell)["virial"]
    h = 1e-5
    for a in range(3):
        for b in range(3):
            eps = np.zeros((3, 3))
            eps[a, b] = h
            Fp = np.eye(3) + eps
            Fm = np.eye(3) - eps
            ep = evaluate(m, pos @ Fp.T, Z, cell @ Fp.T)["energy"]
            em = evaluate(m, pos @ Fm.T, Z, cell @ Fm.T)["energy"]
            assert abs(-(ep - em) / (2 * h) - W[a, b]) < 1e-6 * max(1.0, abs(W[a, b]))


@pytest.mark.parametrize("which", ["small", "real"])
def test_ghost_shell_equals_whole_box(which):
    # section 2.2 / 3.1: communication routines do not alter the outputs
    m = _small_model()[0] if which == "small" else _real_model()[0]
    pos, Z, cell = _tri_struct(seed=9)
    r = evaluate(m, pos, Z, cell)
    for skin in (0.0, 1.0):
        g = evaluate_ghost(m, pos, Z, cell, skin=skin)
        assert abs(g["energy"] - r["energy"]) < 1e-11
        np.testing.assert_allclose(g["atom_energy"], r["atom_energy"], atol=1e-12)
        np.testing.assert_allclose(g["forces"], r["forces"], atol=1e-11)
        np.testing.assert_allclose(g["virial"], r["virial"], atol=1e-10)


@pytest.mark.parametrize("splits", [(2, 1, 1), (2, 2, 2)])
def test_subdomain_emulation(splits):
    m = _small_model()[0]
    s = _tiny_sio2(n_si=16)
    r = evaluate(m, s.pos, s.Z, s.cell)
    d = evaluate_subdomains(m, s.pos, s.Z, s.cell, splits)
    assert abs(d["energy"] - r["energy"]) < 1e-10
    np.testing.assert_allclose(d["atom_energy"], r["atom_energy"], atol=1e-12)
    np.testing.assert_allclose(d["forces"], r["forces"], atol=1e-11)


def _phi(z):
    return ACT_SCALE * z / (1.0 + np.exp(-z))


@pytest.mark.parametrize("which", ["small", "real"])
def test_isolated_atom_by_hand(which):
    # no neighbours: messages vanish, so each block is y = Linsc(h) then the gate
    m, spec = _small_model() if which == "small" else _real_model()
    w = make_weights(spec, 101 if which == "small" else 102)
    cell = np.eye(3) * 30.0
    pos = np.array([[1.0, 2.0, 3.0], [16.0, 17.0, 18.0]])
    Z = np.array([14, 8], dtype=np.int32)
    r = evaluate(m, pos, Z, cell)
    C0 = spec.muls[0]
    for k, s in enumerate([1, 0]):   # species rows are (O, Si)
        h = w["embed"][s]
        for t in range(spec.n_layers):
            y = h @ w[f"l{t}.linsc.0"]
            h = _phi(y[:C0]) if t < spec.n_layers - 1 else _phi(y)
        e = spec.sigma * float((h @ w["readout.0"] @ w["readout.1"])[0])
        assert abs(r["atom_energy"][k] - e) < 1e-12
    np.testing.assert_allclose(r["forces"], 0.0, atol=1e-14)


def test_dimer_first_block_by_hand():
    # one-block model on a dimer along z: the message is the tensor product of
    # the neighbour's features with Y(z) = (1; 0, sqrt3, 0) times the radial weights
    spec = model_spec_small()
    spec.n_layers = 1
    w = make_weights(spec, 5)
    m = OracleModel(spec.config(), w)
    r0 = 2.3
    cell = np.eye(3) * 40.0
    pos = np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 5.0 + r0]])
    Z = np.array([8, 14], dtype=np.int32)
    res = evaluate(m, pos, Z, cell)
    rc = spec.r_cut
    n = np.arange(1, 9)
    x = r0 / rc
    u = 1 - 28 * x ** 6 + 48 * x ** 7 - 21 * x ** 8
    rho = (2 / rc) * np.sin(n * np.pi * r0 / rc) / r0 * u
    wts = _phi(_phi(rho @ w["l0.mlp.0"]) @ w["l0.mlp.1"]) @ w["l0.mlp.2"]
    # last (only) block keeps the scalar path (0,0,0): C = 1
    for k, (s_self, s_nb) in enumerate([(0, 1), (1, 0)]):
        xn = w["embed"][s_nb] @ w["l0.lin1.0"]
        M = wts[:32] * xn / spec.k_avg
        y = M @ w["l0.lin2.0"] + w["embed"][s_self] @ w["l0.linsc.0"]
        e = spec.sigma * float((_phi(y) @ w["readout.0"] @ w["readout.1"])[0])
        assert abs(res["atom_energy"][k] - e) < 1e-12


def test_dimer_smooth_at_cutoff():
    m, spec = _small_model()
    cell = np.eye(3) * 40.0
    Z = np.array([8, 14], dtype=np.int32)
    iso = evaluate(m, np.array([[5.0, 5, 5], [25.0, 25, 25]]), Z, cell)["energy"]
    for r0 in (4.0, 4.5):
        res = evaluate(m, np.array([[5.0, 5, 5], [5.0, 5, 5 + r0]]), Z, cell)
        assert abs(res["energy"] - iso) < 1e-14
        np.testing.assert_allclose(res["forces"], 0.0, atol=1e-14)
    e_in = evaluate(m, np.array([[5.0, 5, 5], [5.0, 5, 5 + 3.999]]), Z, cell)["energy"]
    assert abs(e_in - iso) < 1e-9
