"""Pins of the training-loss oracle (paper eq 9, energy term): the Huber function's closed
form, the loss's derivative with respect to each structure's energy, and the weight
gradients against central finite differences of the loss (no autograd on that side)."""
import numpy as np
import pytest
import torch

from oracle.model import OracleModel
from oracle.train import energy_loss, full_loss, huber, huber_grad
from synth import model_spec_small, model_spec_real, make_weights, sio2_box


def test_huber_closed_form():
    d = 0.01
    r = torch.tensor([0.5 * d, -0.5 * d, 2 * d, -3 * d, d], dtype=torch.float64)
    want = [0.125 * d * d, 0.125 * d * d, 1.5 * d * d, 2.5 * d * d, 0.5 * d * d]
    np.testing.assert_allclose(huber(r, d).numpy(), want, rtol=1e-15)
    # value and slope are continuous at |r| = delta
    e = 1e-9
    lo, hi = huber(torch.tensor([d - e], dtype=torch.float64), d), huber(torch.tensor([d + e], dtype=torch.float64), d)
    assert abs(float(hi - lo)) < 3 * d * e
    np.testing.assert_allclose(huber_grad(np.array([0.3 * d, -0.3 * d, 5 * d, -5 * d]), d),
                               [0.3 * d, -0.3 * d, d, -d])


def _batch():
    return [(s.pos, s.Z, s.cell) for s in (sio2_box(4, seed=3), sio2_box(6, seed=4))]


def _labels(model, batch, residuals):
    # reference energies placing each structure's per-atom residual at a chosen value
    E = energy_loss(model, batch, [0.0] * len(batch), grads=False)["energies"]
    return [E[b] - residuals[b] * len(batch[b][1]) for b in range(len(batch))]


@pytest.mark.parametrize("which", ["small", "real"])
def test_weight_gradients_match_finite_differences(which):
    spec = model_spec_small() if which == "small" else model_spec_real()
    m = OracleModel(spec.config(), make_weights(spec, 11))
    batch = _batch()
    labels = _labels(m, batch, [0.004, -0.2])  # one quadratic, one linear Huber regime
    ref = energy_loss(m, batch, labels)
    rng = np.random.Generator(np.random.PCG64(5))
    worst = 0.0
    for name, g in ref["grads"].items():
        W = m.W[name]
        for _ in range(2):
            idx = tuple(int(rng.integers(0, s)) for s in W.shape)
            h = 1e-5 * max(1.0, abs(float(W[idx])))
            vals = []
            for sgn in (1.0, -1.0):
                W2 = W.clone()
                W2[idx] += sgn * h
                m.W[name] = W2
                vals.append(energy_loss(m, batch, labels, grads=False)["loss"])
            m.W[name] = W
            fd = (vals[0] - vals[1]) / (2 * h)
            # relative to the tensor's largest gradient, plus the difference quotient's own
            # rounding floor (float64 rounding of the energy sums, ~1e-16 in the loss, over 2h)
            worst = max(worst, abs(fd - g[idx]) / (np.abs(g).max() + 1e-5))
    assert worst < 1e-6, worst


def test_loss_derivative_per_structure():
    spec = model_spec_small()
    m = OracleModel(spec.config(), make_weights(spec, 12))
    batch = _batch()
    labels = _labels(m, batch, [-0.003, 0.05])
    out = energy_loss(m, batch, labels, grads=False)
    N = np.array([len(z) for _, z, _ in batch])
    # dGamma/dE_b = huber'(r_b) / (M N_b): r = (-0.003, 0.05), delta 0.01
    np.testing.assert_allclose(out["dloss_dE"], np.array([-0.003, 0.01]) / (2 * N), rtol=1e-9)
    # and the loss itself from the same residuals
    want = (0.5 * 0.003 ** 2 + 0.01 * (0.05 - 0.005)) / 2
    assert abs(out["loss"] - want) < 1e-12


def _full_labels(m, batch, seed=7):
    """Labels near the model's own predictions so every term has residuals on both sides of
    delta: energies shifted per atom, forces and stresses perturbed by seeded noise."""
    ref = full_loss(m, batch, [0.0] * len(batch), [np.zeros((len(z), 3)) for _, z, _ in batch],
                    np.zeros((len(batch), 6)), grads=False)
    rng = np.random.Generator(np.random.PCG64(seed))
    lE = [ref["energies"][b] - [0.004, -0.2][b % 2] * len(batch[b][1]) for b in range(len(batch))]
    lF = [f + rng.normal(0.0, 0.02, f.shape) for f in ref["forces"]]
    lS = ref["stress"] + rng.normal(0.0, 0.05, ref["stress"].shape)
    return lE, lF, lS


def test_full_loss_gradients_match_finite_differences():
    """Second derivatives (forces and stresses inside the loss) against central differences of
    the loss itself, whose forces and stresses are first derivatives only."""
    spec = model_spec_small()
    m = OracleModel(spec.config(), make_weights(spec, 13))
    batch = _batch()
    lE, lF, lS = _full_labels(m, batch)
    ref = full_loss(m, batch, lE, lF, lS)
    rng = np.random.Generator(np.random.PCG64(6))
    worst = 0.0
    for name, g in ref["grads"].items():
        W = m.W[name]
        for _ in range(2):
            idx = tuple(int(rng.integers(0, s)) for s in W.shape)
            h = 1e-5 * max(1.0, abs(float(W[idx])))
            vals = []
            for sgn in (1.0, -1.0):
                W2 = W.clone()
                W2[idx] += sgn * h
                m.W[name] = W2
                vals.append(full_loss(m, batch, lE, lF, lS, grads=False)["loss"])
            m.W[name] = W
            fd = (vals[0] - vals[1]) / (2 * h)
            worst = max(worst, abs(fd - g[idx]) / (np.abs(g).max() + 1e-5))
    assert worst < 1e-6, worst


def test_full_loss_reduces_to_energy_term():
    spec = model_spec_small()
    m = OracleModel(spec.config(), make_weights(spec, 14))
    batch = _batch()
    lE, lF, lS = _full_labels(m, batch)
    a = full_loss(m, batch, lE, lF, lS, mu_f=0.0, mu_s=0.0)
    b = energy_loss(m, batch, lE)
    assert abs(a["loss"] - b["loss"]) < 1e-15
    for k in a["grads"]:
        np.testing.assert_allclose(a["grads"][k], b["grads"][k], rtol=1e-12, atol=1e-18)


def test_stress_is_minus_virial_over_volume_in_gpa():
    """S = -W/V (GPa) with W from the strain derivative of the energy: W_ab = -dE/de_ab,
    positions and cell deformed by (I + e) (checked by central differences of E)."""
    spec = model_spec_small()
    m = OracleModel(spec.config(), make_weights(spec, 15))
    pos, Z, cell = _batch()[0]
    out = full_loss(m, [(pos, Z, cell)], [0.0], [np.zeros((len(Z), 3))], np.zeros((1, 6)), grads=False)
    V = abs(np.linalg.det(cell))
    h = 1e-5
    for (a, b), l in (((0, 0), 0), ((1, 2), 3), ((0, 1), 5)):
        Es = []
        for sgn in (1.0, -1.0):
            e = np.zeros((3, 3))
            e[a, b] += 0.5 * sgn * h
            e[b, a] += 0.5 * sgn * h
            D = np.eye(3) + e
            Es.append(energy_loss(m, [(pos @ D.T, Z, cell @ D.T)], [0.0], grads=False)["energies"][0])
        W_ab = -(Es[0] - Es[1]) / (2 * h)
        assert abs(out["stress"][0][l] - (-W_ab / V * 160.21766208)) < 1e-6 * max(1.0, abs(out["stress"][0][l]))
