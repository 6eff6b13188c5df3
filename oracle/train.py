"""Energy term of the training loss (paper section 5.1, eq 9) and its gradient with respect
to every weight tensor of the model.

TEST INFRASTRUCTURE (see oracle/__init__.py).

For a batch of M structures with N_b atoms each, predicted energies E_b (eq 1) and labels
R_b, the energy term of eq 9 is the mean over the batch of a Huber loss of the per-atom
energies:
    Gamma_E = (1/M) sum_b huber(E_b / N_b - R_b / N_b; delta),
    huber(r; delta) = r^2 / 2 for |r| < delta, delta (|r| - delta / 2) otherwise,
the form that moves from a squared to an absolute error at delta (the paper uses
delta = 0.01).  Its derivative with respect to a structure's energy is
    dGamma_E / dE_b = huber'(r_b) / (M N_b),  huber'(r) = r for |r| < delta, delta sign(r) else.
The weight gradients come from torch.autograd through the same model evaluation as
oracle.model.evaluate.
"""
from __future__ import annotations

import numpy as np
import torch

from .model import OracleModel, atom_energies

DT = torch.float64


def huber(r: torch.Tensor, delta: float) -> torch.Tensor:
    a = r.abs()
    return torch.where(a < delta, 0.5 * r * r, delta * (a - 0.5 * delta))


def huber_grad(r: np.ndarray, delta: float) -> np.ndarray:
    return np.where(np.abs(r) < delta, r, delta * np.sign(r))


def energy_loss(model: OracleModel, structures, labels, delta: float = 0.01, grads: bool = True):
    """Gamma_E of a batch of (pos, Z, cell) structures with reference energies `labels` (eV).
    Returns dict(loss, energies [M], dloss_dE [M], grads {tensor name: dGamma_E/dW} or None)."""
    names = list(model.W.keys())
    saved = dict(model.W)
    if grads:
        for k in names:
            model.W[k] = saved[k].detach().clone().requires_grad_(True)
    try:
        E, N = [], []
        for pos, Z, cell in structures:
            E_i, _, _, _ = atom_energies(model, pos, Z, cell)
            E.append(E_i.sum())
            N.append(len(Z))
        E = torch.stack(E)
        Nt = torch.tensor(N, dtype=DT)
        R = torch.as_tensor(np.asarray(labels, dtype=np.float64))
        r = E / Nt - R / Nt
        loss = huber(r, delta).mean()
        out = dict(loss=float(loss), energies=E.detach().numpy(),
                   dloss_dE=huber_grad(r.detach().numpy(), delta) / (len(N) * np.asarray(N)))
        out["grads"] = None
        if grads:
            g = torch.autograd.grad(loss, [model.W[k] for k in names])
            out["grads"] = {k: gi.detach().numpy() for k, gi in zip(names, g)}
        return out
    finally:
        model.W.update(saved)
