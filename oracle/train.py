"""The training loss of paper section 5.1 (eq 9) and its gradient with respect to every
weight tensor of the model: the energy term alone (energy_loss) and all three terms,
energies, forces and stresses (full_loss).

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


EV_A3_GPA = 160.21766208  # GPa per eV / A^3


def full_loss(model: OracleModel, structures, labels_E, labels_F, labels_S, delta: float = 0.01,
              mu_f: float = 0.1, mu_s: float = 0.01, grads: bool = True):
    """All three terms of eq 9 for a batch:
      Gamma = (1/M) sum_b huber(E_b/N_b - R_b/N_b)
            + mu_f / (3 M sum_b N_b) sum_b sum_j sum_k huber(F_bjk - R^F_bjk)
            + mu_s / (6 M) sum_b sum_l huber(S_bl - R^S_bl)
    with the force-term normalisation as printed (3 M times the total atom count), the stress
    S = -W / V in GPa from the symmetric virial W = -sum_e d_e (x) dE/dd_e, and its six
    components in the order xx, yy, zz, yz, xz, xy.  Forces and virial are first derivatives
    taken with create_graph, so the weight gradients are the second derivatives the force
    and stress terms need.  labels_F: one [N_b, 3] array per structure; labels_S: [M, 6]."""
    names = list(model.W.keys())
    saved = dict(model.W)
    if grads:
        for k in names:
            model.W[k] = saved[k].detach().clone().requires_grad_(True)
    try:
        M = len(structures)
        Ntot = sum(len(z) for _, z, _ in structures)
        le = lf = ls = 0.0
        E_out, F_out, S_out = [], [], []
        for b, (pos, Z, cell) in enumerate(structures):
            E_i, d, pos_t, graph = atom_energies(model, pos, Z, cell)
            E = E_i.sum()
            gpos, gd = torch.autograd.grad(E, [pos_t, d], create_graph=grads)
            F = -gpos
            W = -(d.T @ gd)
            W = 0.5 * (W + W.T)
            V = abs(float(np.linalg.det(np.asarray(cell, dtype=np.float64))))
            Sm = -W / V * EV_A3_GPA
            S = torch.stack([Sm[0, 0], Sm[1, 1], Sm[2, 2], Sm[1, 2], Sm[0, 2], Sm[0, 1]])
            N = len(Z)
            le = le + huber(E / N - float(labels_E[b]) / N, delta)
            lf = lf + huber(F - torch.as_tensor(np.asarray(labels_F[b], np.float64)), delta).sum()
            ls = ls + huber(S - torch.as_tensor(np.asarray(labels_S[b], np.float64)), delta).sum()
            E_out.append(float(E))
            F_out.append(F.detach().numpy())
            S_out.append(S.detach().numpy())
        loss = le / M + mu_f / (3 * M * Ntot) * lf + mu_s / (6 * M) * ls
        out = dict(loss=float(loss), energies=np.array(E_out), forces=F_out, stress=np.array(S_out),
                   grads=None)
        if grads:
            g = torch.autograd.grad(loss, [model.W[k] for k in names])
            out["grads"] = {k: gi.detach().numpy() for k, gi in zip(names, g)}
        return out
    finally:
        model.W.update(saved)


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
