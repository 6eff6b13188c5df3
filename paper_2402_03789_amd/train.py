"""Training step quantities for the energy term of the loss (paper section 5.1, eq 9).

`energy_loss_and_grads` evaluates a batch of structures packed in device memory in
training mode, takes the Huber loss of the per-atom energies against the labels and its
derivatives with the library's host helper, and runs the library's weight-gradient
adjoint.  Everything numeric runs in libsn (kernels, and the B-value loss on the host);
this module only moves arrays.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from ._lib import lib, check, ptr


def huber_energy_loss(energies, labels, natoms, delta: float = 0.01):
    """(loss, dloss/dE_b) of the energy term of eq 9 (sn_huber_energy_loss)."""
    e = np.ascontiguousarray(energies, dtype=np.float64)
    r = np.ascontiguousarray(labels, dtype=np.float64)
    n = np.ascontiguousarray(natoms, dtype=np.int64)
    g = np.zeros_like(e)
    loss = C.c_double()
    check(lib().sn_huber_energy_loss(len(e), ptr(e), ptr(r), ptr(n), float(delta), C.byref(loss),
                                     ptr(g)))
    return loss.value, g


def _pack(structures, dev):
    offs = np.cumsum([0] + [len(z) for _, z, _ in structures]).astype(np.int64)
    pos = torch.tensor(np.concatenate([np.asarray(p, np.float64) for p, _, _ in structures]),
                       device=dev)
    Z = torch.tensor(np.concatenate([np.asarray(z, np.int32) for _, z, _ in structures]), device=dev)
    cells = np.stack([np.asarray(c, np.float64) for _, _, c in structures])
    return offs, pos, Z, cells


def weight_gradients(ctx, structures, grad_energy, device: int = 0) -> dict:
    """Energies [B] and sum_b g_b dE_b/dW per weight tensor for given upstream gradients
    g = grad_energy [B] (the adjoint alone, without the loss)."""
    dev = torch.device(f"cuda:{device}")
    offs, pos, Z, cells = _pack(structures, dev)
    energy = torch.zeros(len(structures), dtype=torch.float64, device=dev)
    ctx.set_training(True)
    try:
        ctx.forward_device(pos, Z, cells, energy, offsets=offs)
        gdev = torch.tensor(np.asarray(grad_energy, np.float64), device=dev)
        wg = torch.zeros(ctx.model.info()["n_params"], dtype=torch.float64, device=dev)
        ctx.backward_train_device(gdev, wg)
        ctx.synchronize()
    finally:
        ctx.set_training(False)
    flat = wg.cpu().numpy()
    return dict(energies=energy.cpu().numpy(),
                grads={name: flat[off:off + cnt] for name, off, cnt in ctx.model.tensors()})


def energy_loss_and_grads(ctx, structures, labels, delta: float = 0.01, device: int = 0) -> dict:
    """Loss, energies [B], dloss/dE [B] and dloss/dW per weight tensor (float64 numpy) for a
    batch of (pos, Z, cell) structures evaluated as one packed graph."""
    dev = torch.device(f"cuda:{device}")
    offs, pos, Z, cells = _pack(structures, dev)
    B = len(structures)
    energy = torch.zeros(B, dtype=torch.float64, device=dev)
    ctx.set_training(True)
    try:
        ctx.forward_device(pos, Z, cells, energy, offsets=offs)
        e = energy.cpu().numpy()
        loss, g = huber_energy_loss(e, labels, np.diff(offs), delta)
        gdev = torch.tensor(g, dtype=torch.float64, device=dev)
        n_params = ctx.model.info()["n_params"]
        wg = torch.zeros(n_params, dtype=torch.float64, device=dev)
        ctx.backward_train_device(gdev, wg)
        ctx.synchronize()
    finally:
        ctx.set_training(False)
    flat = wg.cpu().numpy()
    grads = {name: flat[off:off + cnt] for name, off, cnt in ctx.model.tensors()}
    return dict(loss=loss, energies=e, dloss_dE=g, grads=grads)


def full_loss_and_grads(ctx, structures, labels_E, labels_F, labels_S, delta: float = 0.01,
                        mu_f: float = 0.1, mu_s: float = 0.01, fd_step: float = 0.0,
                        device: int = 0) -> dict:
    """All three terms of eq 9 and dloss/dW per weight tensor (sn_train_loss_grad) for a batch
    of (pos, Z, cell) structures; labels_F: one [N_b, 3] array per structure, labels_S [M, 6]
    (GPa)."""
    from ._lib import Batch
    dev = torch.device(f"cuda:{device}")
    offs, pos, Z, cells = _pack(structures, dev)
    cells = np.ascontiguousarray(cells)
    rE = np.ascontiguousarray(labels_E, dtype=np.float64)
    rF = np.ascontiguousarray(np.concatenate([np.asarray(f, np.float64).reshape(-1, 3) for f in labels_F]))
    rS = np.ascontiguousarray(labels_S, dtype=np.float64).reshape(-1, 6)
    wg = torch.zeros(ctx.model.info()["n_params"], dtype=torch.float64, device=dev)
    b = Batch(len(structures), offs.ctypes.data, cells.ctypes.data, pos.data_ptr(), Z.data_ptr())
    loss = C.c_double()
    check(lib().sn_train_loss_grad(ctx.handle, C.byref(b), ptr(rE), ptr(rF), ptr(rS), float(delta),
                                   float(mu_f), float(mu_s), float(fd_step), C.byref(loss),
                                   ptr(wg)), ctx.handle)
    flat = wg.cpu().numpy()
    return dict(loss=loss.value,
                grads={name: flat[off:off + cnt] for name, off, cnt in ctx.model.tensors()})
