"""Velocity-Verlet molecular dynamics driver on device-resident arrays.

The large-box workload of the paper (amorphous Si3N4 melt-quench, section 5.2)
advances positions with the forces of every evaluation.  This driver keeps
positions, velocities and forces in HBM, calls the library's evaluation and
its Verlet half-step kernel, and rebuilds the neighbour list every
`rebuild_every` steps (the list carries a skin, see Context(skin=...)).

Units: angstrom, fs, eV, amu.  a [A/fs^2] = 0.0096485 F [eV/A] / m [amu].
"""
from __future__ import annotations

import numpy as np
import torch

from . import Context

EV_PER_AMU_A2_FS2 = 103.642697  # 1 amu A^2 / fs^2 in eV
ACC_CONV = 1.0 / EV_PER_AMU_A2_FS2  # 0.0096485: eV/A/amu -> A/fs^2
KB_EV = 8.617333262e-5


def maxwell_boltzmann(masses: np.ndarray, temperature: float, seed: int) -> np.ndarray:
    """Velocities (A/fs) at `temperature` K with zero centre-of-mass momentum."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sigma = np.sqrt(KB_EV * temperature * ACC_CONV / masses)
    v = rng.standard_normal((masses.shape[0], 3)) * sigma[:, None]
    v -= (masses[:, None] * v).sum(0) / masses.sum()
    return v


class VelocityVerlet:
    def __init__(self, ctx: Context, pos, Z, cell, masses, dt: float = 1.0,
                 rebuild_every: int = 10, temperature: float = 1500.0, seed: int = 5,
                 device: str = "cuda:0", capture: bool = False):
        dev = torch.device(device)
        self.ctx = ctx
        ctx.set_capture(capture)  # replay the steps between rebuilds from a HIP graph
        self.cell = np.ascontiguousarray(cell, dtype=np.float64)
        self.n = len(Z)
        self.masses = np.asarray(masses, dtype=np.float64)
        self.pos = torch.tensor(np.asarray(pos, dtype=np.float64), device=dev)
        self.Z = torch.tensor(np.asarray(Z, dtype=np.int32), device=dev)
        self.vel = torch.tensor(maxwell_boltzmann(self.masses, temperature, seed), device=dev)
        self.inv_mass = torch.tensor(ACC_CONV / self.masses, device=dev)
        self.forces = torch.zeros((self.n, 3), dtype=torch.float64, device=dev)
        self.energy = torch.zeros(1, dtype=torch.float64, device=dev)
        self.dt = float(dt)
        self.rebuild_every = int(rebuild_every)
        self.steps_done = 0
        self._evaluate(rebuild=True)

    def _evaluate(self, rebuild: bool):
        self.ctx.set_graph_reuse(not rebuild)
        self.ctx.forward_device(self.pos, self.Z, self.cell, self.energy)
        self.ctx.backward_device(1.0, self.forces, None)

    def step(self):
        self.ctx.verlet(self.pos, self.vel, self.forces, self.inv_mass, self.dt, 0)
        self.steps_done += 1
        self._evaluate(rebuild=(self.steps_done % self.rebuild_every == 0))
        self.ctx.verlet(self.pos, self.vel, self.forces, self.inv_mass, self.dt, 1)

    def run(self, steps: int):
        for _ in range(steps):
            self.step()

    def kinetic_energy(self) -> float:
        self.ctx.synchronize()
        v = self.vel.cpu().numpy()
        return 0.5 * float((self.masses[:, None] * v * v).sum()) * EV_PER_AMU_A2_FS2

    def potential_energy(self) -> float:
        self.ctx.synchronize()
        return float(self.energy.cpu()[0])
