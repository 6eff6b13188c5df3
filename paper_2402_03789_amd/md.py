"""Velocity-Verlet molecular dynamics driver on device-resident arrays.

The large-box workload of the paper (amorphous Si3N4 melt-quench, section 5.2)
advances positions with the forces of every evaluation, and the benchmark runs of
section 4 are NVT with a Nose-Hoover thermostat.  This driver keeps positions,
velocities, forces and the thermostat state in HBM and calls the library's
evaluation, its Verlet half-step kernel and its Nose-Hoover half-step operator
(NH(dt/2) kick drift [forces] kick NH(dt/2)).  The neighbour list (which carries a
skin, see Context(skin=...)) is rebuilt every `rebuild_every` steps, or, with
`rebuild_every=None`, as soon as an atom has moved more than half the skin since
the last build.

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


class NoseHoover:
    """One Nose-Hoover thermostat at `temperature` K with time constant `tau` fs (thermostat
    mass Q = dof kT tau^2)."""

    def __init__(self, temperature: float, tau: float = 100.0):
        if temperature <= 0 or tau <= 0:
            raise ValueError("temperature and tau must be positive")
        self.temperature = float(temperature)
        self.tau = float(tau)


class VelocityVerlet:
    def __init__(self, ctx: Context, pos, Z, cell, masses, dt: float = 1.0,
                 rebuild_every: int | None = 10, temperature: float = 1500.0, seed: int = 5,
                 device: str = "cuda:0", capture: bool = False,
                 thermostat: NoseHoover | None = None, velocities=None):
        dev = torch.device(device)
        if rebuild_every is None and ctx.skin <= 0:
            raise ValueError("a displacement-triggered rebuild needs a context with a skin")
        if rebuild_every is not None and rebuild_every > 1 and ctx.skin <= 0:
            # a kept list without a skin would silently drop pairs that move inside r_c
            raise ValueError("keeping a neighbour list between rebuilds needs a context with a skin")
        if rebuild_every is not None and rebuild_every < 1:
            raise ValueError("rebuild_every must be at least 1")
        self.ctx = ctx
        ctx.set_capture(capture)  # replay the steps between rebuilds from a HIP graph
        self.cell = np.ascontiguousarray(cell, dtype=np.float64)
        self.n = len(Z)
        self.masses = np.asarray(masses, dtype=np.float64)
        self.pos = torch.tensor(np.asarray(pos, dtype=np.float64), device=dev)
        self.Z = torch.tensor(np.asarray(Z, dtype=np.int32), device=dev)
        v0 = (maxwell_boltzmann(self.masses, temperature, seed) if velocities is None
              else np.asarray(velocities, dtype=np.float64).reshape(self.n, 3))
        self.vel = torch.tensor(v0, device=dev)
        self.inv_mass = torch.tensor(ACC_CONV / self.masses, device=dev)
        self.forces = torch.zeros((self.n, 3), dtype=torch.float64, device=dev)
        self.energy = torch.zeros(1, dtype=torch.float64, device=dev)
        self.dt = float(dt)
        self.rebuild_every = None if rebuild_every is None else int(rebuild_every)
        self.steps_done = 0
        self.rebuilds = 0
        self.thermostat = thermostat
        self.dof = 3.0 * self.n - 3.0  # the centre-of-mass momentum stays zero
        if thermostat is not None:
            self.kT = KB_EV * thermostat.temperature
            self.Q = self.dof * self.kT * thermostat.tau ** 2
        self.nh_state = torch.zeros(4, dtype=torch.float64, device=dev)  # xi, eta, scale, K
        self.pos_ref = self.pos.clone()  # positions at the last neighbour-list build
        self._evaluate(rebuild=True)

    def _evaluate(self, rebuild: bool):
        if rebuild:
            self.pos_ref.copy_(self.pos)
            self.rebuilds += 1
        self.ctx.set_graph_reuse(not rebuild)
        self.ctx.forward_device(self.pos, self.Z, self.cell, self.energy)
        self.ctx.backward_device(1.0, self.forces, None)

    def _rebuild_due(self) -> bool:
        if self.rebuild_every is not None:
            return self.steps_done % self.rebuild_every == 0
        return self.ctx.max_displacement(self.pos, self.pos_ref) > 0.5 * self.ctx.skin

    def _thermostat(self):
        if self.thermostat is not None:
            # the thermostat half of a step of length dt (the library applies NH(dt/2))
            self.ctx.nh_half(self.vel, self.inv_mass, self.dt, self.kT, self.dof, self.Q,
                             self.nh_state)

    def step(self):
        self._thermostat()
        self.ctx.verlet(self.pos, self.vel, self.forces, self.inv_mass, self.dt, 0)
        self.steps_done += 1
        self._evaluate(rebuild=self._rebuild_due())
        self.ctx.verlet(self.pos, self.vel, self.forces, self.inv_mass, self.dt, 1)
        self._thermostat()

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

    def temperature(self) -> float:
        return 2.0 * self.kinetic_energy() / (self.dof * KB_EV)

    def thermostat_state(self) -> tuple[float, float]:
        """(xi in 1/fs, eta)."""
        self.ctx.synchronize()
        st = self.nh_state.cpu().numpy()
        return float(st[0]), float(st[1])

    def conserved_energy(self) -> float:
        """K + U, plus Q xi^2 / 2 + dof kT eta with the thermostat (eV)."""
        h = self.kinetic_energy() + self.potential_energy()
        if self.thermostat is not None:
            xi, eta = self.thermostat_state()
            h += 0.5 * self.Q * xi * xi + self.dof * self.kT * eta
        return h
