"""Molecular-dynamics integrators in float64 numpy: velocity Verlet, and velocity Verlet
with one Nose-Hoover thermostat (the NVT setting of the paper's MD benchmarks, section 4).

TEST INFRASTRUCTURE (see oracle/__init__.py).

Equations of motion (Nose-Hoover, one thermostat on all particles):
  dx/dt = v,  dv/dt = a(x) - xi v,  dxi/dt = (2K - g kT) / Q,  deta/dt = xi,
with a = F * inv_mass (inv_mass carries the unit conversion, so that 1 / inv_mass is the
mass in eV fs^2 / A^2 and K = sum v^2 / (2 inv_mass) is in eV), g the thermostatted degrees
of freedom and Q the thermostat mass.  One step of length dt is the symmetric Trotter
splitting
  NH(dt/2)  kick(dt/2)  drift(dt)  [new forces]  kick(dt/2)  NH(dt/2),
where NH(h) integrates the thermostat part for a time h by
  xi += h/2 G(K);  eta += h xi;  v *= exp(-xi h);  xi += h/2 G(K),   G(K) = (2K - g kT) / Q,
each K taken from the velocities at that point.  The conserved quantity is
  H' = K + U + Q xi^2 / 2 + g kT eta.
Without the thermostat the step is plain velocity Verlet.
"""
from __future__ import annotations

import math

import numpy as np


def kinetic(vel, inv_mass) -> float:
    """K = sum_i |v_i|^2 / (2 inv_mass_i), summed atom by atom."""
    k = 0.0
    for i in range(vel.shape[0]):
        k += 0.5 * float(vel[i] @ vel[i]) / float(inv_mass[i])
    return k


def nh_half(vel, inv_mass, h, kT, dof, Q, xi, eta):
    """Thermostat part over a time h: returns the scaled velocities, xi and eta."""
    xi = xi + 0.5 * h * (2.0 * kinetic(vel, inv_mass) - dof * kT) / Q
    eta = eta + h * xi
    vel = vel * math.exp(-xi * h)
    xi = xi + 0.5 * h * (2.0 * kinetic(vel, inv_mass) - dof * kT) / Q
    return vel, xi, eta


def step(pos, vel, forces, inv_mass, dt, force_fn, thermostat=None, state=(0.0, 0.0)):
    """One step.  force_fn(pos) -> (U, F).  thermostat: None or (kT, dof, Q); state: (xi, eta).
    Returns pos, vel, forces, U, (xi, eta)."""
    xi, eta = state
    a = inv_mass[:, None]
    if thermostat is not None:
        kT, dof, Q = thermostat
        vel, xi, eta = nh_half(vel, inv_mass, 0.5 * dt, kT, dof, Q, xi, eta)
    vel = vel + 0.5 * dt * forces * a
    pos = pos + dt * vel
    U, forces = force_fn(pos)
    vel = vel + 0.5 * dt * forces * a
    if thermostat is not None:
        vel, xi, eta = nh_half(vel, inv_mass, 0.5 * dt, kT, dof, Q, xi, eta)
    return pos, vel, forces, U, (xi, eta)


def conserved(U, vel, inv_mass, thermostat=None, state=(0.0, 0.0)) -> float:
    """H' = K + U (+ Q xi^2 / 2 + g kT eta with the thermostat)."""
    h = kinetic(vel, inv_mass) + U
    if thermostat is not None:
        kT, dof, Q = thermostat
        xi, eta = state
        h += 0.5 * Q * xi * xi + dof * kT * eta
    return h


def max_displacement(pos, ref) -> float:
    """max_i |pos_i - ref_i|."""
    return max(math.sqrt(float((pos[i] - ref[i]) @ (pos[i] - ref[i]))) for i in range(pos.shape[0]))
