"""Pins of the oracle's MD integrators (NVE velocity Verlet and Nose-Hoover NVT, the
thermostat of the paper's MD benchmarks, section 4) against closed forms and the
invariants of the equations of motion."""
import math

import numpy as np

from oracle import md


def _springs(k):
    """Independent isotropic springs about the origin: U = sum k_i |x_i|^2 / 2."""
    def force(pos):
        return 0.5 * float((k[:, None] * pos * pos).sum()), -k[:, None] * pos
    return force


def test_verlet_matches_closed_form_harmonic():
    # The kick-drift-kick map for x'' = -w^2 x gives x_{n+1} - 2 x_n + x_{n-1} = -(w dt)^2 x_n,
    # solved by x_n = x_0 cos(n th) + dt v_0 sin(n th) / sin(th), cos(th) = 1 - (w dt)^2 / 2.
    k = np.array([0.7, 2.0, 5.0])
    inv_m = np.array([0.5, 0.25, 0.1])
    dt = 0.1
    x0 = np.array([[0.3, -0.2, 0.1], [0.05, 0.4, -0.3], [-0.2, 0.1, 0.25]])
    v0 = np.array([[0.1, 0.0, -0.2], [0.0, 0.3, 0.1], [0.2, -0.1, 0.0]])
    force = _springs(k)
    pos, vel = x0.copy(), v0.copy()
    _, F = force(pos)
    w2 = k * inv_m
    th = np.arccos(1.0 - 0.5 * w2 * dt * dt)
    for n in range(1, 501):
        pos, vel, F, _, _ = md.step(pos, vel, F, inv_m, dt, force)
        want = x0 * np.cos(n * th)[:, None] + dt * v0 * (np.sin(n * th) / np.sin(th))[:, None]
        np.testing.assert_allclose(pos, want, atol=1e-11)


def _nh_system(seed, n=40):
    rng = np.random.default_rng(seed)
    k = rng.uniform(0.5, 4.0, n)
    inv_m = rng.uniform(0.05, 0.5, n)
    pos = rng.normal(0.0, 0.3, (n, 3))
    vel = rng.normal(0.0, 0.2, (n, 3))
    kT, dof = 0.05, 3.0 * n
    Q = dof * kT * 2.0 ** 2  # tau = 2 time units
    return _springs(k), inv_m, pos, vel, (kT, dof, Q)


def test_nose_hoover_is_time_reversible():
    force, inv_m, pos0, vel0, th = _nh_system(1)
    dt = 0.02
    pos, vel = pos0.copy(), vel0.copy()
    _, F = force(pos)
    state = (0.0, 0.0)
    for _ in range(300):
        pos, vel, F, _, state = md.step(pos, vel, F, inv_m, dt, force, th, state)
    assert abs(state[0]) > 1e-3  # the thermostat did act
    vel, state = -vel, (-state[0], state[1])
    for _ in range(300):
        pos, vel, F, _, state = md.step(pos, vel, F, inv_m, dt, force, th, state)
    np.testing.assert_allclose(pos, pos0, atol=1e-9)
    np.testing.assert_allclose(-vel, vel0, atol=1e-9)
    assert abs(state[0]) < 1e-9


def test_nose_hoover_conserves_extended_energy():
    force, inv_m, pos, vel, th = _nh_system(2)
    dt = 0.01
    U, F = force(pos)
    state = (0.0, 0.0)
    h0 = md.conserved(U, vel, inv_m, th, state)
    hs = []
    for _ in range(2000):
        pos, vel, F, U, state = md.step(pos, vel, F, inv_m, dt, force, th, state)
        hs.append(md.conserved(U, vel, inv_m, th, state))
    hs = np.array(hs)
    scale = md.kinetic(vel, inv_m) + U
    assert np.abs(hs - h0).max() / scale < 2e-4
    # and the plain kinetic + potential energy is not conserved (heat flows to the bath)
    assert abs(md.kinetic(vel, inv_m) + U - h0) / scale > 1e-2


def test_nose_hoover_drives_the_temperature():
    # Oscillators of many distinct frequencies started hot: the time-averaged kinetic
    # temperature 2K / dof settles at the bath's kT.
    rng = np.random.default_rng(3)
    n = 200
    k = rng.uniform(0.5, 8.0, n)
    inv_m = rng.uniform(0.05, 0.5, n)
    force = _springs(k)
    kT, dof = 0.05, 3.0 * n
    th = (kT, dof, dof * kT * 0.5 ** 2)
    pos = np.zeros((n, 3))
    vel = rng.normal(0.0, 1.0, (n, 3)) * np.sqrt(4.0 * kT * inv_m)[:, None]  # four times hotter
    _, F = force(pos)
    state = (0.0, 0.0)
    temps = []
    for s in range(4000):
        pos, vel, F, _, state = md.step(pos, vel, F, inv_m, 0.02, force, th, state)
        if s >= 2000:
            temps.append(2.0 * md.kinetic(vel, inv_m) / dof)
    assert abs(np.mean(temps) / kT - 1.0) < 0.05


def test_max_displacement_brute_force():
    rng = np.random.default_rng(4)
    a, b = rng.normal(size=(50, 3)), rng.normal(size=(50, 3))
    want = max(math.dist(a[i], b[i]) for i in range(50))
    assert abs(md.max_displacement(a, b) - want) < 1e-15
