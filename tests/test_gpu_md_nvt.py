"""NVT molecular dynamics (the Nose-Hoover setting of the paper's MD benchmarks, section 4)
and the skin-triggered neighbour-list rebuild, through the library's MD entry points."""
import numpy as np
import pytest

from gpu_common import log, write_model

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2402_03789_amd as sn  # noqa: E402
from paper_2402_03789_amd.md import NoseHoover, VelocityVerlet  # noqa: E402
from oracle import md as omd  # noqa: E402
from oracle.model import OracleModel, evaluate  # noqa: E402
from synth import make_weights, model_spec_small, sio2_box  # noqa: E402

KB = 8.617333262e-5            # eV / K
AMU_A2_FS2 = 103.642697        # 1 amu A^2 / fs^2 in eV


def _velocities(masses, temperature, seed):
    """Seeded Gaussian velocities (A/fs) with zero total momentum (an input, not method)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((len(masses), 3)) * np.sqrt(KB * temperature / (AMU_A2_FS2 * masses))[:, None]
    return v - (masses[:, None] * v).sum(0) / masses.sum()


@pytest.fixture(scope="module")
def small(tmp_path_factory):
    spec = model_spec_small()
    path, w = write_model(tmp_path_factory.mktemp("m"), spec, 101)
    return spec, path, w


def test_nvt_trajectory_matches_oracle(small):
    spec, path, w = small
    s = sio2_box(16, seed=11)
    m = s.masses()
    v0 = _velocities(m, 900.0, 21)
    dt, steps, T0, tau = 0.5, 10, 300.0, 10.0
    log(f"nvt parity: n={s.n} steps={steps}")
    ctx = sn.Context(sn.Model(path), precision="fp64", skin=0.5)
    run = VelocityVerlet(ctx, s.pos, s.Z, s.cell, m, dt=dt, rebuild_every=None, velocities=v0,
                         thermostat=NoseHoover(T0, tau))
    run.run(steps)
    ctx.synchronize()
    gpu_pos, gpu_vel = run.pos.cpu().numpy(), run.vel.cpu().numpy()
    xi, eta = run.thermostat_state()

    om = OracleModel(spec.config(), w)

    def force(p):
        r = evaluate(om, p, s.Z, s.cell)
        return r["energy"], r["forces"]

    inv_m = 1.0 / (AMU_A2_FS2 * m)
    dof = 3.0 * s.n - 3.0
    kT = KB * T0
    th = (kT, dof, dof * kT * tau * tau)
    pos, vel = s.pos.copy(), v0.copy()
    _, F = force(pos)
    state = (0.0, 0.0)
    for _ in range(steps):
        pos, vel, F, _, state = omd.step(pos, vel, F, inv_m, dt, force, th, state)
    log(f"|dx|={np.abs(gpu_pos - pos).max():.2e} |dv|={np.abs(gpu_vel - vel).max():.2e} "
        f"xi {xi:.6e} vs {state[0]:.6e}, eta {eta:.6e} vs {state[1]:.6e}, rebuilds {run.rebuilds}")
    assert abs(state[0]) > 1e-4  # the thermostat acted
    np.testing.assert_allclose(gpu_pos, pos, atol=1e-9)
    np.testing.assert_allclose(gpu_vel, vel, atol=1e-11)
    assert abs(xi - state[0]) <= 1e-9 * abs(state[0])
    assert abs(eta - state[1]) <= 1e-9 * max(abs(state[1]), 1e-12)


def test_displacement_trigger_equals_fresh_lists(small):
    _, path, _ = small
    s = sio2_box(24, seed=12)
    m = s.masses()
    v0 = _velocities(m, 3000.0, 22)
    log("skin-triggered rebuild vs a fresh list every step")
    runs = []
    for every in (None, 1):
        ctx = sn.Context(sn.Model(path), precision="fp64", skin=0.3)
        r = VelocityVerlet(ctx, s.pos, s.Z, s.cell, m, dt=1.0, rebuild_every=every, velocities=v0,
                           thermostat=NoseHoover(1500.0, 20.0))
        r.run(30)
        ctx.synchronize()
        runs.append(r)
    trig, fresh = runs
    log(f"rebuilds: triggered {trig.rebuilds}, fresh {fresh.rebuilds}; "
        f"|dx|={np.abs(trig.pos.cpu().numpy() - fresh.pos.cpu().numpy()).max():.2e}")
    assert 1 < trig.rebuilds < fresh.rebuilds
    np.testing.assert_allclose(trig.pos.cpu().numpy(), fresh.pos.cpu().numpy(), atol=1e-8)
    np.testing.assert_allclose(trig.vel.cpu().numpy(), fresh.vel.cpu().numpy(), atol=1e-9)


def test_nvt_conserved_quantity(small):
    _, path, _ = small
    s = sio2_box(24, seed=13)
    m = s.masses()
    log("nvt conserved energy")
    ctx = sn.Context(sn.Model(path), precision="fp64", skin=1.0)
    r = VelocityVerlet(ctx, s.pos, s.Z, s.cell, m, dt=0.25, rebuild_every=None,
                       velocities=_velocities(m, 1200.0, 23), thermostat=NoseHoover(300.0, 10.0))
    h0 = r.conserved_energy()
    e0 = r.kinetic_energy() + r.potential_energy()
    r.run(200)
    h1 = r.conserved_energy()
    e1 = r.kinetic_energy() + r.potential_energy()
    log(f"H' {h0:.6f} -> {h1:.6f}; K+U {e0:.6f} -> {e1:.6f}; T {r.temperature():.1f} K")
    assert abs(h1 - h0) / s.n < 2e-4
    assert abs(e1 - e0) / s.n > 2e-3  # energy left through the thermostat


def test_md_entry_points_reject_bad_arguments(small):
    _, path, _ = small
    ctx = sn.Context(sn.Model(path), precision="fp64")
    dev = torch.device("cuda:0")
    v = torch.zeros((4, 3), dtype=torch.float64, device=dev)
    im = torch.ones(4, dtype=torch.float64, device=dev)
    st = torch.zeros(4, dtype=torch.float64, device=dev)
    with pytest.raises(sn.SNError):
        ctx.nh_half(v, im, 0.5, 0.0, 9.0, 1.0, st)  # kT must be positive
    with pytest.raises(sn.SNError):
        ctx.nh_half(v, im, 0.5, 0.025, 9.0, -1.0, st)  # Q must be positive
    with pytest.raises(ValueError):
        ctx.nh_half(v.float(), im, 0.5, 0.025, 9.0, 1.0, st)  # float32 velocities
    with pytest.raises(ValueError):
        ctx.max_displacement(v, torch.zeros((3, 3), dtype=torch.float64, device=dev))
    assert ctx.max_displacement(v, v) == 0.0
