"""Device entry points: torch.autograd.Function, neighbour-list reuse, Verlet harness."""
import numpy as np
import pytest

from gpu_common import log, write_model

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2402_03789_amd as sn  # noqa: E402
from paper_2402_03789_amd.md import VelocityVerlet  # noqa: E402
from synth import model_spec_real, sio2_box  # noqa: E402


@pytest.fixture(scope="module")
def model_path(tmp_path_factory):
    path, _ = write_model(tmp_path_factory.mktemp("m"), model_spec_real(), 102)
    return path


def test_autograd_function_matches_forces(model_path):
    s = sio2_box(24, seed=3)
    log("autograd")
    ctx = sn.Context(sn.Model(model_path), precision="fp64")
    ref = ctx.compute(s.pos, s.Z, s.cell)
    dev = torch.device("cuda:0")
    pos = torch.tensor(s.pos, dtype=torch.float64, device=dev, requires_grad=True)
    Z = torch.tensor(s.Z, dtype=torch.int32, device=dev)
    E = sn.energy(pos, Z, s.cell, ctx)
    assert abs(float(E) - ref["energy"]) < 1e-10
    (2.5 * E).backward()
    np.testing.assert_allclose(pos.grad.cpu().numpy(), -2.5 * ref["forces"], atol=1e-10)
    W = ctx.last_virial.cpu().numpy().reshape(3, 3)
    np.testing.assert_allclose(W, 2.5 * ref["virial"], atol=1e-9)


def test_graph_reuse_equals_fresh_build(model_path):
    s = sio2_box(40, seed=5)
    rng = np.random.default_rng(0)
    moved = s.pos + rng.uniform(-0.3, 0.3, size=s.pos.shape)  # < skin / 2
    log("graph reuse")
    dev = torch.device("cuda:0")
    ctx = sn.Context(sn.Model(model_path), precision="fp64", skin=1.0)
    Z = torch.tensor(s.Z, dtype=torch.int32, device=dev)
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    f = torch.zeros((s.n, 3), dtype=torch.float64, device=dev)
    ctx.forward_device(torch.tensor(s.pos, device=dev), Z, s.cell, e)
    ctx.backward_device(1.0, f, None)
    ctx.set_graph_reuse(True)
    ctx.forward_device(torch.tensor(moved, device=dev), Z, s.cell, e)
    ctx.backward_device(1.0, f, None)
    ctx.synchronize()
    fresh = sn.Context(sn.Model(model_path), precision="fp64", skin=1.0).compute(moved, s.Z, s.cell)
    assert abs(float(e.cpu()[0]) - fresh["energy"]) < 1e-9
    np.testing.assert_allclose(f.cpu().numpy(), fresh["forces"], atol=1e-10)


def test_verlet_energy_conservation(model_path):
    s = sio2_box(16, seed=9)
    log("verlet nve")
    ctx = sn.Context(sn.Model(model_path), precision="fp64", skin=1.0)
    md = VelocityVerlet(ctx, s.pos, s.Z, s.cell, s.masses(), dt=0.25, rebuild_every=10,
                        temperature=300.0, seed=5)
    e0 = md.kinetic_energy() + md.potential_energy()
    md.run(40)
    e1 = md.kinetic_energy() + md.potential_energy()
    log(f"E0={e0:.6f} E1={e1:.6f} drift per atom={(e1 - e0) / s.n:.2e}")
    assert abs(e1 - e0) / s.n < 2e-4
