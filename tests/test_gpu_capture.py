"""hipGraph replay of reused-neighbour-list evaluations: every replay equals the eager
launches bitwise, with eager work and synchronisations between replays, across pointer
changes and rebuilds; the MD driver gives the same trajectory with and without replay."""
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
def model(tmp_path_factory):
    path, _ = write_model(tmp_path_factory.mktemp("m"), model_spec_real(), 108)
    return sn.Model(path)


def _bufs(n, dev):
    return (torch.zeros(1, dtype=torch.float64, device=dev),
            torch.zeros(n, dtype=torch.float64, device=dev),
            torch.zeros((n, 3), dtype=torch.float64, device=dev),
            torch.zeros(9, dtype=torch.float64, device=dev))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_replays_equal_eager(model, precision):
    s = sio2_box(50, seed=21)
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(4)
    Z = torch.tensor(s.Z, dtype=torch.int32, device=dev)
    cap = sn.Context(model, precision=precision, skin=1.0)
    cap.set_graph_reuse(True)
    cap.set_capture(True)
    ref = sn.Context(model, precision=precision, skin=1.0)
    ref.set_edge_compaction(False)  # replay evaluates the whole list; so does the reference
    ref.set_graph_reuse(True)
    pos_c = torch.tensor(s.pos, device=dev)
    pos_r = torch.tensor(s.pos, device=dev)
    out_c = _bufs(s.n, dev)
    out_r = _bufs(s.n, dev)
    replayed = 0
    for step in range(8):
        if step == 5:  # other output pointers: a new recording
            out_c = _bufs(s.n, dev)
        moved = s.pos + rng.uniform(-0.2, 0.2, size=s.pos.shape)
        pos_c.copy_(torch.tensor(moved, device=dev))
        pos_r.copy_(torch.tensor(moved, device=dev))
        cap.forward_device(pos_c, Z, s.cell, out_c[0], out_c[1])
        cap.backward_device(1.0, out_c[2], out_c[3])
        cap.synchronize()
        replayed += len(cap.timings()) == 0
        ref.forward_device(pos_r, Z, s.cell, out_r[0], out_r[1])  # eager work between replays
        ref.backward_device(1.0, out_r[2], out_r[3])
        ref.synchronize()
        for a, b in zip(out_c, out_r):
            assert torch.equal(a, b), f"step {step}"
    log(f"  {precision}: {replayed} of 8 steps replayed from recorded graphs")
    assert replayed >= 5


def test_md_trajectory_same_with_replay(model):
    s = sio2_box(24, seed=22)
    runs = []
    for capture in (False, True):
        ctx = sn.Context(model, precision="fp64", skin=1.0)
        ctx.set_edge_compaction(False)  # replay evaluates the whole list; so does the eager run
        md = VelocityVerlet(ctx, s.pos, s.Z, s.cell, s.masses(), dt=0.5, rebuild_every=10,
                            temperature=600.0, seed=3, capture=capture)
        md.run(25)
        ctx.synchronize()
        runs.append((md.pos.cpu().numpy(), md.vel.cpu().numpy(), md.potential_energy()))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
    assert runs[0][2] == runs[1][2]
