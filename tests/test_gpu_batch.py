"""Packed multi-structure evaluation: every structure's result is the same alone and in
the mix (same kernels, same per-structure summation order), and matches the oracle."""
import numpy as np
import pytest

from gpu_common import log, write_model, errors, TOL_E_REL_FP64, TOL_F_ABS_FP64

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2402_03789_amd as sn  # noqa: E402
from synth import model_spec_real, serving_stream, sio2_box, make_weights  # noqa: E402

ALL_Z = tuple(range(1, 90))


@pytest.fixture(scope="module")
def model_path(tmp_path_factory):
    path, _ = write_model(tmp_path_factory.mktemp("m"), model_spec_real(ALL_Z), 104)
    return path


def _mix():
    reqs = [s for _, s in serving_stream(count=7, seed=11, n_min=8, n_max=400)]
    reqs.append(sio2_box(60, seed=12))
    return [(s.pos, s.Z, s.cell) for s in reqs]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_alone_equals_mixed(model_path, precision):
    mix = _mix()
    log(f"batch alone-vs-mixed precision={precision} sizes={[len(z) for _, z, _ in mix]}")
    ctx = sn.Context(sn.Model(model_path), precision=precision)
    packed = ctx.compute_batch(mix)
    for b, (p, z, c) in enumerate(mix):
        alone = ctx.compute(p, z, c)
        got = packed[b]
        assert got["energy"] == alone["energy"], (b, got["energy"], alone["energy"])
        np.testing.assert_array_equal(got["atom_energy"], alone["atom_energy"])
        np.testing.assert_array_equal(got["forces"], alone["forces"])
        np.testing.assert_array_equal(got["virial"], alone["virial"])


def test_mixed_matches_oracle(model_path):
    from oracle.model import OracleModel, evaluate
    mix = _mix()[:4]
    log(f"batch vs oracle sizes={[len(z) for _, z, _ in mix]}")
    ctx = sn.Context(sn.Model(model_path), precision="fp64")
    packed = ctx.compute_batch(mix)
    spec = model_spec_real(ALL_Z)
    om = OracleModel(spec.config(), make_weights(spec, 104))
    for b, (p, z, c) in enumerate(mix):
        ref = evaluate(om, p, z, c)
        err = errors(packed[b], ref)
        log(f"  structure {b} n={len(z)} {err}")
        assert err["e_rel"] <= TOL_E_REL_FP64 and err["f_abs"] <= TOL_F_ABS_FP64
        assert err["w_rel"] <= 1e-9


def test_batch_rejects_empty_structure(model_path):
    ctx = sn.Context(sn.Model(model_path), precision="fp32")
    s = sio2_box(16, seed=1)
    with pytest.raises(sn.SNError):
        ctx.compute_batch([(s.pos, s.Z, s.cell), (np.zeros((0, 3)), np.zeros(0, np.int32), s.cell)])
    # the context stays usable after the rejected call
    r = ctx.compute_batch([(s.pos, s.Z, s.cell)])
    assert np.isfinite(r[0]["energy"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_device_batch_autograd_equals_host_batch(model_path, precision):
    """A packed batch resident in device memory through the autograd Function (forward:
    energies [B]; backward: per-structure upstream gradients on the device) gives the
    host-buffer batch entry point's results bit for bit, scaled by each structure's
    upstream gradient."""
    mix = _mix()[:3]
    log(f"device batch autograd precision={precision} sizes={[len(z) for _, z, _ in mix]}")
    model = sn.Model(model_path)
    ref = sn.Context(model, precision=precision, allocator=None).compute_batch(mix)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    ctx = sn.Context(model, precision=precision)  # workspace from torch's caching allocator
    dev = torch.device("cuda:0")
    offs = np.cumsum([0] + [len(z) for _, z, _ in mix])
    pos = torch.tensor(np.concatenate([p for p, _, _ in mix]), device=dev, requires_grad=True)
    Z = torch.tensor(np.concatenate([z for _, z, _ in mix]).astype(np.int32), device=dev)
    cells = np.stack([c for _, _, c in mix])
    E = sn.energies(pos, Z, cells, offs, ctx)
    assert E.shape == (3,)
    g = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device=dev)
    (E * g).sum().backward()
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - before
    log(f"  context memory {ctx.memory() / 2**20:.1f} MiB, torch allocator grew {held / 2**20:.1f} MiB")
    assert held >= ctx.memory() > 0  # weights and workspace came through torch
    grad = pos.grad.cpu().numpy()
    W = ctx.last_virial.cpu().numpy().reshape(3, 3, 3)
    for b in range(3):
        assert float(E[b]) == ref[b]["energy"]
        gb = float(g[b])
        np.testing.assert_array_equal(-grad[offs[b]:offs[b + 1]], gb * ref[b]["forces"])
        np.testing.assert_array_equal(W[b], gb * ref[b]["virial"])
    ctx.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - before < held  # released back to torch
