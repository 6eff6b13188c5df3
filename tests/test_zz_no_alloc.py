"""sn_compute_noalloc: the host-buffer evaluation with every device buffer taken from the
library's static per-device scratch.  Its results equal sn_compute's on the same context
(same kernels, same order), over two calls in a row with the second smaller, it leaves the
context's own memory and torch's allocator untouched, and a structure too large for the
scratch is refused with SN_ENOMEM while the context stays usable."""
import numpy as np
import pytest

from gpu_common import log, write_model

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2402_03789_amd as sn  # noqa: E402
from synth import model_spec_small, model_spec_real, sio2_box  # noqa: E402


@pytest.fixture(scope="module")
def models(tmp_path_factory):
    d = tmp_path_factory.mktemp("m")
    return {"small": write_model(d, model_spec_small(), 101)[0],
            "real": write_model(d, model_spec_real(), 102)[0]}


def _same(a, b):
    assert a["energy"] == b["energy"]
    for k in ("atom_energy", "forces", "virial"):
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("which,precision,sizes", [
    ("small", "fp64", (64, 16)),   # 192 then 48 atoms
    ("small", "fp32", (64, 16)),
    ("real", "fp32", (40, 8)),     # 120 then 24 atoms
    ("real", "bf16", (40, 8)),
])
def test_noalloc_equals_compute(models, which, precision, sizes):
    model = sn.Model(models[which])
    ctx = sn.Context(model, precision=precision)
    torch.cuda.synchronize()
    mem0, torch0 = ctx.memory(), torch.cuda.memory_allocated()
    boxes = [sio2_box(n_si, seed=60 + n_si) for n_si in sizes]
    got = []
    for s in boxes:
        log(f"noalloc {which} {precision} n={s.n}")
        got.append(ctx.compute(s.pos, s.Z, s.cell, noalloc=True))
    torch.cuda.synchronize()
    assert ctx.memory() == mem0 and torch.cuda.memory_allocated() == torch0
    for s, g in zip(boxes, got):
        _same(g, ctx.compute(s.pos, s.Z, s.cell))
    # and once more after the pool-backed calls, smaller first
    for s in reversed(boxes):
        _same(ctx.compute(s.pos, s.Z, s.cell, noalloc=True), ctx.compute(s.pos, s.Z, s.cell))


def test_noalloc_refuses_oversize(models):
    ctx = sn.Context(sn.Model(models["real"]), precision="fp32")
    big = sio2_box(1000, seed=61)  # 3,000 atoms: several GiB of workspace
    log(f"noalloc oversize n={big.n}")
    with pytest.raises(sn.SNError) as ei:
        ctx.compute(big.pos, big.Z, big.cell, noalloc=True)
    assert ei.value.status == sn._lib.SN_ENOMEM and "static scratch" in str(ei.value)
    s = sio2_box(8, seed=62)
    _same(ctx.compute(s.pos, s.Z, s.cell, noalloc=True), ctx.compute(s.pos, s.Z, s.cell))
