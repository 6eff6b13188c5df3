"""Lists built with a skin are evaluated over their pairs inside r_c only.  Beyond r_c the
envelope and its derivative are exact zeros (paper section 5.1), so the compacted
evaluation gives the energies, forces and virial of the whole list up to the grouping of
floating-point sums (a degree narrower than a wave deals a receiver's edges to lane
groups by position, and the virial is summed in chunks of the list), on the build and on
every kept-list step."""
import numpy as np
import pytest

from gpu_common import log, write_model

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2402_03789_amd as sn  # noqa: E402
from synth import model_spec_real, sio2_box  # noqa: E402


@pytest.fixture(scope="module")
def model_path(tmp_path_factory):
    path, _ = write_model(tmp_path_factory.mktemp("m"), model_spec_real(), 107)
    return path


def _contexts(model_path, precision, skin, domains=None):
    m = sn.Model(model_path)
    on = sn.Context(m, precision=precision, skin=skin)
    off = sn.Context(m, precision=precision, skin=skin)
    off.set_edge_compaction(False)
    if domains:
        on.set_domains(*domains)
        off.set_domains(*domains)
    return on, off


# rounding-level bounds per form: relative to the RMS per-atom energy, the largest force
# component and the largest virial component
TOL = {"fp64": (1e-12, 1e-12, 1e-12), "fp32": (1e-6, 1e-6, 1e-6), "bf16": (2e-2, 2e-2, 2e-2)}


def _same(a, b, precision):
    te, tf, tw = TOL[precision]
    rms = np.sqrt(np.mean(b["atom_energy"] ** 2))
    de = np.abs(a["atom_energy"] - b["atom_energy"]).max() / rms
    df = np.abs(a["forces"] - b["forces"]).max() / np.abs(b["forces"]).max()
    dw = np.abs(a["virial"] - b["virial"]).max() / np.abs(b["virial"]).max()
    log(f"  compacted vs whole list: energy {de:.1e}, forces {df:.1e}, virial {dw:.1e}")
    assert de <= te and df <= tf and dw <= tw


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_compacted_build_equals_whole_list(model_path, precision):
    s = sio2_box(64, seed=11)
    on, off = _contexts(model_path, precision, 1.0)
    a = on.compute(s.pos, s.Z, s.cell)
    b = off.compute(s.pos, s.Z, s.cell)
    built = on.graph_size()[2]
    e_on, p_on = on.evaluated_edges()
    e_off, p_off = off.evaluated_edges()
    log(f"{precision}: built {built} edges, evaluated {e_on} ({p_on} pairs) against {e_off}")
    assert off.graph_size()[2] == built == e_off
    assert 0 < e_on < built and p_on < p_off
    _same(a, b, precision)


@pytest.mark.parametrize("domains", [None, (2, 1, 1)])
def test_kept_list_steps_equal_whole_list(model_path, domains):
    s = sio2_box(80, seed=12)
    rng = np.random.default_rng(4)
    on, off = _contexts(model_path, "fp64", 1.0, domains)
    pos = s.pos.copy()
    for step in range(4):
        if step:
            # at most 0.08 A per coordinate and step: |displacement| <= 0.42 A < skin / 2
            pos = pos + rng.uniform(-0.08, 0.08, size=pos.shape)
        a = on.compute(pos, s.Z, s.cell)
        b = off.compute(pos, s.Z, s.cell)
        _same(a, b, "fp64")
        log(f"step {step}: evaluated {on.evaluated_edges()[0]} of {on.graph_size()[2]} edges")
        if step == 0:
            on.set_graph_reuse(True)
            off.set_graph_reuse(True)
    # the kept, compacted list against a fresh build at the final positions
    fresh = sn.Context(sn.Model(model_path), precision="fp64", skin=1.0).compute(pos, s.Z, s.cell)
    assert abs(a["energy"] - fresh["energy"]) < 1e-9 * s.n
    np.testing.assert_allclose(a["forces"], fresh["forces"], atol=1e-10)
