"""The C-ABI library loads and exports what include/sn.h declares (no device needed).

Host-only entry points are exercised here: the weights-file loader and the
Clebsch-Gordan table export, compared with the oracle's independently
generated tables.
"""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(sn_[a-z_0-9]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    import paper_2402_03789_amd as sn
    L = sn.lib()
    decl = _declared()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(L, name), name
    assert decl <= set(sn.EXPORTED) | decl


def test_cg_tables_match_oracle():
    import paper_2402_03789_amd as sn
    from oracle.cg import real_cg
    for l1 in range(4):
        for l2 in range(4):
            for l3 in range(abs(l1 - l2), min(l1 + l2, 3) + 1):
                np.testing.assert_allclose(sn.cg_table(l1, l2, l3), real_cg(l1, l2, l3), atol=1e-13)
    with pytest.raises(sn.SNError):
        sn.cg_table(1, 1, 3)


def test_model_load_and_parameter_count(tmp_path):
    import paper_2402_03789_amd as sn
    from synth import model_spec_real, model_spec_small, make_weights, write_weights
    spec = model_spec_real(species=tuple(range(1, 90)))
    p = str(tmp_path / "m.snw")
    write_weights(p, spec, make_weights(spec, 1))
    info = sn.Model(p).info()
    assert info["n_params"] == 842_432
    assert info["muls"] == [128, 64, 32] and info["n_layers"] == 5
    spec = model_spec_small()
    write_weights(p, spec, make_weights(spec, 1))
    assert sn.Model(p).info()["n_params"] == 56_400
    # a benchmark-family model (l_max 3 features and harmonics, section 4)
    from synth import model_spec_bench
    spec = model_spec_bench(32, 3)
    write_weights(p, spec, make_weights(spec, 1))
    info = sn.Model(p).info()
    assert info["l_max"] == 3 and info["l_sh"] == 3 and info["muls"] == [32] * 4
    assert info["n_params"] == sum(a.size for a in make_weights(spec, 1).values())


def test_model_load_rejects_bad_files(tmp_path):
    import paper_2402_03789_amd as sn
    p = tmp_path / "bad.snw"
    p.write_bytes(b"not a weights file")
    with pytest.raises(sn.SNError):
        sn.Model(str(p))
    with pytest.raises(sn.SNError):
        sn.Model(str(tmp_path / "missing.snw"))


def test_model_tensor_table_and_huber_helper(tmp_path):
    """Host-only training helpers: the weight-tensor table (names, offsets, counts matching the
    weights file) and the energy term of eq 9 against the oracle's closed form."""
    import ctypes as C
    import paper_2402_03789_amd as sn
    from paper_2402_03789_amd.train import huber_energy_loss
    from synth import model_spec_small, make_weights, write_weights
    spec = model_spec_small()
    path = str(tmp_path / "m.snw")
    write_weights(path, spec, make_weights(spec, 3))
    m = sn.Model(path)
    tabs = m.tensors()
    shapes = {name: shape for name, shape, _ in spec.tensor_shapes()}
    assert sorted(t[0] for t in tabs) == sorted(shapes)
    off = 0
    for name, shape, _ in spec.tensor_shapes():  # file order: contiguous, in drawing order
        o, cnt = next((o, c) for n, o, c in tabs if n == name)
        assert o == off and cnt == int(np.prod(shape))
        off += cnt
    assert off == m.info()["n_params"]
    # Huber energy term: quadratic and linear regimes
    E = np.array([-100.0, -50.0])
    ref = np.array([-100.0 + 0.004 * 12, -50.0 - 0.2 * 18])
    loss, g = huber_energy_loss(E, ref, [12, 18], 0.01)
    r = np.array([-0.004, 0.2])
    want = (0.5 * r[0] ** 2 + 0.01 * (0.2 - 0.005)) / 2
    assert abs(loss - want) < 1e-13 * want
    # (E/N - ref/N is rounded in float64: residual -0.004 to about 1e-14 relative)
    np.testing.assert_allclose(g, [r[0] / (2 * 12), 0.01 / (2 * 18)], rtol=1e-11)
    with pytest.raises(sn.SNError):
        huber_energy_loss(E, ref, [12, 0], 0.01)


def test_server_warmup_without_device_returns_error(tmp_path):
    """With no usable device every worker exits at start; a warm-up must report that
    (SN_EHIP) instead of waiting for workers that will never run it."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    import sys
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import paper_2402_03789_amd as sn
    from paper_2402_03789_amd.serve import Server
    from paper_2402_03789_amd._lib import SNError, SN_EHIP
    from gpu_common import write_model
    from synth import model_spec_small, serving_stream
    path, _ = write_model(tmp_path, model_spec_small((8, 14)), 5)
    srv = Server(sn.Model(path), n_streams=3, precision="fp32")
    _, s = serving_stream(count=1, seed=1, n_min=8, n_max=20)[0]
    Z = np.where(s.Z % 2 == 0, 8, 14)
    with pytest.raises(SNError) as e:
        srv.warmup(s.pos, Z, s.cell)
    assert e.value.status == SN_EHIP
    srv.close()
