"""Pin of the oracle's receiver-chunked message aggregation.

Above a size threshold the oracle evaluates the convolution over receiver-aligned
edge chunks, each recomputed in the backward pass (a memory bound only: the sum of
paper eq 3 over a receiver's edges is the same however the receivers are grouped).
The full-size stored reference values were written through that branch, so it is
checked here against the unchunked evaluation, which the other oracle tests pin
(finite differences, invariances, hand-computed special cases), with chunk sizes
small enough that every structure spans many chunks and chunk bounds fall inside
receivers' edge lists.
"""
import numpy as np
import pytest

from oracle.model import OracleModel, evaluate, evaluate_ghost
from synth import model_spec_small, model_spec_real, make_weights, sio2_box, rsa_box


def _model(which):
    spec = model_spec_small() if which == "small" else model_spec_real()
    return OracleModel(spec.config(), make_weights(spec, 101 if which == "small" else 102))


def _structures():
    s = sio2_box(8, seed=21)
    cell = np.array([[7.0, 0, 0], [1.5, 6.5, 0], [-1.0, 2.0, 6.8]])
    pos = rsa_box(cell, 16, 1.4, np.random.Generator(np.random.PCG64(5)))
    Z = np.where(np.arange(16) % 3 == 0, 14, 8).astype(np.int32)
    return [(s.pos, s.Z, s.cell), (pos, Z, cell)]


def _close(a, b, tol=1e-12):
    scale = max(1.0, float(np.max(np.abs(b))))
    assert np.max(np.abs(np.asarray(a) - np.asarray(b))) <= tol * scale


@pytest.mark.parametrize("which", ["small", "real"])
@pytest.mark.parametrize("fn", [evaluate, evaluate_ghost], ids=["whole_box", "ghost_shell"])
@pytest.mark.parametrize("chunk", [1, 37])
def test_chunked_equals_unchunked(which, fn, chunk):
    m = _model(which)
    for pos, Z, cell in _structures():
        m.chunk_edges = 200_000
        ref = fn(m, pos, Z, cell)
        n_edges = len(ref["edge_grad"])
        assert n_edges > 4 * chunk  # many chunks
        m.chunk_edges = chunk
        got = fn(m, pos, Z, cell)
        assert abs(got["energy"] - ref["energy"]) <= 1e-12 * max(1.0, abs(ref["energy"]))
        _close(got["atom_energy"], ref["atom_energy"])
        _close(got["forces"], ref["forces"])
        _close(got["forces_autograd"], ref["forces_autograd"])
        _close(got["virial"], ref["virial"])
