"""Pins of the oracle's neighbour lists, ghost shells and subdomains."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle.graph import periodic_edges, ghost_shell, subdomains, wrap
from synth import sio2_box, rsa_box


def _edge_set(recv, send, shift):
    return set(zip(recv.tolist(), send.tolist(), map(tuple, shift.tolist())))


def test_cubic_box_matches_kdtree():
    s = sio2_box(64, seed=11)
    L = s.cell[0, 0]
    rc = 4.0
    recv, send, shift = periodic_edges(s.pos, s.cell, rc)
    tree = cKDTree(s.pos, boxsize=L)
    pairs = tree.query_pairs(rc, output_type="ndarray")
    assert len(recv) == 2 * len(pairs)  # L > 2 rc: one image per pair, both directions
    got = set(zip(recv.tolist(), send.tolist()))
    want = set(map(tuple, pairs.tolist())) | set((b, a) for a, b in pairs.tolist())
    assert got == want


@pytest.mark.parametrize("a,rc,count", [(2.0, 2.5, 6), (2.0, 3.0, 18), (2.0, 3.5, 26), (2.0, 4.1, 32)])
def test_simple_cubic_self_images(a, rc, count):
    # one atom in a cubic cell smaller than r_c: neighbours are its own images
    recv, send, shift = periodic_edges(np.zeros((1, 3)), np.eye(3) * a, rc)
    assert len(recv) == count


def test_fcc_coordination():
    # conventional fcc cell (4 atoms, a = 4): 12 nearest neighbours at a/sqrt(2)
    a = 4.0
    frac = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    recv, send, shift = periodic_edges(frac * a, np.eye(3) * a, 3.0)
    assert len(recv) == 4 * 12


def _triclinic(seed):
    rng = np.random.default_rng(seed)
    cell = np.array([[6.0, 0, 0], [2.5, 5.5, 0], [-1.5, 1.8, 5.2]])
    pos = rsa_box(cell, 20, 1.2, np.random.Generator(np.random.PCG64(seed)))
    return pos, cell


@pytest.mark.parametrize("seed", [0, 1])
def test_ghost_shell_reproduces_periodic_edges(seed):
    pos, cell = _triclinic(seed)
    posw = wrap(pos, cell)
    rc = 4.0
    recv, send, shift = periodic_edges(posw, cell, rc)
    D = ghost_shell(posw, cell, rc)
    owner = np.concatenate([D["local"], D["ghost_owner"]])
    sh = np.concatenate([np.zeros((len(D["local"]), 3), int), D["ghost_shift"]])
    got = _edge_set(D["local"][D["recv"]], owner[D["send"]], sh[D["send"]])
    assert got == _edge_set(recv, send, shift)


def test_subdomains_partition_and_edges():
    pos, cell = _triclinic(3)
    posw = wrap(pos, cell)
    rc = 3.5
    recv, send, shift = periodic_edges(posw, cell, rc)
    doms = subdomains(posw, cell, rc, (2, 2, 1))
    locs = np.concatenate([d["local"] for d in doms])
    assert sorted(locs.tolist()) == list(range(len(pos)))
    got = set()
    for D in doms:
        owner = np.concatenate([D["local"], D["ghost_owner"]])
        sh = np.concatenate([np.zeros((len(D["local"]), 3), int), D["ghost_shift"]])
        got |= _edge_set(D["local"][D["recv"]], owner[D["send"]], sh[D["send"]])
    assert got == _edge_set(recv, send, shift)


def test_wrap_into_cell():
    pos, cell = _triclinic(4)
    shifted = pos + np.array([3, -2, 5]) @ cell
    f = wrap(shifted, cell) @ np.linalg.inv(cell)
    assert f.min() >= 0 and f.max() < 1
    np.testing.assert_allclose(wrap(shifted, cell), wrap(pos, cell), atol=1e-12)


def test_kdtree_path_matches_brute_force():
    from oracle.graph import _kdtree_edges
    s = sio2_box(400, seed=13)  # 1200 atoms: brute force is still quick
    a = periodic_edges(s.pos, s.cell, 5.0)
    b = _kdtree_edges(wrap(s.pos, s.cell), s.cell, 5.0)
    c = periodic_edges(wrap(s.pos, s.cell), s.cell, 5.0)
    assert _edge_set(*b) == _edge_set(*c)
    assert len(a[0]) == len(b[0])
