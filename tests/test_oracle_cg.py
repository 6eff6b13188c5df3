"""Pins of the oracle's Clebsch-Gordan tables (the convolution's tensor product)."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle.cg import real_cg, complex_cg
from oracle.basis import real_sph_harm

PATHS2 = [(l1, l2, l3) for l1 in range(3) for l2 in range(3)
          for l3 in range(abs(l1 - l2), min(l1 + l2, 2) + 1)]
# the l_max = 3 benchmark models of the paper (section 4) use l <= 3
PATHS = [(l1, l2, l3) for l1 in range(4) for l2 in range(4)
         for l3 in range(abs(l1 - l2), min(l1 + l2, 3) + 1)]


def test_racah_matches_sympy():
    sympy = pytest.importorskip("sympy")
    from sympy.physics.quantum.cg import CG
    for j1 in range(4):
        for j2 in range(4):
            for J in range(abs(j1 - j2), min(j1 + j2, 3) + 1):
                for m1 in range(-j1, j1 + 1):
                    for m2 in range(-j2, j2 + 1):
                        M = m1 + m2
                        if abs(M) > J:
                            continue
                        ref = float(CG(j1, m1, j2, m2, J, M).doit())
                        assert abs(complex_cg(j1, m1, j2, m2, J, M) - ref) < 1e-14


def test_textbook_values():
    assert abs(complex_cg(1, 1, 1, -1, 0, 0) - 1 / math.sqrt(3)) < 1e-15
    assert abs(complex_cg(1, 0, 1, 0, 0, 0) + 1 / math.sqrt(3)) < 1e-15
    assert abs(complex_cg(1, 0, 1, 0, 2, 0) - math.sqrt(2 / 3)) < 1e-15
    assert abs(complex_cg(1, 1, 1, 0, 1, 1) - 1 / math.sqrt(2)) < 1e-15


def test_nonzero_counts():
    counts = [int((np.abs(real_cg(*p)) > 1e-12).sum()) for p in PATHS2]
    assert counts == [1, 3, 5, 3, 3, 6, 11, 11, 16, 5, 11, 16, 5, 16, 25]
    assert sum(counts) == 137
    assert len(PATHS) == 34


@pytest.mark.parametrize("p", PATHS)
def test_orthonormal_columns(p):
    C = real_cg(*p)
    np.testing.assert_allclose(np.einsum("abc,abd->cd", C, C), np.eye(2 * p[2] + 1), atol=1e-13)


@pytest.mark.parametrize("l1,l2", [(1, 1), (1, 2), (2, 2), (2, 1), (3, 1), (3, 3)])
def test_completeness(l1, l2):
    tot = np.zeros((2 * l1 + 1, 2 * l2 + 1, 2 * l1 + 1, 2 * l2 + 1))
    for l3 in range(abs(l1 - l2), l1 + l2 + 1):
        C = real_cg(l1, l2, l3)
        tot += np.einsum("abc,dec->abde", C, C)
    eye = np.einsum("ad,be->abde", np.eye(2 * l1 + 1), np.eye(2 * l2 + 1))
    np.testing.assert_allclose(tot, eye, atol=1e-13)


def test_closed_forms():
    for l in range(4):
        np.testing.assert_allclose(real_cg(0, l, l)[0], np.eye(2 * l + 1), atol=1e-15)
        np.testing.assert_allclose(real_cg(l, 0, l)[:, 0, :], np.eye(2 * l + 1), atol=1e-15)
        np.testing.assert_allclose(real_cg(l, l, 0)[:, :, 0], np.eye(2 * l + 1) / math.sqrt(2 * l + 1),
                                   atol=1e-15)
    # (1,1,1) is the cross product / sqrt(2) in (y, z, x) labels
    C = real_cg(1, 1, 1)
    a, b = np.random.default_rng(0).normal(size=(2, 3))
    P = [1, 2, 0]  # (y,z,x) component k holds xyz component P[k]
    ax, bx = np.zeros(3), np.zeros(3)
    ax[P], bx[P] = a, b
    z = np.einsum("abc,a,b->c", C, a, b)
    np.testing.assert_allclose(z, np.cross(ax, bx)[P] / math.sqrt(2), atol=1e-14)


def _wigner(l, R, pts):
    Y = real_sph_harm(torch.tensor(pts), 3)[l].numpy()
    Yr = real_sph_harm(torch.tensor(pts @ R.T), 3)[l].numpy()
    return np.linalg.lstsq(Y, Yr, rcond=None)[0].T


@pytest.mark.parametrize("p", PATHS)
def test_equivariance(p):
    rng = np.random.default_rng(1)
    pts = rng.normal(size=(40, 3))
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    C = real_cg(*p)
    for seed in range(3):
        R = Rotation.random(random_state=seed).as_matrix()
        D = [_wigner(l, R, pts) for l in range(4)]
        u, v = rng.normal(size=2 * p[0] + 1), rng.normal(size=2 * p[1] + 1)
        lhs = np.einsum("abc,a,b->c", C, D[p[0]] @ u, D[p[1]] @ v)
        rhs = D[p[2]] @ np.einsum("abc,a,b->c", C, u, v)
        np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_sign_rule():
    for p in PATHS:
        flat = real_cg(*p).reshape(-1)
        assert flat[np.nonzero(np.abs(flat) > 1e-12)[0][0]] > 0
