"""Pins of the oracle's edge basis against closed forms and library routines.

Section 5.1 of the paper: spherical harmonics up to l = 2 and 8 radial Bessel
functions; the envelope is a p = 6 polynomial (the paper does not print it).
"""
import math

import numpy as np
import pytest
import torch
from scipy import integrate, special
from scipy.spatial.transform import Rotation

from oracle.basis import real_sph_harm, bessel_basis, poly_envelope, radial_basis


def _unit(n, seed):
    v = np.random.default_rng(seed).normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_sh_at_z_axis():
    Y = real_sph_harm(torch.tensor([[0.0, 0.0, 1.0]], dtype=torch.float64), 3)
    got = torch.cat(Y, dim=1)[0].numpy()
    want = [1, 0, math.sqrt(3), 0, 0, 0, math.sqrt(5), 0, 0, 0, 0, 0, math.sqrt(7), 0, 0, 0]
    np.testing.assert_allclose(got, want, atol=1e-15)


def test_sh_component_normalisation():
    Y = real_sph_harm(torch.tensor(_unit(200, 1)), 3)
    for l in range(4):
        np.testing.assert_allclose((Y[l] ** 2).sum(1).numpy(), 2 * l + 1, rtol=1e-13)


def test_sh_addition_theorem_legendre():
    a, b = _unit(100, 2), _unit(100, 3)
    Ya = real_sph_harm(torch.tensor(a), 3)
    Yb = real_sph_harm(torch.tensor(b), 3)
    cos = (a * b).sum(1)
    for l in range(4):
        lhs = (Ya[l] * Yb[l]).sum(1).numpy()
        np.testing.assert_allclose(lhs, (2 * l + 1) * special.eval_legendre(l, cos), atol=1e-12)


def test_sh_orthogonal_on_sphere():
    # Gauss-Legendre in cos(theta) x uniform phi: exact for these polynomials
    xs, ws = np.polynomial.legendre.leggauss(8)
    phis = np.arange(16) * 2 * np.pi / 16
    ct, ph = np.meshgrid(xs, phis, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    pts = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wts = (ws[:, None] * np.ones_like(phis)[None] * (2 * np.pi / 16)).reshape(-1) / (4 * np.pi)
    Y = torch.cat(real_sph_harm(torch.tensor(pts), 3), dim=1).numpy()
    gram = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-13)


def test_sh_match_scipy_real_harmonics():
    # real combinations of scipy's complex Y_l^m (Condon-Shortley phase):
    # m > 0: sqrt(2) (-1)^m Re Y_l^m ; m < 0: sqrt(2) (-1)^m Im Y_l^|m| ; times sqrt(4 pi)
    pts = _unit(30, 4)
    theta = np.arccos(pts[:, 2])
    phi = np.arctan2(pts[:, 1], pts[:, 0])
    Y = real_sph_harm(torch.tensor(pts), 3)
    for l in range(4):
        for m in range(-l, l + 1):
            c = special.sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                ref = math.sqrt(2) * (-1) ** m * c.real
            elif m < 0:
                ref = math.sqrt(2) * (-1) ** m * c.imag
            else:
                ref = c.real
            np.testing.assert_allclose(Y[l][:, m + l].numpy(), math.sqrt(4 * math.pi) * ref,
                                       atol=1e-12)


def test_sh_rotation_orthogonal():
    pts = _unit(40, 5)
    R = Rotation.random(random_state=7).as_matrix()
    Y = real_sph_harm(torch.tensor(pts), 3)
    Yr = real_sph_harm(torch.tensor(pts @ R.T), 3)
    for l in range(1, 4):
        D = np.linalg.lstsq(Y[l].numpy(), Yr[l].numpy(), rcond=None)[0].T
        np.testing.assert_allclose(D @ D.T, np.eye(2 * l + 1), atol=1e-12)
        np.testing.assert_allclose(Y[l].numpy() @ D.T, Yr[l].numpy(), atol=1e-12)
    # l = 1 is the rotation itself in (y, z, x) order
    P = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]])
    D1 = np.linalg.lstsq(Y[1].numpy(), Yr[1].numpy(), rcond=None)[0].T
    np.testing.assert_allclose(D1, P @ R @ P.T, atol=1e-12)


@pytest.mark.parametrize("rc", [4.0, 5.0])
def test_bessel_orthogonality(rc):
    for n in range(1, 9):
        for m in range(1, 9):
            f = lambda r: float(bessel_basis(torch.tensor([r], dtype=torch.float64), rc, 8)[0, n - 1]
                                * bessel_basis(torch.tensor([r], dtype=torch.float64), rc, 8)[0, m - 1]) * r * r
            v, _ = integrate.quad(f, 1e-9, rc, limit=200)
            assert abs(v - (2.0 / rc if n == m else 0.0)) < 1e-8


def test_bessel_small_r_limit():
    rc = 5.0
    b = bessel_basis(torch.tensor([1e-7], dtype=torch.float64), rc, 8)[0].numpy()
    np.testing.assert_allclose(b, 2 * np.arange(1, 9) * np.pi / rc ** 2, rtol=1e-10)


def test_envelope_values_and_derivatives():
    x = torch.tensor([0.0, 1.0, 1.2], dtype=torch.float64, requires_grad=True)
    u = poly_envelope(x, 6)
    assert float(u[0]) == 1.0 and abs(float(u[1])) < 1e-14 and float(u[2]) == 0.0
    (g,) = torch.autograd.grad(u.sum(), x, create_graph=True)
    (g2,) = torch.autograd.grad(g.sum(), x)
    assert abs(float(g[1])) < 1e-12 and abs(float(g2[1])) < 1e-10
    assert abs(float(g[0])) < 1e-14
    # coefficients 28, 48, 21 for p = 6
    xs = torch.tensor([0.3, 0.7], dtype=torch.float64)
    want = 1 - 28 * xs ** 6 + 48 * xs ** 7 - 21 * xs ** 8
    np.testing.assert_allclose(poly_envelope(xs, 6).numpy(), want.numpy(), rtol=1e-15)


def test_radial_basis_vanishes_at_cutoff():
    r = torch.tensor([4.999999, 5.0, 6.0], dtype=torch.float64)
    rho = radial_basis(r, 5.0, 8)
    assert float(rho.abs().max()) < 1e-20 + 1e-12


def test_activation_scale():
    from synth import ACT_SCALE
    f = lambda z: (z * special.expit(z)) ** 2 * math.exp(-z * z / 2) / math.sqrt(2 * math.pi)
    v, _ = integrate.quad(f, -40, 40, epsabs=1e-14)
    assert abs(ACT_SCALE - 1 / math.sqrt(v)) < 1e-12
