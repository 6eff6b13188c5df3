"""Edge basis: real spherical harmonics, Bessel radial functions, envelope.

TEST INFRASTRUCTURE (see oracle/__init__.py).

The paper (section 5.1) builds the convolution filter from spherical
harmonics up to l = 2 (l = 3 in the benchmark models of section 4)
and 8 radial Bessel functions of the interatomic
distance; the distance and unit displacement enter the edge feature
(section 2).  The exact basis, ordering and normalisation are not printed;
the reading used throughout is:

  Y^0 = 1
  Y^1 = sqrt(3) (y, z, x)                          m = -1, 0, 1
  Y^2 = (sqrt(15) xy, sqrt(15) yz, sqrt(5)/2 (3z^2 - 1),
         sqrt(15) xz, sqrt(15)/2 (x^2 - y^2))       m = -2 .. 2
  Y^3 = (sqrt(70)/4 y(3x^2 - y^2), sqrt(105) xyz, sqrt(42)/4 y(5z^2 - 1),
         sqrt(7)/2 z(5z^2 - 3), sqrt(42)/4 x(5z^2 - 1),
         sqrt(105)/2 z(x^2 - y^2), sqrt(70)/4 x(x^2 - 3y^2))   m = -3 .. 3
         (for the l_max = 3 benchmark models of section 4)
  (|Y^l|^2 = 2l + 1 on the unit sphere)

  B_n(r) = (2 / r_c) sin(n pi r / r_c) / r,  n = 1..8
  u(x)   = 1 - (p+1)(p+2)/2 x^p + p(p+2) x^(p+1) - p(p+1)/2 x^(p+2),  x = r/r_c < 1
  rho_n  = B_n(r) u(r / r_c)
"""
from __future__ import annotations

import math

import torch


def real_sph_harm(rhat: torch.Tensor, l_max: int) -> list:
    """Real spherical harmonics of unit vectors rhat [..., 3]; list per l of [..., 2l+1]."""
    x, y, z = rhat[..., 0], rhat[..., 1], rhat[..., 2]
    out = [torch.ones_like(x)[..., None]]
    if l_max >= 1:
        s3 = math.sqrt(3.0)
        out.append(torch.stack([s3 * y, s3 * z, s3 * x], dim=-1))
    if l_max >= 2:
        s15 = math.sqrt(15.0)
        s5 = math.sqrt(5.0)
        out.append(torch.stack([
            s15 * x * y,
            s15 * y * z,
            0.5 * s5 * (3.0 * z * z - 1.0),
            s15 * x * z,
            0.5 * s15 * (x * x - y * y),
        ], dim=-1))
    if l_max >= 3:  # on the unit sphere (r = 1); m = -3..3
        c3, c2, c1, c0 = math.sqrt(70.0) / 4.0, math.sqrt(105.0), math.sqrt(42.0) / 4.0, math.sqrt(7.0) / 2.0
        out.append(torch.stack([
            c3 * y * (3.0 * x * x - y * y),
            c2 * x * y * z,
            c1 * y * (5.0 * z * z - 1.0),
            c0 * z * (5.0 * z * z - 3.0),
            c1 * x * (5.0 * z * z - 1.0),
            0.5 * c2 * z * (x * x - y * y),
            c3 * x * (x * x - 3.0 * y * y),
        ], dim=-1))
    if l_max >= 4:
        raise NotImplementedError("l_max <= 3 in this model family")
    return out


def bessel_basis(r: torch.Tensor, r_cut: float, n_basis: int) -> torch.Tensor:
    """B_n(r) = (2/r_c) sin(n pi r / r_c) / r for n = 1..n_basis; r [...] -> [..., n_basis]."""
    n = torch.arange(1, n_basis + 1, dtype=r.dtype)
    return (2.0 / r_cut) * torch.sin(n * math.pi * r[..., None] / r_cut) / r[..., None]


def poly_envelope(x: torch.Tensor, p: int = 6) -> torch.Tensor:
    """Polynomial cutoff envelope with u(0)=1 and u(1)=u'(1)=u''(1)=0; zero for x >= 1."""
    c1 = (p + 1) * (p + 2) / 2.0
    c2 = p * (p + 2.0)
    c3 = p * (p + 1) / 2.0
    u = 1.0 - c1 * x ** p + c2 * x ** (p + 1) - c3 * x ** (p + 2)
    return torch.where(x < 1.0, u, torch.zeros_like(x))


def radial_basis(r: torch.Tensor, r_cut: float, n_basis: int, p: int = 6) -> torch.Tensor:
    """rho_n(r) = B_n(r) u(r / r_c)."""
    return bessel_basis(r, r_cut, n_basis) * poly_envelope(r / r_cut, p)[..., None]
