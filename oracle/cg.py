"""Real Clebsch-Gordan coupling tensors, from Racah's closed formula.

TEST INFRASTRUCTURE (see oracle/__init__.py).

The convolution couples a neighbour feature of degree l1 with the edge
spherical harmonic of degree l2 into degree l3 (the tensor product of the
paper's convolution block, section 2.2 and section 5.1).  Built here as:

  1. complex CG <l1 m1 l2 m2 | l3 m3> from Racah's formula (exact rationals
     under a square root);
  2. change of basis to the real harmonics of oracle/basis.py with the
     unitary Q (real_m = sum_mu Q[m, mu] complex_mu, Condon-Shortley phase);
  3. removal of the global phase (the result is real or purely imaginary);
  4. normalisation sum_{m1,m2} C[m1,m2,m3] C[m1,m2,m3'] = delta (it is
     already orthonormal; asserted);
  5. sign rule: the first nonzero entry in row-major (m1, m2, m3) order is
     positive.  A sign flip of a path is the same as negating that path's
     radial weights, so the rule is part of the model definition.

Parity is ignored (every triangle-allowed path is used): the paper lists
irreps as 128x0e+64x1e+32x2e yet couples them with l = 1 harmonics.
"""
from __future__ import annotations

import functools
import math
from fractions import Fraction

import numpy as np


def _f(n: int) -> int:
    return math.factorial(n)


def complex_cg(j1: int, m1: int, j2: int, m2: int, J: int, M: int) -> float:
    """<j1 m1 j2 m2 | J M> by Racah's formula (integer angular momenta)."""
    if m1 + m2 != M or abs(m1) > j1 or abs(m2) > j2 or abs(M) > J:
        return 0.0
    if J < abs(j1 - j2) or J > j1 + j2:
        return 0.0
    pre = Fraction((2 * J + 1) * _f(J + j1 - j2) * _f(J - j1 + j2) * _f(j1 + j2 - J),
                   _f(j1 + j2 + J + 1))
    pre *= _f(J + M) * _f(J - M) * _f(j1 - m1) * _f(j1 + m1) * _f(j2 - m2) * _f(j2 + m2)
    s = Fraction(0)
    for k in range(0, j1 + j2 + J + 2):
        args = [k, j1 + j2 - J - k, j1 - m1 - k, j2 + m2 - k, J - j2 + m1 + k, J - j1 - m2 + k]
        if min(args) < 0:
            continue
        den = 1
        for a in args:
            den *= _f(a)
        s += Fraction((-1) ** k, den)
    return math.sqrt(pre) * float(s) if s >= 0 else -math.sqrt(pre) * float(-s)


def real_basis_change(l: int) -> np.ndarray:
    """Q with real_m = sum_mu Q[m, mu] complex_mu, rows/cols ordered m = -l..l."""
    Q = np.zeros((2 * l + 1, 2 * l + 1), dtype=np.complex128)
    r2 = 1.0 / math.sqrt(2.0)
    for m in range(-l, l + 1):
        i = m + l
        if m > 0:
            Q[i, m + l] = (-1) ** m * r2
            Q[i, -m + l] = r2
        elif m < 0:
            Q[i, -m + l] = -1j * (-1) ** m * r2
            Q[i, m + l] = 1j * r2
        else:
            Q[i, l] = 1.0
    return Q


@functools.lru_cache(maxsize=None)
def real_cg(l1: int, l2: int, l3: int) -> np.ndarray:
    """Real coupling tensor C[m1, m2, m3] of shape (2l1+1, 2l2+1, 2l3+1)."""
    if not (abs(l1 - l2) <= l3 <= l1 + l2):
        raise ValueError("triangle rule violated")
    Cc = np.zeros((2 * l1 + 1, 2 * l2 + 1, 2 * l3 + 1))
    for m1 in range(-l1, l1 + 1):
        for m2 in range(-l2, l2 + 1):
            for m3 in range(-l3, l3 + 1):
                Cc[m1 + l1, m2 + l2, m3 + l3] = complex_cg(l1, m1, l2, m2, l3, m3)
    Q1, Q2, Q3 = real_basis_change(l1), real_basis_change(l2), real_basis_change(l3)
    # z_R = Q3 CG(Q1^H u_R, Q2^H v_R)
    C = np.einsum("ca,db,fe,abe->cdf", Q1.conj(), Q2.conj(), Q3, Cc)
    if np.abs(C.imag).max() > np.abs(C.real).max():
        C = C.imag
    else:
        C = C.real
    C = np.where(np.abs(C) < 1e-14, 0.0, C)
    gram = np.einsum("abc,abd->cd", C, C)
    assert np.allclose(gram, np.eye(2 * l3 + 1), atol=1e-12), (l1, l2, l3)
    flat = C.reshape(-1)
    first = flat[np.nonzero(np.abs(flat) > 1e-12)[0][0]]
    if first < 0:
        C = -C
    return C
