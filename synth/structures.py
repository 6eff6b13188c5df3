"""Seeded synthetic atomic structures.

Random sequential addition (RSA): atoms are inserted one at a time at
uniformly random fractional coordinates and rejected when closer than a
minimum distance to any periodic image of an atom already placed.  The
boxes reproduce the densities and compositions of the paper's workloads:

* SiO2 at 2.2 g/cm^3 (the benchmark section measures alpha-quartz SiO2);
* Si3N4 at 3.1 g/cm^3 (the large-scale amorphous Si3N4 section);
* a stream of small triclinic multi-element cells standing in for the
  Materials Project structures behind the general-purpose model.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

AMU_G = 1.66053906660e-24  # grams per atomic mass unit
A3_CM3 = 1e-24  # cm^3 per cubic angstrom

# Standard atomic weights (amu) for Z = 1..89, rounded.  Used only to turn a
# drawn mass density into a cell volume.
_MASS_TABLE = [
    1.008, 4.003, 6.94, 9.012, 10.81, 12.011, 14.007, 15.999, 18.998, 20.180,
    22.990, 24.305, 26.982, 28.085, 30.974, 32.06, 35.45, 39.948, 39.098, 40.078,
    44.956, 47.867, 50.942, 51.996, 54.938, 55.845, 58.933, 58.693, 63.546, 65.38,
    69.723, 72.630, 74.922, 78.971, 79.904, 83.798, 85.468, 87.62, 88.906, 91.224,
    92.906, 95.95, 97.0, 101.07, 102.91, 106.42, 107.87, 112.41, 114.82, 118.71,
    121.76, 127.60, 126.90, 131.29, 132.91, 137.33, 138.91, 140.12, 140.91, 144.24,
    145.0, 150.36, 151.96, 157.25, 158.93, 162.50, 164.93, 167.26, 168.93, 173.05,
    174.97, 178.49, 180.95, 183.84, 186.21, 190.23, 192.22, 195.08, 196.97, 200.59,
    204.38, 207.2, 208.98, 209.0, 210.0, 222.0, 223.0, 226.0, 227.0,
]
MASSES = {z: m for z, m in enumerate(_MASS_TABLE, start=1)}
MASSES[14] = 28.0855  # Si
MASSES[8] = 15.999    # O
MASSES[7] = 14.007    # N


@dataclasses.dataclass
class Structure:
    """One periodic configuration.  Cell rows are the lattice vectors (A)."""
    pos: np.ndarray          # [N, 3] float64, Cartesian, angstrom
    Z: np.ndarray            # [N] int32 atomic numbers
    cell: np.ndarray         # [3, 3] float64, rows a1, a2, a3
    pbc: tuple = (True, True, True)
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def masses(self) -> np.ndarray:
        return np.array([MASSES[int(z)] for z in self.Z], dtype=np.float64)


def _perp_widths(cell: np.ndarray) -> np.ndarray:
    vol = abs(np.linalg.det(cell))
    a, b, c = cell
    return np.array([vol / np.linalg.norm(np.cross(b, c)),
                     vol / np.linalg.norm(np.cross(c, a)),
                     vol / np.linalg.norm(np.cross(a, b))])


def rsa_box(cell: np.ndarray, n: int, dmin: float, rng: np.random.Generator,
            max_tries: int = 200) -> np.ndarray:
    """Random sequential addition of n points in a periodic cell.

    Bins tile fractional space with a perpendicular width of at least dmin,
    so every conflicting image lies in one of the 27 surrounding bins.  Each
    try draws one uniform fractional point (three doubles from `rng`) and is
    rejected when any stored point image in those bins lies closer than dmin.
    """
    cell = np.asarray(cell, dtype=np.float64)
    widths = _perp_widths(cell)
    if np.any(widths <= dmin):
        raise ValueError("cell thinner than the minimum distance")
    nb = np.maximum(1, np.floor(widths / dmin).astype(int))
    n0, n1, n2 = (int(x) for x in nb)
    bins = [[] for _ in range(n0 * n1 * n2)]
    neigh: dict = {}  # bin -> distinct (neighbour bin, image shift) pairs
    frac = np.empty((n, 3))
    d2min = dmin * dmin
    offs = [(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)]
    placed = 0
    tries = 0
    limit = max_tries * n
    while placed < n:
        tries += 1
        if tries > limit:
            raise RuntimeError(f"RSA failed after {tries} tries ({placed}/{n})")
        f = rng.random(3)
        b0 = min(int(f[0] * n0), n0 - 1)
        b1 = min(int(f[1] * n1), n1 - 1)
        b2 = min(int(f[2] * n2), n2 - 1)
        home = (b0 * n1 + b1) * n2 + b2
        nl = neigh.get(home)
        if nl is None:
            nl = []
            seen = set()
            for o in offs:
                c0, c1, c2 = b0 + o[0], b1 + o[1], b2 + o[2]
                sh = (c0 // n0, c1 // n1, c2 // n2)
                k = ((c0 - sh[0] * n0) * n1 + (c1 - sh[1] * n1)) * n2 + (c2 - sh[2] * n2)
                if (k,) + sh in seen:
                    continue
                seen.add((k,) + sh)
                nl.append((k, sh))
            neigh[home] = nl
        idx = []
        shifts = []
        for k, sh in nl:
            lst = bins[k]
            if lst:
                idx.extend(lst)
                shifts.extend([sh] * len(lst))
        if idx:
            d = (frac[idx] + np.array(shifts, dtype=np.float64) - f) @ cell
            if np.any(np.einsum("ij,ij->i", d, d) < d2min):
                continue
        frac[placed] = f
        bins[home].append(placed)
        placed += 1
    return frac @ cell


def _cubic_box(counts: dict, density: float, dmin: float, seed: int,
               jitter: float = 0.0, name: str = "") -> Structure:
    mass = sum(MASSES[z] * c for z, c in counts.items())
    vol = mass * AMU_G / density / A3_CM3
    L = vol ** (1.0 / 3.0)
    cell = np.eye(3) * L
    n = sum(counts.values())
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rsa_box(cell, n, dmin, rng)
    Z = np.concatenate([np.full(c, z, dtype=np.int32) for z, c in counts.items()])
    Z = Z[rng.permutation(n)]
    if jitter > 0:
        pos = pos + rng.normal(0.0, jitter, size=pos.shape)
    return Structure(pos=pos, Z=Z.astype(np.int32), cell=cell, name=name)


def sio2_box(n_si: int, density: float = 2.2, dmin: float = 1.4, seed: int = 1) -> Structure:
    """SiO2 at the density of the benchmark section's silica."""
    return _cubic_box({14: n_si, 8: 2 * n_si}, density, dmin, seed,
                      name=f"SiO2-{3 * n_si}")


def si3n4_box(n_si: int, density: float = 3.1, dmin: float = 1.5, seed: int = 4,
              jitter: float = 0.05) -> Structure:
    """Amorphous-density Si3N4 as in the large-scale melt-quench section."""
    n_n = n_si * 4 // 3
    return _cubic_box({14: n_si, 7: n_n}, density, dmin, seed, jitter=jitter,
                      name=f"Si3N4-{n_si + n_n}")


def _random_cell(rng: np.random.Generator, vol: float) -> np.ndarray:
    while True:
        ang = np.radians(rng.uniform(60.0, 120.0, size=3))
        ca, cb, cg = np.cos(ang)
        metric_det = 1 - ca * ca - cb * cb - cg * cg + 2 * ca * cb * cg
        if metric_det <= 0.05:
            continue
        ratios = rng.uniform(1.0, 1.5, size=3)
        sg = math.sin(ang[2])
        a = np.array([1.0, 0.0, 0.0])
        b = np.array([cg, sg, 0.0])
        cx = cb
        cy = (ca - cb * cg) / sg
        cz = math.sqrt(max(1.0 - cx * cx - cy * cy, 0.0))
        c = np.array([cx, cy, cz])
        cell = np.stack([a * ratios[0], b * ratios[1], c * ratios[2]])
        scale = (vol / abs(np.linalg.det(cell))) ** (1.0 / 3.0)
        return cell * scale


def serving_stream(count: int = 2000, seed: int = 6, n_min: int = 8, n_max: int = 2048,
                   rate: float = 200.0, dmin: float = 1.0):
    """Stream of requests: (arrival_time_s, Structure).

    Atom counts are log-uniform in [n_min, n_max]; 1-4 species drawn from
    Z = 1..89; triclinic cells with angles in [60, 120] degrees and length
    ratios in [1, 1.5]; volume from a mass density in [2, 6] g/cm^3 with a
    floor of 10 A^3 per atom; Poisson arrivals at `rate` per second.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for r in range(count):
        n = int(math.floor(math.exp(rng.uniform(math.log(n_min), math.log(n_max + 1)))))
        n = min(max(n, n_min), n_max)
        k = int(rng.integers(1, 5))
        species = rng.choice(np.arange(1, 90), size=k, replace=False)
        Z = species[rng.integers(0, k, size=n)].astype(np.int32)
        rho = rng.uniform(2.0, 6.0)
        mass = float(sum(MASSES[int(z)] for z in Z))
        vol = max(mass * AMU_G / rho / A3_CM3, 10.0 * n)
        cell = _random_cell(rng, vol)
        pos = rsa_box(cell, n, dmin, rng)
        t += rng.exponential(1.0 / rate)
        out.append((t, Structure(pos=pos, Z=Z, cell=cell, name=f"req{r}")))
    return out


# The five workloads.  Index 0 is the small case that the oracle finishes in
# seconds; index 1 is the real-size SiO2 box.
CONFIGS = {
    "small": dict(kind="sio2", n_si=64, seed=1, weights_seed=101, model="small"),
    "sio2_24k": dict(kind="sio2", n_si=8000, seed=2, weights_seed=102, model="real"),
    "si3n4_112k": dict(kind="si3n4", n_si=48000, seed=4, weights_seed=102, model="real"),
}


def config_structure(name: str) -> Structure:
    c = CONFIGS[name]
    if c["kind"] == "sio2":
        return sio2_box(c["n_si"], seed=c["seed"])
    if c["kind"] == "si3n4":
        return si3n4_box(c["n_si"], seed=c["seed"])
    raise KeyError(name)
