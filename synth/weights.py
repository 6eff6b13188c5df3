"""Seeded synthetic model weights and the weights-file writer.

The trained general-purpose model is not available, so every weight is drawn
from N(0, 1/fan_in) with NumPy's PCG64 generator, in the fixed order listed
by `ModelSpec.tensor_shapes()`.  fan_in is the number of input channels of
each matrix (the species count for the embedding).

Weights file layout ("SNW1"): 8-byte magic, little-endian u64 header length,
a UTF-8 JSON header {"format", "config", "tensors": [{name, shape, offset}]},
zero padding to a 64-byte boundary, then every tensor as little-endian
float64 in row-major order at its `offset` from the start of the data block.
"""
from __future__ import annotations

import dataclasses
import json
import math
import struct

import numpy as np

# 1 / sqrt(E[SiLU(z)^2]) for z ~ N(0, 1): second-moment normalisation of the
# activation, so random-init signals keep unit scale through the layers.
ACT_SCALE = 1.6765324703310913

MAGIC = b"SNW1\0\0\0\0"


@dataclasses.dataclass
class ModelSpec:
    n_layers: int
    muls: tuple                # channel multiplicity per l = 0..l_max
    l_sh: int                  # highest spherical-harmonic degree on edges
    r_cut: float               # cutoff radius, angstrom
    species: tuple             # atomic numbers, in embedding-row order
    n_basis: int = 8           # radial Bessel functions
    hidden: int = 64           # radial-MLP hidden width
    envelope_p: int = 6        # polynomial envelope exponent
    k_avg: float = 1.0         # average neighbour count used to normalise messages
    sigma: float = 1.0         # per-atom energy scale
    shift: tuple = ()          # per-species energy shift (eV); zeros if empty
    act_scale: float = ACT_SCALE
    gate: str = "silu"         # activation applied to gate scalars

    @property
    def l_max(self) -> int:
        return len(self.muls) - 1

    def _in_ls(self, t):
        return [0] if t == 0 else [l for l in range(self.l_max + 1) if self.muls[l] > 0]

    def _out_ls(self, t):
        if t == self.n_layers - 1:
            return [0]
        return [l for l in range(self.l_max + 1) if self.muls[l] > 0]

    def _paths(self, t):
        ins, outs = self._in_ls(t), self._out_ls(t)
        return [(l1, l2, l3) for l1 in ins for l2 in range(self.l_sh + 1)
                for l3 in range(abs(l1 - l2), min(l1 + l2, self.l_max) + 1) if l3 in outs]

    def _gate_mul(self, t, l):
        if t == self.n_layers - 1:
            return self.muls[0] if l == 0 else 0
        if l == 0:
            return sum(self.muls)
        return self.muls[l]

    def tensor_shapes(self):
        """[(name, shape, fan_in)] in drawing order."""
        C0 = self.muls[0]
        out = [("embed", (len(self.species), C0), len(self.species))]
        for t in range(self.n_layers):
            ins = self._in_ls(t)
            for l in ins:
                m = self.muls[l]
                out.append((f"l{t}.lin1.{l}", (m, m), m))
            for l in ins:
                g = self._gate_mul(t, l)
                if g > 0:
                    out.append((f"l{t}.linsc.{l}", (self.muls[l], g), self.muls[l]))
            paths = self._paths(t)
            P = sum(self.muls[l1] for (l1, _, _) in paths)
            out.append((f"l{t}.mlp.0", (self.n_basis, self.hidden), self.n_basis))
            out.append((f"l{t}.mlp.1", (self.hidden, self.hidden), self.hidden))
            out.append((f"l{t}.mlp.2", (self.hidden, P), self.hidden))
            for l in self._out_ls(t):
                mid = sum(self.muls[l1] for (l1, _, l3) in paths if l3 == l)
                out.append((f"l{t}.lin2.{l}", (mid, self._gate_mul(t, l)), mid))
        out.append(("readout.0", (C0, C0 // 2), C0))
        out.append(("readout.1", (C0 // 2, 1), C0 // 2))
        return out

    def config(self) -> dict:
        d = dataclasses.asdict(self)
        d["muls"] = list(self.muls)
        d["species"] = list(self.species)
        d["shift"] = list(self.shift) if self.shift else [0.0] * len(self.species)
        return d


def make_weights(spec: ModelSpec, seed: int) -> dict:
    """Draw every tensor from N(0, 1/fan_in) with PCG64(seed), in order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = {}
    for name, shape, fan_in in spec.tensor_shapes():
        w[name] = rng.standard_normal(shape) / math.sqrt(fan_in)
    return w


def write_weights(path: str, spec: ModelSpec, weights: dict) -> None:
    tensors = []
    off = 0
    blobs = []
    for name, shape, _ in spec.tensor_shapes():
        a = np.ascontiguousarray(weights[name], dtype="<f8")
        assert tuple(a.shape) == tuple(shape), (name, a.shape, shape)
        tensors.append({"name": name, "shape": list(shape), "offset": off})
        blobs.append(a.tobytes())
        off += a.nbytes
    header = json.dumps({"format": "snw1", "config": spec.config(),
                         "tensors": tensors}).encode("utf-8")
    pre = len(MAGIC) + 8 + len(header)
    pad = (-pre) % 64
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<Q", len(header) + pad))
        f.write(header)
        f.write(b" " * pad)
        for b in blobs:
            f.write(b)


def read_weights_header(path: str) -> dict:
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError("not an SNW1 file")
        (n,) = struct.unpack("<Q", f.read(8))
        return json.loads(f.read(n).decode("utf-8").rstrip())


def _number_density_kavg(n_atoms: int, volume: float, r_cut: float) -> float:
    # expected neighbour count of a uniform gas of the same number density
    return n_atoms / volume * 4.0 / 3.0 * math.pi * r_cut ** 3


# Per-atom energy scales, chosen so that the RMS force on each model's seed
# structure is about 1 eV/A (measured with the FP64 reference evaluation).
SIGMA_SMALL = 12.87
SIGMA_REAL = 20.41

# SiO2 at 2.2 g/cm^3 has 0.06615 atoms per cubic angstrom.
_SIO2_NUMBER_DENSITY = 192 / 14.264434 ** 3
# alpha-quartz, 2.65 g/cm^3
_QUARTZ_NUMBER_DENSITY = _SIO2_NUMBER_DENSITY * 2.65 / 2.2


def model_spec_small(species=(8, 14)) -> ModelSpec:
    """3 layers, 32x0e+32x1e, l_max 1, 8 Bessel functions, r_c 4 A."""
    return ModelSpec(n_layers=3, muls=(32, 32), l_sh=1, r_cut=4.0, species=tuple(species),
                     k_avg=_number_density_kavg(192, 192 / _SIO2_NUMBER_DENSITY, 4.0),
                     sigma=SIGMA_SMALL)


def model_spec_real(species=(8, 14)) -> ModelSpec:
    """The general-purpose model's shape: 5 layers, 128x0e+64x1e+32x2e,
    l_max 2, 8 Bessel functions, r_c 5 A."""
    return ModelSpec(n_layers=5, muls=(128, 64, 32), l_sh=2, r_cut=5.0, species=tuple(species),
                     k_avg=_number_density_kavg(192, 192 / _SIO2_NUMBER_DENSITY, 5.0),
                     sigma=SIGMA_REAL)


def model_spec_bench(channels: int, layers: int, species=(8, 14), sigma: float = 1.0) -> ModelSpec:
    """One of the paper's benchmark models (section 4): `layers` interaction blocks,
    `channels` channels at every degree l = 0..3 (l_max 3), 8 Bessel functions, r_c 4 A;
    messages normalised by the neighbour count of SiO2 at the alpha-quartz density."""
    return ModelSpec(n_layers=layers, muls=(channels,) * 4, l_sh=3, r_cut=4.0,
                     species=tuple(species),
                     k_avg=_number_density_kavg(192, 192 / _QUARTZ_NUMBER_DENSITY, 4.0),
                     sigma=sigma)
