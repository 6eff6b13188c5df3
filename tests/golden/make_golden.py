"""Write oracle reference values for the full-size workloads (calls only oracle/ and synth/).

Output: tests/golden/<name>.json with the total energy, the virial, the edge count,
and per-atom energies and forces of a seeded sample of atoms, all from the FP64
oracle (paper eqs 1-2 and the virial), for use by the GPU parity tests at full size.

    python tests/golden/make_golden.py sio2_24k
    python tests/golden/make_golden.py quartz_4608_32x4
    python tests/golden/make_golden.py si3n4_112k     (about 80 minutes on 6 threads, 30 GB)

quartz_4608_32x4 is one of the paper's benchmark models (section 4: 32 channels at every
degree l <= 3, 4 interaction blocks, r_c 4 A) on a 4,608-atom SiO2 box at the alpha-quartz
density (the weak-scaling share per GPU), with a fixed energy scale sigma = 100.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.model import OracleModel, evaluate  # noqa: E402
from synth import (config_structure, make_weights, model_spec_bench, model_spec_real,  # noqa: E402
                   sio2_box, CONFIGS)

SAMPLE = 256
SAMPLE_SEED = 3


# paper benchmark-model workloads: (channels, blocks, Si count, structure seed, weights seed)
BENCH = {"quartz_4608_32x4": (32, 4, 1536, 7, 624)}
BENCH_SIGMA = 100.0


def main(name):
    if name in BENCH:
        ch, blocks, n_si, sseed, wseed = BENCH[name]
        species = (8, 14)
        spec = model_spec_bench(ch, blocks, sigma=BENCH_SIGMA)
        w = make_weights(spec, wseed)
        s = sio2_box(n_si, density=2.65, seed=sseed)
        c = {"weights_seed": wseed, "seed": sseed}
    else:
        c = CONFIGS[name]
        species = (8, 14) if c["kind"] == "sio2" else (7, 14)
        spec = model_spec_real(species)
        w = make_weights(spec, c["weights_seed"])
        s = config_structure(name)
    t0 = time.time()
    r = evaluate(OracleModel(spec.config(), w), s.pos, s.Z, s.cell)
    dt = time.time() - t0
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    idx = np.sort(rng.choice(s.n, size=SAMPLE, replace=False))
    out = {
        "workload": name, "n_atoms": s.n, "species": list(species), "sigma": spec.sigma,
        "weights_seed": c["weights_seed"], "structure_seed": c["seed"],
        "n_edges": int(len(r["graph"][0])),
        "energy": r["energy"], "virial": r["virial"].reshape(-1).tolist(),
        "atom_energy_rms": float(np.sqrt(np.mean(r["atom_energy"] ** 2))),
        "force_rms": float(np.sqrt(np.mean(r["forces"] ** 2))),
        "sample_index": idx.tolist(),
        "sample_atom_energy": r["atom_energy"][idx].tolist(),
        "sample_forces": r["forces"][idx].tolist(),
        "oracle_seconds": dt,
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=0)
    print(f"{name}: E={r['energy']:.10f} edges={out['n_edges']} in {dt:.1f} s")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "sio2_24k")
