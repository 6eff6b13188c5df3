"""Write oracle reference values for the full-size workloads (calls only oracle/ and synth/).

Output: tests/golden/<name>.json with the total energy, the virial, the edge count,
and per-atom energies and forces of a seeded sample of atoms, all from the FP64
oracle (paper eqs 1-2 and the virial), for use by the GPU parity tests at full size.

    python tests/golden/make_golden.py sio2_24k
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.model import OracleModel, evaluate  # noqa: E402
from synth import config_structure, make_weights, model_spec_real, CONFIGS  # noqa: E402

SAMPLE = 256
SAMPLE_SEED = 3


def main(name):
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
        "workload": name, "n_atoms": s.n, "species": list(species),
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
