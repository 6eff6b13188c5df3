"""Helpers shared by the GPU tests: model files, library contexts, tolerances."""
import os
import sys

import numpy as np

# Tolerances (FP32 form): per-atom energy error relative to the RMS per-atom
# energy, max-abs force error, relative Frobenius virial error.
TOL_E_REL_FP32 = 1e-6
TOL_F_ABS_FP32 = 1e-4
TOL_W_REL_FP32 = 1e-5
# BF16 form: relative RMS force error; relative Frobenius virial error.
TOL_F_RMS_BF16 = 2e-2
TOL_W_REL_BF16 = 2e-2
# FP64 form: both sides compute the same sums in float64.
TOL_E_REL_FP64 = 1e-10
TOL_F_ABS_FP64 = 1e-10


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def write_model(tmpdir, spec, seed):
    from synth import make_weights, write_weights
    w = make_weights(spec, seed)
    path = os.path.join(str(tmpdir), f"model_{seed}_{spec.n_layers}_{len(spec.species)}.snw")
    write_weights(path, spec, w)
    return path, w


def errors(got, ref):
    e_ref = ref["atom_energy"]
    rms = np.sqrt(np.mean(e_ref ** 2))
    de = np.abs(got["atom_energy"] - e_ref).max() / rms
    df = np.abs(got["forces"] - ref["forces"]).max()
    f_rms = np.sqrt(np.mean(ref["forces"] ** 2))
    df_rms = np.sqrt(np.mean((got["forces"] - ref["forces"]) ** 2)) / f_rms
    dw = np.linalg.norm(got["virial"] - ref["virial"]) / max(np.linalg.norm(ref["virial"]), 1e-30)
    return dict(e_rel=de, f_abs=df, f_rms_rel=df_rms, w_rel=dw,
                dE_total=abs(got["energy"] - ref["energy"]))
