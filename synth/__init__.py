"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package holds no arithmetic of the model: it only draws random
structures (positions, species, cells) and random model weights, and writes
the weights file.  The paper's own datasets and trained weights are not
available, so every input is synthetic with the shapes, densities and
compositions of the paper's workloads (alpha-quartz/amorphous SiO2 of the
benchmark section, Si3N4 of the large-scale melt-quench section, and a
multi-element stream standing in for the Materials Project structures used
to train the general-purpose model).
"""
from .structures import (  # noqa: F401
    Structure, rsa_box, sio2_box, si3n4_box, serving_stream, config_structure,
    MASSES, CONFIGS,
)
from .weights import (  # noqa: F401
    ModelSpec, make_weights, write_weights, read_weights_header,
    model_spec_small, model_spec_real, model_spec_bench, ACT_SCALE,
)
