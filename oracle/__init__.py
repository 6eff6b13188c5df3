"""FP64 CPU oracle for the SevenNet/NequIP energy, force and virial evaluation.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
`cpu_baseline` leg of `bench.py` may import this package.  It shares no code
with the GPU library (no kernels, headers, tables or helpers) and imports
nothing from it; the GPU library computes its own Clebsch-Gordan tables by a
different method.

What it computes (paper sections 2-3):
  * E = sum_i E_i (eq 1), F_i = -grad_i E (eq 2);
  * NequIP message passing (eqs 3-4) with real spherical harmonics up to
    l = 2 (l = 3 for the benchmark models of section 4), 8 Bessel radial functions under a p = 6 polynomial envelope, a
    radial MLP, channel-wise Clebsch-Gordan tensor-product convolutions
    normalised by the average neighbour count, linear self-connections in
    place of the species-dependent tensor product, gated nonlinearities, and
    a last block that keeps only scalar-output paths (section 5.1);
  * edge forces (eq 5) and their assembly into atomic forces (eq 6), and the
    virial W = -sum_e d_e (x) dE/dd_e;
  * the ghost-shell evaluation of one subdomain whose ghost features are
    refreshed from their owners before every layer after the first, with
    gradients and partial forces folded back (section 3.1), and a
    multi-subdomain emulation of the same scheme;
  * (oracle/md.py) velocity Verlet and the Nose-Hoover NVT integrator of the
    paper's MD benchmarks (section 4), driven by any force function;
  * (oracle/train.py) the energy term of the training loss (eq 9, Huber on per-atom
    energies) and its gradient with respect to every weight tensor.

Every floating-point quantity is float64.  Derivatives are taken with
torch.autograd on CPU.  Pins (closed forms, invariances, finite differences,
brute force) live in tests/test_oracle_*.py.

Parity status: every function here is pinned by a test except the absolute
values of the model energy for given weights, which no printed example in
the paper fixes ("parity unpinned" for absolute energies; they are pinned
only by self-consistency: invariances, finite differences, special cases).
"""
from .basis import real_sph_harm, bessel_basis, poly_envelope, radial_basis  # noqa: F401
from .cg import real_cg, complex_cg  # noqa: F401
from .graph import periodic_edges, ghost_shell, subdomains  # noqa: F401
from .model import OracleModel, evaluate, evaluate_ghost, evaluate_subdomains  # noqa: F401
