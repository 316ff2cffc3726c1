"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package produces *data only*: sparse symmetric-definite FEM pencils
(A, B) in CSR form, pole/weight tables for the rational filter, seeded start
blocks and element data for the eigenvalue-gradient path.  It contains none of
the eigensolver's arithmetic (no shifted solves, no Krylov iteration, no
Rayleigh-Ritz), so that both the HIP path and the CPU oracle can consume the
same inputs without sharing any code of the method.

The paper measures on FEM vibration models (a pyramid, a hollow platform and a
fish-like body, Section 3.1) whose meshes are not public; the pencils here stand
in for them: tensor-product Q1 Laplace pencils, Q1 diffusion pencils with
per-element coefficients, and trilinear-hex linear elasticity with consistent
mass.
"""

from .pencils import (  # noqa: F401
    Pencil,
    q1_kron_pencil,
    q1_diffusion_pencil,
    hex_elasticity_pencil,
    hex_element_matrices,
)
from .poles import slrf_poles, quadrature_poles  # noqa: F401
from .blocks import start_block, seeded_rng  # noqa: F401
from .configs import (  # noqa: F401
    config_q1_2d,
    config_q1_3d,
    config_elasticity,
    q1_gamma_nev,
    q1_eigenvalues_1d,
    batched_pencils,
)
