"""Seeded synthetic inputs for the pipelined BiCGStab solver and its oracle.

This package only builds problem data (sparse matrices in CSR form, stencil
descriptors, DIA5 coefficient arrays, right-hand sides).  It holds none of the
Krylov method's arithmetic and is the only code that the solver's tests, the
oracle's tests and the benchmark share.
"""

from .generators import (  # noqa: F401
    Problem,
    Stencil,
    convdiff2d_c1,
    poisson2d_c2,
    convdiff3d_c3,
    random_banded_c4,
    kappa_field_c5,
    dia5_from_kappa,
    inverse_problem_c5,
    stencil_to_csr,
    dia5_to_csr,
    tp2_unsymmetric,
    tp3_helmholtz,
    random_dense_system,
)
