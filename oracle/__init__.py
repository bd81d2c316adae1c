"""CPU oracle for the preconditioned (pipelined) BiCGStab method.

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library imports, links or
calls this package; only the test-suite, the smoke check and the benchmark's
CPU baseline do.  It shares no code with the GPU path.

Contents
--------
``krylov``   classic preconditioned BiCGStab (Algorithm 1) and preconditioned
             pipelined BiCGStab (Algorithm 2) with periodic residual
             replacement (Section 3.6, eq:rr), written step by step in the
             paper's order and notation.  One implementation serves two
             arithmetics: IEEE double (NumPy/SciPy) and exact rationals
             (``fractions.Fraction``) for tiny systems.
``gaps``     exact evaluation of the local rounding errors and the gaps
             between true and recursive quantities of a recorded double
             precision run (Section 3.1-3.2, eq:auxrec, eq:Dr-eq:Dz,
             eq:system), and the local error bounds eq:errbounds1-4.
``adjoint``  the reverse-mode rule of the linear solve (dense reference for
             small systems) and the chain rule from face coefficients to a
             node coefficient field.

Pins (what fixes each function independently of itself) are listed in the
module docstrings and exercised by ``tests/test_oracle_*.py``.
"""

from .krylov import (  # noqa: F401
    STATUS,
    BlockJacobiOps,
    Float64Ops,
    ExactOps,
    SolveResult,
    classic_bicgstab,
    pipelined_bicgstab,
    unit_roundoff,
)
