"""MI355X-native pipelined BiCGStab (gfx950 HIP kernels behind a C ABI).

The library (libpbicgstab.so, built by ``paper_1809_01948_amd.build``) is
loaded on first use; there is no CPU fallback.
"""

from ._lib import LIB_PATH, STATUS_NAMES, PbcgError, load  # noqa: F401


def __getattr__(name):
    if name in ("Solver", "SparseSolve", "KappaSolve"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
