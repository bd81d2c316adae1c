"""Sliced-ELL products with a Jacobi vector read a copy of their input that
the phase kernels (and the replacement) have already multiplied by the
Jacobi vector, instead of gathering dinv_j beside every z_j.  The copy holds
the same products dinv_j * z_j that the gathering form computes, so whole
solves agree bit for bit with the gathering form (selected with
PBCG_PREMULT=0 when the solver is created): periodic and automated
replacement, FP32 storage, the transposed operator, a ragged row count.
"""

import numpy as np
import pytest

from gpu_util import dev, history_buffer, host, solver_env
from workloads import random_banded_c4

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Solver():
    from paper_1809_01948_amd.solver import Solver as S
    return S


_CASES = [
    # name, rows, precision, solve kwargs
    ("fp64-P10", 20000, "fp64", dict(tol=0.0, maxit=40, rr_period=10)),
    ("fp64-auto", 20000, "fp64", dict(tol=1e-12, maxit=300, rr_auto=True)),
    ("mixed-P7", 20000, "mixed", dict(tol=0.0, maxit=30, rr_period=7)),
    ("fp64-transpose", 20000, "fp64", dict(tol=1e-12, maxit=300, transpose=True, rr_period=25)),
    ("fp64-ragged", 20011, "fp64", dict(tol=0.0, maxit=25, rr_period=5)),
    ("mixed-ragged-auto", 20011, "mixed", dict(tol=1e-8, maxit=200, rr_auto=True)),
]


@pytest.mark.parametrize("name,rows,prec,sk", _CASES, ids=[c[0] for c in _CASES])
def test_premultiplied_equals_gathering(Solver, name, rows, prec, sk):
    p = random_banded_c4(rows, band=300)
    out = {}
    for pre in (1, 0):
        with solver_env(PBCG_PREMULT=pre):
            S = Solver.from_problem(p, form="csr", precision=prec, precond="jacobi")
        hist = history_buffer(sk["maxit"])
        x, st = S.solve(dev(p.b), history=hist, **sk)
        vecs = {v: host(S.get_vector(v)) for v in ("r", "w", "z", "v", "t", "g", "s", "l", "k")}
        out[pre] = (host(x), st, host(hist), vecs)
        S.close()
    (xa, sa, ha, va), (xb, sb, hb, vb) = out[1], out[0]
    print(name, sa["status_name"], sa["iterations"], sa["replacements"])
    assert sa["iterations"] == sb["iterations"] and sa["status"] == sb["status"]
    assert sa["replacements"] == sb["replacements"]
    assert sa["iterations"] > 0
    assert np.array_equal(xa, xb)
    assert np.array_equal(ha, hb)
    for v in va:
        assert np.array_equal(va[v], vb[v]), v


def test_premultiplied_kernel_timing(Solver):
    """The timing entry points run the products on the pre-multiplied copy."""
    p = random_banded_c4(20000, band=300)
    S = Solver.from_problem(p, form="csr", precision="fp64", precond="jacobi")
    S.solve(dev(p.b), tol=0.0, maxit=10, rr_period=5)
    for k in ("spmv1", "spmv2", "spmv_bare", "iteration"):
        assert S.time_kernel(k, reps=3) > 0.0
    S.close()


# The sliced-ELL iteration products stage each block's column window of
# their input in LDS (banded matrices: the window of 1024 rows spans the band
# plus the rows); the rows are summed in the same order as the gathering
# kernel, so solves agree bit for bit with PBCG_SELL_LDS=0.  The last case's
# window (the whole 40000-row range) exceeds the LDS of a block, so it takes
# the gathering kernel either way.
_LDS_CASES = _CASES + [
    ("fp64-gather-input", 20000, "fp64", dict(tol=0.0, maxit=30, rr_period=10)),
    ("fp64-wide-window", 40000, "fp64", dict(tol=0.0, maxit=10, rr_period=5)),
]


@pytest.mark.parametrize("name,rows,prec,sk", _LDS_CASES, ids=[c[0] for c in _LDS_CASES])
def test_lds_window_equals_global_gathers(Solver, name, rows, prec, sk):
    band = 40000 if name == "fp64-wide-window" else 300
    p = random_banded_c4(rows, band=band)
    pre = 0 if name == "fp64-gather-input" else 1
    out = {}
    for lds in (1, 0):
        with solver_env(PBCG_SELL_LDS=lds, PBCG_PREMULT=pre):
            S = Solver.from_problem(p, form="csr", precision=prec, precond="jacobi")
        hist = history_buffer(sk["maxit"])
        x, st = S.solve(dev(p.b), history=hist, **sk)
        # (t of the stopping iteration is not compared: its product is skipped
        # once the GLRED 2 final has stopped the solve -- entirely here, by the
        # blocks that start after the final in the fused form)
        vecs = {v: host(S.get_vector(v)) for v in ("r", "w", "z", "v")}
        out[lds] = (host(x), st, host(hist), vecs)
        S.close()
    (xa, sa, ha, va), (xb, sb, hb, vb) = out[1], out[0]
    print(name, sa["status_name"], sa["iterations"], sa["replacements"])
    assert sa["iterations"] == sb["iterations"] and sa["status"] == sb["status"]
    assert sa["iterations"] > 0
    assert np.array_equal(xa, xb)
    assert np.array_equal(ha, hb)
    for v in va:
        assert np.array_equal(va[v], vb[v]), v
