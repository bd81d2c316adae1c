"""GPU parity of the FP32-storage path against the low-precision oracle
(oracle.mixed: the same lines, the same FP32 roundings, FP64 dots, x,
scalars and replacement).

The FP32 vectors of the two sides are identical as long as the FP64
scalars round to the same FP32 values: the dot products differ only in
their summation order (~1e-16 relative), which the rounding of alpha, beta,
omega to FP32 absorbs, so the trajectories stay together far longer than
in FP64 (where every last-bit difference is propagated).  The FP64 x is
updated with the FP64 scalars and carries those last-bit differences.
"""

import numpy as np
import pytest
import torch

from gpu_util import dev, history_buffer, host, rel, split_history
from oracle.mixed import pipelined_bicgstab_lowprec
from workloads import convdiff2d_c1, convdiff3d_c3, inverse_problem_c5, poisson2d_c2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Solver():
    from paper_1809_01948_amd.solver import Solver as S
    return S


def _cases():
    return [
        ("c1-csr", lambda: convdiff2d_c1(32), "csr", False),
        ("c1-stencil", lambda: convdiff2d_c1(32), "stencil", False),
        ("poisson64-jacobi", lambda: poisson2d_c2(64), "stencil", True),
        ("c3-24-jacobi", lambda: convdiff3d_c3(24, with_csr=True), "stencil", True),
        ("dia5-48-jacobi", lambda: inverse_problem_c5(48, sigma=1.0, with_csr=True), "dia5", True),
    ]


_CASES = _cases()


@pytest.mark.parametrize("name,make,form,jacobi", _CASES, ids=[c[0] for c in _CASES])
def test_mixed_trace(Solver, name, make, form, jacobi):
    p = make()
    A = p.scipy_csr()
    its = 40
    ref = pipelined_bicgstab_lowprec(A, p.b, jacobi=jacobi, tol=0.0, maxit=its)
    S = Solver.from_problem(p, form=form, precision="mixed",
                            precond="jacobi" if jacobi else "none")
    hist = history_buffer(its)
    x, st = S.solve(dev(p.b), tol=0.0, maxit=its, history=hist)
    assert st["iterations"] == its == ref.iterations
    rn, al, om, be = split_history(hist, its)
    assert np.all(rel(al, ref.alpha) <= 1e-12)
    assert np.all(rel(om, ref.omega) <= 1e-12)
    assert np.all(rel(rn, ref.rnorm) <= 1e-12)
    assert np.linalg.norm(host(x) - ref.x) <= 1e-12 * np.linalg.norm(ref.x)
    S.close()


@pytest.mark.parametrize("k", [1, 6])
def test_mixed_vectors_bitwise(Solver, k):
    """The stored FP32 vectors after k iterations equal the oracle's bit for
    bit (read back widened to FP64)."""
    p = poisson2d_c2(64)
    A = p.scipy_csr()
    ref = pipelined_bicgstab_lowprec(A, p.b, jacobi=True, tol=0.0, maxit=k, record=True)
    sn = ref.snapshots[-1]
    S = Solver.from_problem(p, form="stencil", precision="mixed", precond="jacobi")
    x, st = S.solve(dev(p.b), tol=0.0, maxit=k)
    for name, want in {"r": sn["r1"], "k": sn["k1"], "w": sn["w1"], "g": sn["g"], "s": sn["s"],
                       "l": sn["l"], "z": sn["z"], "v": sn["v"]}.items():
        got = host(S.get_vector(name))
        assert np.array_equal(got, want.astype(np.float64)), name
    S.close()


def test_mixed_periodic_replacement_trace(Solver):
    """Through replacements (FP64 sums, rounded to FP32): 100 iterations
    with replacement every 25, and convergence of the full solve."""
    p = convdiff2d_c1(32)
    A = p.scipy_csr()
    its = 100
    ref = pipelined_bicgstab_lowprec(A, p.b, tol=0.0, maxit=its, rr_period=25)
    S = Solver.from_problem(p, form="csr", precision="mixed", precond="none")
    hist = history_buffer(its)
    x, st = S.solve(dev(p.b), tol=0.0, maxit=its, rr_period=25, history=hist)
    assert st["replacements"] == ref.replacements == 4
    rn, al, om, be = split_history(hist, its)
    assert np.all(rel(al, ref.alpha) <= 1e-10)
    assert np.all(rel(om, ref.omega) <= 1e-10)
    ref2 = pipelined_bicgstab_lowprec(A, p.b, tol=1e-10, maxit=3000, rr_period=25)
    x2, st2 = S.solve(dev(p.b), tol=1e-10, maxit=3000, rr_period=25)
    assert st2["status"] == 0 == ref2.status
    assert abs(st2["iterations"] - ref2.iterations) <= max(3, 0.2 * ref2.iterations)
    assert np.linalg.norm(p.b - A @ host(x2)) <= 1e-10 * np.linalg.norm(p.b) * 1.01
    S.close()


def test_mixed_automated_bound_trace(Solver):
    """The automated bound with FP32 recurrences (square-root estimate,
    epsilon 2^-24, restart with 2^-53, tau 2^-12) logged per iteration
    equals the oracle's."""
    p = poisson2d_c2(64)
    A = p.scipy_csr()
    k = 20
    ref = pipelined_bicgstab_lowprec(A, p.b, jacobi=True, tol=0.0, maxit=k, rr_mode="auto")
    S = Solver.from_problem(p, form="stencil", precision="mixed", precond="jacobi")
    bh = torch.zeros(k, dtype=torch.float64, device="cuda")
    x, st = S.solve(dev(p.b), tol=0.0, maxit=k, rr_auto=True, bound_history=bh)
    assert st["replacements"] == ref.replacements
    assert np.all(rel(host(bh), np.array(ref.fr)) <= 1e-9)
    S.close()
