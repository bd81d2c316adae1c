"""GPU parity of the termination rule and of the automated bound's inputs.

* Confirm-and-replace: when the recursive residual meets the tolerance but
  the FP64 true residual ||b - A x|| does not, and replacement is enabled,
  both sides perform a replacement (eq:rr) and iterate on; the replaced
  residual is not tested in that iteration, and after three such forced
  replacements the solve ends with TRUE_RES_NOT_MET.  FP32 storage drives
  the branch within a few iterations: its recursive residual reaches 1e-6
  while the true residual is still above it.  Status, iteration count,
  replacement count and x are compared with the oracle's.
* After ``assemble_kappa`` the operator bounds of the automated criterion
  (||A||, ||M^-1||, mu) are those of the assembled operator: the logged
  bound equals that of a solver created directly from the same
  coefficients.
"""

import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel
from oracle.mixed import pipelined_bicgstab_lowprec
from workloads import (convdiff2d_c1, dia5_from_kappa, kappa_field_c5, random_dense_system)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Solver():
    from paper_1809_01948_amd.solver import Solver as S
    return S


_CASES = [
    ("dense8-csr", lambda: random_dense_system(8, 1, shift=6.0), "csr"),
    ("c1-6-csr", lambda: convdiff2d_c1(6), "csr"),
    ("c1-6-stencil", lambda: convdiff2d_c1(6), "stencil"),
    ("c1-8-stencil", lambda: convdiff2d_c1(8), "stencil"),
]


@pytest.mark.parametrize("name,make,form", _CASES, ids=[c[0] for c in _CASES])
def test_forced_replacement_matches_oracle(Solver, name, make, form):
    p = make()
    A = p.scipy_csr()
    tol, maxit, period = 1e-6, 60, 1000        # the period never comes round
    ref = pipelined_bicgstab_lowprec(A, p.b, tol=tol, maxit=maxit, rr_period=period)
    # the case drives the branch: one forced replacement, then convergence
    assert ref.status == 0 and ref.replacements == 1, (ref.status_name, ref.replacements)
    print(f"{name}: oracle forced replacement in iteration {ref.rr_iters}, converged after "
          f"{ref.iterations}", flush=True)
    S = Solver.from_problem(p, form=form, precision="mixed", precond="none")
    x, st = S.solve(dev(p.b), tol=tol, maxit=maxit, rr_period=period)
    assert st["status"] == ref.status
    assert st["iterations"] == ref.iterations
    assert st["replacements"] == ref.replacements
    xh = host(x)
    assert np.max(np.abs(xh - ref.x)) <= 1e-12 * np.max(np.abs(ref.x))
    assert st["rel_res_true"] <= tol
    S.close()


def test_bound_after_kappa_assembly_equals_direct(Solver):
    n = 40
    h = 1.0 / (n + 1)
    kap = kappa_field_c5(n, seed=5, sigma=4.0)
    kap0 = kappa_field_c5(n, seed=7, sigma=4.0)
    b = np.full(n * n, h * h)
    k = 30
    direct = Solver.from_stencil("dia5", (n, n), dia5_from_kappa(kap, h))
    bh1 = torch.zeros(k, dtype=torch.float64, device="cuda")
    x1, st1 = direct.solve(dev(b), tol=0.0, maxit=k, rr_auto=True, bound_history=bh1)
    # created for another field, then reassembled on the device for kap
    other = Solver.from_stencil("dia5", (n, n), dia5_from_kappa(kap0, h))
    other.assemble_kappa(dev(kap), (1.0, 0.0), h)
    bh2 = torch.zeros(k, dtype=torch.float64, device="cuda")
    x2, st2 = other.solve(dev(b), tol=0.0, maxit=k, rr_auto=True, bound_history=bh2)
    assert st1["iterations"] == st2["iterations"] == k
    assert np.all(rel(host(bh2), host(bh1)) <= 1e-12)
    assert np.array_equal(host(x1), host(x2))
    direct.close()
    other.close()
