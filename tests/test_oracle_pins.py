"""Pins of the CPU oracle against facts fixed outside the oracle itself.

* a hand-derived 2x2 iteration (tests/golden/bicgstab_2x2_worked.txt);
* SciPy's textbook BiCGStab (same operation order as Algorithm 1 with right
  preconditioning) iterate by iterate;
* exact-rational equality of Algorithm 1, Algorithm 2 and Algorithm 2 with
  residual replacement (identical iterates in exact arithmetic; eq:rr only
  re-evaluates quantities that the recurrences already equal exactly);
* finite termination in exact arithmetic and the dense LU solution;
* closed-form special cases (Jacobi on a diagonal matrix, b = 0,
  skew-symmetric breakdown, non-finite input).
"""

import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import (STATUS, ExactOps, Float64Ops, classic_bicgstab,
                    pipelined_bicgstab, unit_roundoff)
from workloads import (Stencil, convdiff2d_c1, inverse_problem_c5, random_dense_system,
                       stencil_to_csr)


def _load_golden(path):
    vals = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split("=")
        vals[k.strip()] = [Fraction(t.strip()) for t in v.split(",")]
    return vals


A22 = sp.csr_matrix(np.array([[2.0, 1.0], [1.0, 3.0]]))
B22 = np.array([1.0, 0.0])


@pytest.mark.parametrize("method", ["classic", "pipelined"])
def test_worked_2x2_exact(golden_dir, method):
    g = _load_golden(f"{golden_dir}/bicgstab_2x2_worked.txt")
    ops = ExactOps(A22)
    fn = classic_bicgstab if method == "classic" else pipelined_bicgstab
    res = fn(ops, B22, tol=0.0, maxit=5, record=True)
    assert res.status == STATUS["CONVERGED"]
    assert res.iterations == 2
    assert res.alpha[0] == g["alpha0"][0]
    assert res.omega[0] == g["omega0"][0]
    assert res.beta[0] == g["beta1"][0]
    assert res.alpha[1] == g["alpha1"][0]
    assert res.omega[1] == 0
    assert list(res.snapshots[0]["x1"]) == g["x1"]
    assert list(res.snapshots[0]["r1"]) == g["r1"]
    assert list(res.x) == g["x2"]


def test_worked_2x2_float64(golden_dir):
    g = _load_golden(f"{golden_dir}/bicgstab_2x2_worked.txt")
    for fn in (classic_bicgstab, pipelined_bicgstab):
        res = fn(Float64Ops(A22), B22, tol=1e-15, maxit=10)
        assert res.status == STATUS["CONVERGED"]
        assert abs(res.alpha[0] - 0.5) <= 1e-16
        assert abs(res.omega[0] - 0.3) <= 1e-16
        np.testing.assert_allclose(res.x, [float(v) for v in g["x2"]], rtol=0, atol=1e-15)


@pytest.mark.parametrize("jacobi", [False, True])
def test_classic_matches_scipy_bicgstab(jacobi):
    """SciPy's bicgstab (van der Vorst's BiCGStab, right-preconditioned) and
    Algorithm 1 share the operation order, so the early iterates agree."""
    p = convdiff2d_c1(32)
    A = p.scipy_csr()
    dinv = 1.0 / A.diagonal() if jacobi else None
    kw = {}
    if jacobi:
        kw["M"] = spla.LinearOperator(A.shape, matvec=lambda v: dinv * v)
    xs = []
    spla.bicgstab(A, p.b, rtol=1e-30, atol=0.0, maxiter=12,
                  callback=lambda xk: xs.append(xk.copy()), **kw)
    res = classic_bicgstab(Float64Ops(A, dinv), p.b, tol=0.0, maxit=12, record=True)
    for i in range(10):
        xi = res.snapshots[i]["x1"]
        assert np.linalg.norm(xi - xs[i]) <= 1e-13 * np.linalg.norm(xs[i]), i


def _exact_case(name):
    if name == "dense6":
        p = random_dense_system(6, 7, shift=6.0, integer=True)
        A = p.scipy_csr()
        return A, p.b, 1.0 / A.diagonal(), p.x_exact
    st = Stencil("2d5", (4, 4), {"C": 4.0, "E": -2.0, "W": -1.0, "N": -1.0, "S": 0.5})
    rowptr, col, val = stencil_to_csr(st)
    A = sp.csr_matrix((val, col, rowptr))
    xex = np.arange(16.0)
    return A, A @ xex, None, xex


@pytest.mark.parametrize("case", ["dense6", "stencil4x4"])
def test_exact_classic_equals_pipelined(case):
    A, b, dinv, xex = _exact_case(case)
    its = 6 if case == "dense6" else 5
    ops = ExactOps(A, dinv)
    rc = classic_bicgstab(ops, b, tol=0.0, maxit=its, record=True)
    rp = pipelined_bicgstab(ops, b, tol=0.0, maxit=its, record=True)
    assert rc.iterations == rp.iterations
    assert rc.alpha == rp.alpha
    assert rc.omega == rp.omega
    assert rc.beta == rp.beta
    for sc, sp_ in zip(rc.snapshots, rp.snapshots):
        assert list(sc["x1"]) == list(sp_["x1"])
        assert list(sc["r1"]) == list(sp_["r1"])
    # residual replacement is a no-op on exact iterates (eq:rr recomputes
    # quantities the recurrences already equal exactly)
    rr = pipelined_bicgstab(ops, b, tol=0.0, maxit=its, rr_period=2, rr_tau=0.0)
    assert rr.replacements >= 2
    assert list(rr.x) == list(rp.x)
    assert rr.alpha == rp.alpha and rr.omega == rp.omega


@pytest.mark.parametrize("case", ["dense6", "stencil4x4"])
def test_exact_replacement_with_nv_refresh_is_a_no_op(case):
    """Option outside the paper (rr_nv): a replacement that also recomputes
    n_i = M^-1 z_i and v_i = A n_i from the replaced z_i leaves exact iterates
    unchanged, as eq:rr's six quantities alone do (on exact iterates every
    recomputed quantity equals its recurrence); a refresh from a wrong
    vector (z without M^-1, or the previous iteration's z) would not."""
    A, b, dinv, xex = _exact_case(case)
    its = 6 if case == "dense6" else 5
    ops = ExactOps(A, dinv)
    rp = pipelined_bicgstab(ops, b, tol=0.0, maxit=its)
    rr = pipelined_bicgstab(ops, b, tol=0.0, maxit=its, rr_period=2, rr_tau=0.0, rr_nv=True)
    assert rr.replacements >= 2
    assert list(rr.x) == list(rp.x)
    assert rr.alpha == rp.alpha and rr.omega == rp.omega and rr.beta == rp.beta


def test_nv_refresh_values():
    """With rr_nv the n and v that the next iteration uses are M^-1 and
    A M^-1 of the replaced z (FP64, the oracle's own PREC and SPMV)."""
    p = convdiff2d_c1(10)
    A = p.scipy_csr()
    dinv = 1.0 / A.diagonal()
    ops = Float64Ops(A, dinv)
    res = pipelined_bicgstab(ops, p.b, tol=0.0, maxit=12, rr_period=4, rr_tau=0.0,
                             rr_nv=True, record=True)
    reps = [sn["rep"] for sn in res.snapshots if sn["replaced"]]
    assert len(reps) == 3
    for rep in reps:
        assert np.array_equal(rep["n"], dinv * rep["z"])
        assert np.array_equal(rep["v"], A @ rep["n"])
    # without the option n, v stay those of the recursive z of the iteration
    lit = pipelined_bicgstab(ops, p.b, tol=0.0, maxit=12, rr_period=4, rr_tau=0.0,
                             record=True)
    for sn in lit.snapshots:
        if sn["replaced"]:
            assert np.array_equal(sn["rep"]["n"], sn["n"])
            assert np.array_equal(sn["rep"]["v"], sn["v"])
            assert not np.array_equal(sn["rep"]["z"], sn["z"])


def test_nv_refresh_on_the_coefficient_field_problem():
    """Observation (FP64 oracle, an option outside the paper): on the 384^2
    coefficient-field operator with Jacobi and replacement every 50
    iterations, refreshing n and v at each replacement converges to 1e-6 in
    under 1000 iterations.  With the six quantities of eq:rr alone the same
    solve is at the mercy of rounding here (v_i = A M^-1 z_i of the
    recursive z_i enters the next z recurrence beside the replaced z_i, an
    error of |beta omega| ||A M^-1 (z_replaced - z_i)|| injected at every
    replacement): it stalls at 3e-3 after 1200 iterations with one BLAS
    summation order and converges with another; at 512^2 it diverges, and on
    the GPU at 2048^2 it breaks down at every period."""
    p = inverse_problem_c5(384, with_csr=True)
    A = p.scipy_csr()
    ops = Float64Ops(A, 1.0 / A.diagonal())
    nv = pipelined_bicgstab(ops, p.b, tol=1e-6, maxit=1200, rr_period=50, rr_nv=True)
    assert nv.status == STATUS["CONVERGED"] and nv.iterations < 1000
    assert np.linalg.norm(p.b - A @ nv.x) <= 1e-6 * np.linalg.norm(p.b)


def test_exact_finite_termination():
    A, b, dinv, xex = _exact_case("dense6")
    res = pipelined_bicgstab(ExactOps(A, dinv), b, tol=0.0, maxit=12)
    assert res.status == STATUS["CONVERGED"]
    assert res.iterations <= 6
    assert [float(v) for v in res.x] == list(xex)


@pytest.mark.parametrize("method,rr", [("classic", 0), ("pipelined", 0), ("pipelined", 50)])
def test_dense_lu_agreement(method, rr):
    p = convdiff2d_c1(32)
    A = p.scipy_csr()
    x_lu = np.linalg.solve(A.toarray(), p.b)
    kappa = np.linalg.cond(A.toarray())
    ops = Float64Ops(A)
    if method == "classic":
        res = classic_bicgstab(ops, p.b, tol=1e-10, maxit=2000)
    else:
        res = pipelined_bicgstab(ops, p.b, tol=1e-10, maxit=2000, rr_period=rr)
    assert res.status == STATUS["CONVERGED"]
    assert res.true_rel_res <= 1e-10
    fwd = np.linalg.norm(res.x - x_lu) / np.linalg.norm(x_lu)
    assert fwd <= kappa * 1e-10
    assert np.linalg.norm(x_lu - p.x_exact) <= 1e-12 * np.linalg.norm(p.x_exact)


def test_jacobi_on_diagonal_matrix_one_step():
    """M^-1 A = I: alpha_0 = 1, q_0 = 0, so x_1 = M^-1 b (closed form)."""
    rng = np.random.default_rng(3)
    d = 2.0 ** rng.integers(-3, 4, 50)      # powers of two: 1/d is exact
    A = sp.diags(d).tocsr()
    b = rng.uniform(-1, 1, 50)
    for fn in (classic_bicgstab, pipelined_bicgstab):
        res = fn(ExactOps(A, 1.0 / d), b, tol=0.0, maxit=3)
        assert res.status == STATUS["CONVERGED"] and res.iterations == 1
        assert res.alpha[0] == 1
        assert all(res.x[i] * Fraction(float(d[i])) == Fraction(float(b[i])) for i in range(50))
        resf = fn(Float64Ops(A, 1.0 / d), b, tol=1e-14, maxit=3)
        assert resf.status == STATUS["CONVERGED"]
        np.testing.assert_allclose(resf.x, b / d, rtol=1e-15)


@pytest.mark.parametrize("fn", [classic_bicgstab, pipelined_bicgstab])
def test_zero_rhs(fn):
    p = convdiff2d_c1(8)
    res = fn(Float64Ops(p.scipy_csr()), np.zeros(p.n), tol=1e-10, maxit=10)
    assert res.status == STATUS["CONVERGED"] and res.iterations == 0
    assert not np.any(res.x)


@pytest.mark.parametrize("fn", [classic_bicgstab, pipelined_bicgstab])
def test_skew_symmetric_breakdown(fn):
    """(r0, A r0) = 0 for skew-symmetric A: the first alpha is undefined."""
    rng = np.random.default_rng(5)
    S = rng.integers(-3, 4, size=(8, 8)).astype(float)
    A = sp.csr_matrix(S - S.T)
    b = rng.integers(-3, 4, size=8).astype(float)
    res = fn(ExactOps(A), b, tol=1e-10, maxit=10)
    assert res.status == STATUS["BREAKDOWN_RHO"] and res.iterations == 0
    A2 = sp.csr_matrix(np.array([[0.0, 1.0], [-1.0, 0.0]]))
    res = fn(Float64Ops(A2), np.array([1.0, 1.0]), tol=1e-10, maxit=10)
    assert res.status == STATUS["BREAKDOWN_RHO"] and res.iterations == 0


@pytest.mark.parametrize("fn", [classic_bicgstab, pipelined_bicgstab])
def test_nonfinite(fn):
    p = convdiff2d_c1(8)
    b = p.b.copy()
    b[3] = np.nan
    res = fn(Float64Ops(p.scipy_csr()), b, tol=1e-10, maxit=10)
    assert res.status == STATUS["NONFINITE"]


def test_maxit_and_true_residual_not_met():
    p = convdiff2d_c1(16)
    ops = Float64Ops(p.scipy_csr())
    res = pipelined_bicgstab(ops, p.b, tol=1e-10, maxit=5)
    assert res.status == STATUS["MAXIT"] and res.iterations == 5
    # a tolerance below the attainable accuracy: the recursive residual keeps
    # falling while the true residual stagnates (Section 2.2, Figure captions)
    p = convdiff2d_c1(6)
    ops = Float64Ops(p.scipy_csr())
    res = pipelined_bicgstab(ops, p.b, tol=1e-14, maxit=2000)
    assert res.status == STATUS["TRUE_RES_NOT_MET"]
    assert res.rnorm[-1] <= 1e-14 * res.bnorm
    assert res.true_rel_res > 1e-14


def test_replacement_schedule():
    """Replacements only when (i+1) mod P == 0 and the last reduced
    ||r_i|| >= sqrt(u) ||r_0|| (Section 3.6, periodic setting)."""
    p = convdiff2d_c1(32)
    ops = Float64Ops(p.scipy_csr())
    P = 7
    res = pipelined_bicgstab(ops, p.b, tol=1e-12, maxit=2000, rr_period=P)
    tau = math.sqrt(unit_roundoff())
    rn = [res.rnorm0] + res.rnorm
    periodic = [i for i in res.rr_iters if (i + 1) % P == 0]
    assert periodic, "expected periodic replacements"
    for i in periodic:
        assert rn[i] >= tau * res.rnorm0
    for i in range(len(res.rnorm)):
        if (i + 1) % P == 0 and rn[i] >= tau * res.rnorm0 and i < res.iterations - 1:
            assert i in res.rr_iters


def test_replacement_recomputes_true_quantities():
    """After a replacement (eq:rr) r, k, w come from x_{i+1} and s, l, z from
    g_i; their gaps are then single rounding errors, bounded as in Section 2
    and Section 3.2 (initial-gap bound ((mu sqrt(N)+1)||A|| ||x|| + ||b||) eps,
    SPMV bound mu sqrt(N) ||A|| ||v|| eps)."""
    from oracle.gaps import ExactMatrix, exact_norm, to_exact
    p = convdiff2d_c1(10)
    A = p.scipy_csr()
    dinv = 1.0 / A.diagonal()
    res = pipelined_bicgstab(Float64Ops(A, dinv), p.b, tol=1e-13, maxit=400,
                             rr_period=10, record=True)
    eps = unit_roundoff()
    N = p.n
    mu = int(np.max(np.diff(A.indptr)))
    nA = np.linalg.norm(A.toarray(), 2)
    Ax = ExactMatrix(A)
    D = to_exact(dinv)
    checked = 0
    for sn in res.snapshots:
        if not sn["replaced"]:
            continue
        rep = sn["rep"]
        x1, g = to_exact(sn["x1"]), to_exact(sn["g"])
        r, k, w, s, l, z = (to_exact(rep[c]) for c in "rkwslz")
        gap_r = exact_norm((to_exact(p.b) - Ax @ x1) - r)
        assert gap_r <= ((mu * math.sqrt(N) + 1) * nA * np.linalg.norm(sn["x1"])
                         + np.linalg.norm(p.b)) * eps
        assert exact_norm(k - D * r) <= np.linalg.norm(rep["k"]) * eps
        assert exact_norm(Ax @ k - w) <= mu * math.sqrt(N) * nA * np.linalg.norm(rep["k"]) * eps
        assert exact_norm(Ax @ g - s) <= mu * math.sqrt(N) * nA * np.linalg.norm(sn["g"]) * eps
        assert exact_norm(l - D * s) <= np.linalg.norm(rep["l"]) * eps
        assert exact_norm(Ax @ l - z) <= mu * math.sqrt(N) * nA * np.linalg.norm(rep["l"]) * eps
        checked += 1
    assert checked >= 2
    assert res.status == STATUS["CONVERGED"]


def test_attainable_accuracy_ordering():
    """Section 4 (Figures 1-4): p-BiCGStab attains a markedly worse true
    residual than classic BiCGStab, and periodic residual replacement brings
    it back to the classic level."""
    p = convdiff2d_c1(32)
    A = p.scipy_csr()
    ops = Float64Ops(A)
    nb = np.linalg.norm(p.b)

    def best_true(res):
        return min(np.linalg.norm(p.b - A @ s["x1"]) / nb for s in res.snapshots)

    cl = best_true(classic_bicgstab(ops, p.b, tol=1e-30, maxit=400, record=True))
    pi = best_true(pipelined_bicgstab(ops, p.b, tol=1e-30, maxit=400, record=True))
    rr = best_true(pipelined_bicgstab(ops, p.b, tol=1e-30, maxit=400, rr_period=20,
                                      record=True))
    assert cl < 1e-13
    assert pi > 10 * cl
    assert rr < 3 * cl


def test_automated_replacement_behaviour():
    """Section 4.5: with the automated criterion few replacements are made,
    early in the iteration, and the attainable accuracy is that of classic
    BiCGStab (compare test_attainable_accuracy_ordering)."""
    p = convdiff2d_c1(32)
    A = p.scipy_csr()
    ops = Float64Ops(A)
    nb = np.linalg.norm(p.b)
    cl = classic_bicgstab(ops, p.b, tol=1e-30, maxit=300, record=True)
    au = pipelined_bicgstab(ops, p.b, tol=1e-30, maxit=300, rr_mode="auto", record=True)
    best = lambda r: min(np.linalg.norm(p.b - A @ s["x1"]) / nb for s in r.snapshots)
    assert 1 <= au.replacements <= 10
    assert max(au.rr_iters) < 100
    assert best(au) < 3 * best(cl)
    res = pipelined_bicgstab(ops, p.b, tol=1e-10, maxit=2000, rr_mode="auto")
    assert res.status == STATUS["CONVERGED"] and res.true_rel_res <= 1e-10


def test_automated_replacement_paper_tp2():
    """The unsymmetric model problem of Table tab:specs (TP2), normalised to
    ||A||_2 = 1, b = A 1/sqrt(N): with automated replacement p-BiCGStab
    reaches a 1e-13 relative residual with a few replacements, all early in
    the iteration (Section 4.5 reports ten on this problem at 1000^2; here
    200^2, where the oracle replaces 9 times).  Whether the run still
    reaches 1e-13 after its last replacement is rounding-sensitive: across
    grid sizes 100^2-1000^2 some runs stall or break down instead (the
    design notes list them)."""
    from workloads import tp2_unsymmetric
    p = tp2_unsymmetric(200)
    ops = Float64Ops(p.scipy_csr())
    res = pipelined_bicgstab(ops, p.b, tol=1e-13, maxit=3000, rr_mode="auto")
    assert res.status == STATUS["CONVERGED"] and res.true_rel_res <= 1e-13
    assert 3 <= res.replacements <= 15
    assert max(res.rr_iters[:-1]) < 150


@pytest.mark.parametrize("reading", ["nested", "products"])
@pytest.mark.parametrize("estimate", [False, True], ids=["bound", "estimate"])
def test_automated_replacement_tp2_with_nv_refresh(reading, estimate):
    """TP2 200^2 with the automated criterion in every variant (both
    readings of eq:DDr_bound, worst case and square-root estimate) when each
    replacement also refreshes n and v (rr_nv, an option outside the paper):
    every variant reaches 1e-13 with a handful of replacements, as Section
    4.5 reports (about ten); with the six quantities of eq:rr alone the
    products reading breaks down here (rho' = 0 after ~940 and ~1,560
    iterations, one BLAS thread), and at 1000^2 every variant fails, while
    with the refresh all four converge there too (589-846 iterations, 8-21
    replacements, 4.8e-14-9.7e-14)."""
    from workloads import tp2_unsymmetric
    p = tp2_unsymmetric(200)
    ops = Float64Ops(p.scipy_csr())
    res = pipelined_bicgstab(ops, p.b, tol=1e-13, maxit=3000, rr_mode="auto",
                             rr_estimate=estimate, rr_reading=reading, rr_nv=True)
    assert res.status == STATUS["CONVERGED"] and res.true_rel_res <= 1e-13
    assert 3 <= res.replacements <= 30


_BD_A = np.array([[-2.0, -2.0, -2.0], [-2.0, -2.0, -1.0], [-2.0, 2.0, -1.0]])
_BD_B = np.array([0.0, -1.0, 0.0])


def test_breakdown_and_restart_exact():
    """A 3x3 system on which (r0, r_1) = 0 exactly after the first iteration
    (alpha_0 = -1/2, omega_0 = 1/2: dyadic, so double arithmetic is exact up
    to there).  Without restarts the method stops with BREAKDOWN_RHO; with
    one restart from x_1 it reaches A^-1 b = (3/4, 1/4, -1) two iterations
    later: exactly in rational arithmetic, to rounding in double."""
    A = sp.csr_matrix(_BD_A)
    for ops in (ExactOps(A), Float64Ops(A)):
        r0 = pipelined_bicgstab(ops, _BD_B, tol=0.0, maxit=10)
        assert r0.status == STATUS["BREAKDOWN_RHO"] and r0.iterations == 1
        assert r0.alpha == [-0.5] and r0.omega == [0.5]
        r1 = pipelined_bicgstab(ops, _BD_B, tol=1e-14, maxit=10, restarts=1)
        assert r1.status == STATUS["CONVERGED"] and r1.restarts == 1
        assert r1.iterations == 3
        x = np.array([float(v) for v in r1.x])
        if ops.exact:
            assert list(r1.x) == [Fraction(3, 4), Fraction(1, 4), Fraction(-1)]
        else:
            assert np.allclose(x, [0.75, 0.25, -1.0], rtol=0, atol=1e-14)
    assert np.allclose(np.linalg.solve(_BD_A, _BD_B), [0.75, 0.25, -1.0], rtol=0, atol=1e-15)


# -----------------------------------------------------------------------------
# block-Jacobi preconditioner (oracle.BlockJacobiOps)
# -----------------------------------------------------------------------------

def test_block_jacobi_special_cases():
    """Blocks of one row are the Jacobi preconditioner (bitwise the same
    iterates); one block of N rows is M = A, so A M^-1 = I and the method
    stops after one iteration at rounding level."""
    from oracle import BlockJacobiOps
    p = convdiff2d_c1(16)
    A = p.scipy_csr()
    jac = pipelined_bicgstab(Float64Ops(A, 1.0 / A.diagonal()), p.b, tol=1e-10, maxit=500,
                             rr_period=50)
    b1 = pipelined_bicgstab(BlockJacobiOps(A, 1), p.b, tol=1e-10, maxit=500, rr_period=50)
    assert jac.alpha == b1.alpha and jac.omega == b1.omega
    assert np.array_equal(jac.x, b1.x)
    small = convdiff2d_c1(6)
    As = small.scipy_csr()
    one = pipelined_bicgstab(BlockJacobiOps(As, small.n), small.b, tol=1e-12, maxit=5)
    assert one.status == STATUS["CONVERGED"] and one.iterations == 1
    assert np.allclose(one.x, np.linalg.solve(As.toarray(), small.b), rtol=1e-13, atol=1e-15)


def test_block_jacobi_prec_is_inverse_of_block_diagonal():
    """PREC with ragged blocks (N = 36, blocks of 5) equals the solve with the
    block diagonal of A assembled independently (dense, entries outside the
    blocks zeroed)."""
    from oracle import BlockJacobiOps
    p = convdiff2d_c1(6)
    A = p.scipy_csr().toarray()
    n, bs = p.n, 5
    M = np.zeros_like(A)
    for lo in range(0, n, bs):
        hi = min(n, lo + bs)
        M[lo:hi, lo:hi] = A[lo:hi, lo:hi]
    v = np.random.default_rng(1).standard_normal(n)
    ops = BlockJacobiOps(sp.csr_matrix(A), bs)
    assert np.allclose(ops.prec(v), np.linalg.solve(M, v), rtol=1e-13, atol=1e-14)


def test_block_jacobi_classic_equals_pipelined_early():
    """Algorithms 1 and 2 with the same (block) preconditioner give the same
    iterates in exact arithmetic; in double precision the first iterations
    agree to 1e-10 on the 32^2 convection-diffusion operator with blocks of
    8 rows."""
    from oracle import BlockJacobiOps
    p = convdiff2d_c1(32)
    ops = BlockJacobiOps(p.scipy_csr(), 8)
    cl = classic_bicgstab(ops, p.b, tol=0.0, maxit=10)
    pi = pipelined_bicgstab(ops, p.b, tol=0.0, maxit=10)
    rel = lambda a, b: np.max(np.abs(np.array(a) - np.array(b)) / np.abs(np.array(b)))
    assert rel(pi.alpha, cl.alpha) <= 1e-10 and rel(pi.omega, cl.omega) <= 1e-10
    assert rel(pi.rnorm, cl.rnorm) <= 1e-10


# -----------------------------------------------------------------------------
# a fixed shadow vector in place of r_0 (an option outside the paper)
# -----------------------------------------------------------------------------

@pytest.mark.parametrize("fn", [classic_bicgstab, pipelined_bicgstab])
def test_shadow_vector_r0_is_the_default(fn):
    """Passing r_0 itself as the shadow vector changes nothing, bit for bit."""
    p = convdiff2d_c1(16)
    ops = Float64Ops(p.scipy_csr())
    kw = dict(rr_period=7) if fn is pipelined_bicgstab else {}
    a = fn(ops, p.b, tol=1e-12, maxit=300, record=True, **kw)
    b = fn(ops, p.b, tol=1e-12, maxit=300, record=True, rhat=p.b.copy(), **kw)
    assert a.iterations == b.iterations and a.status == b.status
    assert a.alpha == b.alpha and a.omega == b.omega and a.beta == b.beta
    assert np.array_equal(a.x, b.x)


@pytest.mark.parametrize("case", ["dense6", "stencil4x4"])
def test_exact_classic_equals_pipelined_with_shadow_vector(case):
    """The exact-arithmetic identity of Algorithms 1 and 2 holds for any
    shadow vector (the derivation of Algorithm 2 never uses rhat = r_0), and
    it differs from the run with r_0."""
    A, b, dinv, xex = _exact_case(case)
    its = 5
    rh = np.random.default_rng(3).integers(-4, 5, size=A.shape[0]).astype(float)
    ops = ExactOps(A, dinv)
    rc = classic_bicgstab(ops, b, tol=0.0, maxit=its, record=True, rhat=rh)
    rp = pipelined_bicgstab(ops, b, tol=0.0, maxit=its, record=True, rhat=rh)
    assert rc.iterations == rp.iterations == its
    assert rc.alpha == rp.alpha and rc.omega == rp.omega and rc.beta == rp.beta
    for sc, sp_ in zip(rc.snapshots, rp.snapshots):
        assert list(sc["x1"]) == list(sp_["x1"])
    r0 = pipelined_bicgstab(ops, b, tol=0.0, maxit=its)
    assert r0.alpha != rp.alpha


def test_shadow_vector_avoids_the_exact_breakdown():
    """The 3x3 system whose (r_0, r_1) vanishes exactly: with another shadow
    vector the iteration does not break down and reaches A^-1 b exactly
    (finite termination in rational arithmetic) without a restart.  (Not
    every vector will do: (1, 2, 3) is orthogonal to A r_0 = (2, 2, -2), so
    its first alpha-denominator vanishes.)"""
    A = sp.csr_matrix(_BD_A)
    bad = pipelined_bicgstab(ExactOps(A), _BD_B, tol=0.0, maxit=6,
                             rhat=np.array([1.0, 2.0, 3.0]))
    assert bad.status == STATUS["BREAKDOWN_RHO"] and bad.iterations == 0
    res = pipelined_bicgstab(ExactOps(A), _BD_B, tol=0.0, maxit=6,
                             rhat=np.array([1.0, 1.0, 1.0]))
    assert res.status == STATUS["CONVERGED"] and res.restarts == 0
    assert res.iterations <= 3
    assert list(res.x) == [Fraction(3, 4), Fraction(1, 4), Fraction(-1)]
    resc = classic_bicgstab(ExactOps(A), _BD_B, tol=0.0, maxit=6,
                            rhat=np.array([1.0, 1.0, 1.0]))
    assert list(resc.x) == list(res.x)


def test_mixed_shadow_vector_r0_is_the_default():
    """The FP32-storage oracle: r_0 (as stored) passed as the shadow vector
    is the default, bit for bit."""
    from oracle.mixed import pipelined_bicgstab_lowprec
    p = convdiff2d_c1(16)
    A = p.scipy_csr()
    a = pipelined_bicgstab_lowprec(A, p.b, jacobi=True, tol=1e-6, maxit=200, rr_period=10)
    b = pipelined_bicgstab_lowprec(A, p.b, jacobi=True, tol=1e-6, maxit=200, rr_period=10,
                                   rhat=p.b.astype(np.float32).astype(np.float64))
    assert a.iterations == b.iterations and np.array_equal(a.x, b.x)
