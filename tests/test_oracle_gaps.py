"""The oracle's double precision runs satisfy the paper's rounding-error
analysis exactly: the gap recurrences eq:Dr, eq:Ds, eq:Dw, eq:Dz and the
4x4 system eq:system hold with zero residual in rational arithmetic, and every
local rounding error is within its bound eq:errbounds1-4 (classic:
eq:auxrec0 and eq:classic_nomatrix).  A wrongly wired recurrence (a dropped
term, a wrong index or sign) would produce a "local error" far above its
rounding bound."""

import math

import numpy as np
import pytest

from oracle import Float64Ops, classic_bicgstab, pipelined_bicgstab, unit_roundoff
from oracle import gaps
from workloads import convdiff2d_c1, random_dense_system


def _run(precond, n=6, its=16):
    p = convdiff2d_c1(n)
    A = p.scipy_csr()
    dinv = 1.0 / A.diagonal() if precond else None
    res = pipelined_bicgstab(Float64Ops(A, dinv), p.b, tol=0.0, maxit=its, record=True)
    return p, A, dinv, res


@pytest.mark.parametrize("precond", [False, True])
def test_pipelined_gap_recurrences_exact(precond):
    p, A, dinv, res = _run(precond)
    errs = gaps.pipelined_local_errors(A, p.b, res.snapshots)
    resid = gaps.pipelined_gap_residuals(errs)
    assert len(resid) == 16
    for r in resid:
        for k, v in r.items():
            assert v == 0, (k, v)


def test_pipelined_gap_recurrences_dense_unsymmetric():
    p = random_dense_system(7, 11, shift=4.0)
    A = p.scipy_csr()
    res = pipelined_bicgstab(Float64Ops(A), p.b, tol=0.0, maxit=6, record=True)
    resid = gaps.pipelined_gap_residuals(gaps.pipelined_local_errors(A, p.b, res.snapshots))
    assert all(v == 0 for r in resid for v in r.values())


@pytest.mark.parametrize("precond", [False, True])
def test_pipelined_local_error_bounds(precond):
    p, A, dinv, res = _run(precond)
    errs = gaps.pipelined_local_errors(A, p.b, res.snapshots)
    bounds = gaps.pipelined_error_bounds(A, errs, res.snapshots, dinv=dinv,
                                         eps=unit_roundoff())
    for it, bd in enumerate(bounds):
        for k, (nv, bv) in bd.items():
            assert nv <= bv * (1 + 1e-9), (it, k, nv, bv)
    # the errors are genuinely rounding-sized (not all zero): the bound test bites
    assert max(bd["d_x"][0] for bd in bounds) > 0


def test_pipelined_componentwise_first_order_bounds():
    """Componentwise form of the g-, x- and r-bounds (each operation rounds
    once, |delta| <= u |operand|): |dg| <= (|k| + 3|b g'| + 4|b w' l'|) u."""
    p, A, dinv, res = _run(True)
    errs = gaps.pipelined_local_errors(A, p.b, res.snapshots)
    u = unit_roundoff()
    prev = None
    for d, sn in zip(errs, res.snapshots):
        b, wp = abs(sn["beta"]), abs(sn["omega_prev"])
        gp = np.zeros(p.n) if prev is None else prev["g"]
        lp = np.zeros(p.n) if prev is None else prev["l"]
        bound = (np.abs(sn["k"]) + 3 * b * np.abs(gp) + 4 * b * wp * np.abs(lp)) * u
        dg = np.array([float(v) for v in d["d_g"]])
        assert np.all(np.abs(dg) <= bound * (1 + 1e-9))
        a, w = abs(sn["alpha"]), abs(sn["omega"])
        bx = (2 * np.abs(sn["x"]) + 3 * a * np.abs(sn["g"]) + 2 * w * np.abs(sn["u"])) * u
        dx = np.array([float(v) for v in d["d_x"]])
        assert np.all(np.abs(dx) <= bx * (1 + 1e-9))
        br = (np.abs(sn["q"]) + 2 * w * np.abs(sn["y"])) * u
        dr = np.array([float(v) for v in d["d_r"]])
        assert np.all(np.abs(dr) <= br * (1 + 1e-9))
        prev = sn


def test_classic_gap_is_pure_accumulation():
    p = convdiff2d_c1(6)
    A = p.scipy_csr()
    res = classic_bicgstab(Float64Ops(A), p.b, tol=0.0, maxit=14, record=True)
    errs = gaps.classic_local_errors(A, p.b, res.snapshots)
    assert all(d["identity"] == 0 for d in errs)
    u = unit_roundoff()
    mu = int(np.max(np.diff(A.indptr)))
    nA = np.linalg.norm(A.toarray(), 2)
    N = p.n
    for d, sn in zip(errs, res.snapshots):
        a, w = abs(sn["alpha"]), abs(sn["omega"])
        assert gaps.exact_norm(d["d_x"]) <= (2 * np.linalg.norm(sn["x"]) + 3 * a * np.linalg.norm(sn["g"])
                                             + 2 * w * np.linalg.norm(sn["u"])) * u * (1 + 1e-9)
        assert gaps.exact_norm(d["d_r"]) <= (np.linalg.norm(sn["q"]) + 2 * w * np.linalg.norm(sn["y"])) * u * (1 + 1e-9)
        assert gaps.exact_norm(d["d_q"]) <= (np.linalg.norm(sn["r"]) + 2 * a * np.linalg.norm(sn["s"])) * u * (1 + 1e-9)
        assert gaps.exact_norm(d["e_s"]) <= mu * math.sqrt(N) * nA * np.linalg.norm(sn["g"]) * u


def test_wrong_wiring_is_caught():
    """Plant a mistake in a copy of the oracle's output (use l_i instead of
    l_{i-1} in the g-recurrence) and check the bound test rejects it."""
    p, A, dinv, res = _run(False, its=6)
    snaps = [dict(s) for s in res.snapshots]
    for i in range(1, len(snaps)):
        s, prev = snaps[i], snaps[i - 1]
        s["g"] = s["k"] + s["beta"] * (prev["g"] - s["omega_prev"] * s["l"])
    errs = gaps.pipelined_local_errors(A, p.b, snaps)
    bounds = gaps.pipelined_error_bounds(A, errs, snaps)
    assert any(nv > bv for bd in bounds[1:] for (nv, bv) in [bd["d_g"]])


def test_automated_bound_dominates_exact_gap():
    """f^r of Section 3.6 (eq:DDr_bound) is an upper bound of the residual gap
    ||(b - A x_i) - r_i||, here evaluated exactly in rational arithmetic
    (rr_tau = 0 disables the replacements so the gap is never reset)."""
    p = convdiff2d_c1(6)
    A = p.scipy_csr()
    d = 1.0 / A.diagonal()
    res = pipelined_bicgstab(Float64Ops(A, d), p.b, tol=0.0, maxit=20, rr_mode="auto",
                             rr_tau=0.0, record=True)
    assert res.replacements == 0
    errs = gaps.pipelined_local_errors(A, p.b, res.snapshots)
    ratios = [gaps.exact_norm(e["Dr1"]) / f for e, f in zip(errs, res.fr)]
    assert len(ratios) == 20
    assert max(ratios) <= 1.0
    assert min(ratios) > 0.0


def test_automated_bound_after_replacements():
    """With replacements the bound restarts from the recomputation error and
    still dominates the exact gap in every later iteration."""
    p = random_dense_system(9, 3, shift=5.0)
    A = p.scipy_csr()
    res = pipelined_bicgstab(Float64Ops(A), p.b, tol=0.0, maxit=14, rr_mode="auto",
                             rr_tau=1e-3, record=True)
    assert res.replacements >= 1
    errs = gaps.pipelined_local_errors(A, p.b, res.snapshots)
    for e, f, sn in zip(errs, res.fr, res.snapshots):
        if not sn["replaced"]:
            assert gaps.exact_norm(e["Dr1"]) <= f


def test_automated_estimate_is_below_bound():
    """The square-root estimate (mu sqrt(N) -> sqrt(mu), mu~ sqrt(N) -> 1) of
    the same recursion never exceeds the worst-case bound, and without
    replacements (rr_tau = 0) it leaves the iterates untouched."""
    p = convdiff2d_c1(8)
    A = p.scipy_csr()
    d = 1.0 / A.diagonal()
    kw = dict(tol=0.0, maxit=25, rr_mode="auto", rr_tau=0.0)
    wc = pipelined_bicgstab(Float64Ops(A, d), p.b, **kw)
    es = pipelined_bicgstab(Float64Ops(A, d), p.b, rr_estimate=True, **kw)
    assert wc.alpha == es.alpha and wc.omega == es.omega
    ratio = np.array(es.fr) / np.array(wc.fr)
    mu = int(np.max(np.diff(A.indptr)))
    assert np.all(ratio <= 1.0)
    # the start value shrinks by (sqrt(mu) + 1) / (mu sqrt(N) + 1) at most
    assert ratio.min() >= 1.0 / (mu * math.sqrt(p.n))
