"""Pins of the automated-replacement bound f^r (Section 3.6, eq:DDr_bound).

The oracle's running recursion (``oracle.krylov._GapBound``: local bounds
typed in from eq:errbounds1-4, gap norms carried one iteration at a time) is
compared with an evaluation that shares none of its code
(``oracle.gapbound_matrix``): local bounds derived by a generic first-order
rounding model from the expression trees of Algorithm 2's recurrences, and
the propagation through the explicit error propagation matrices of
eq:all_matrices composed as eq:matrix_expr.  The two must agree to rounding
on two operators, with and without replacements; a planted mistake in the
recursion (a dropped term, a wrong coefficient) must break the agreement.
The bound must also dominate the residual gap evaluated exactly in rational
arithmetic, in both readings of Section 3.6.
"""

import numpy as np
import pytest

import oracle.krylov as K
from oracle import Float64Ops, gaps, pipelined_bicgstab
from oracle import gapbound_matrix as GM
from workloads import convdiff2d_c1, tp2_unsymmetric


def _problem(name):
    if name == "c1_6_jacobi":
        p = convdiff2d_c1(6)
        A = p.scipy_csr()
        return p, A, 1.0 / A.diagonal()
    if name == "tp2_50":
        p = tp2_unsymmetric(50)
        return p, p.scipy_csr(), None
    raise ValueError(name)


def _run(name, replacements, maxit=80, reading="nested", estimate=False):
    p, A, dinv = _problem(name)
    ops = Float64Ops(A, dinv)
    # rr_tau = 1e300: the criterion never fires, f^r is still evaluated
    tau = None if replacements else 1e300
    res = pipelined_bicgstab(ops, p.b, tol=1e-300, maxit=maxit, rr_mode="auto", rr_tau=tau,
                             record=True, rr_reading=reading, rr_estimate=estimate)
    nM = ops.norm_bound_M()
    return p, A, ops, res, nM


def _matrix_form(ops, res, n, nM, reading="nested", estimate=False):
    return np.array(GM.bound_history_from_run(res, ops.norm_bound_A(), nM, ops.max_row_nnz(), n,
                                              res.bnorm, reading=reading, estimate=estimate))


@pytest.mark.parametrize("name", ["c1_6_jacobi", "tp2_50"])
@pytest.mark.parametrize("replacements", [False, True])
@pytest.mark.parametrize("reading", ["nested", "products"])
@pytest.mark.parametrize("estimate", [False, True])
def test_recursion_equals_matrix_form(name, replacements, reading, estimate):
    """The running bound of either reading (``_GapBound``: gap norms carried
    one iteration at a time; ``_GapBoundProducts``: the columns of the nine
    products moved one column at a time) equals the explicit matrices, for
    the worst-case bound and its square-root estimate (mu sqrt(N) -> sqrt(mu)
    and mu~ sqrt(N) -> 1, applied by the generic rounding model to its
    operator terms)."""
    p, A, ops, res, nM = _run(name, replacements, reading=reading, estimate=estimate)
    assert res.iterations == 80 and len(res.fr) == 80
    if replacements:
        assert res.replacements >= 1
    else:
        assert res.replacements == 0
    fm = _matrix_form(ops, res, p.n, nM, reading, estimate)
    rel = np.abs(fm - np.array(res.fr)) / np.array(res.fr)
    assert rel.max() <= 1e-12, rel.max()


class _DroppedTerm(K._GapBound):
    """The recursion with the 3 |beta_i| ||z_{i-1}|| term of the delta^z bound
    (eq:errbounds2) left out."""

    def local_bounds(self, a, b, w, wp, nm):
        d = super().local_bounds(a, b, w, wp, nm)
        d["z"] -= 3 * b * self.prev["z"]
        return d


class _WrongCoefficient(K._GapBound):
    """The recursion with 2 ||x_i|| in the delta^x bound (eq:errbounds1)
    written as 1 ||x_i||."""

    def local_bounds(self, a, b, w, wp, nm):
        d = super().local_bounds(a, b, w, wp, nm)
        d["x"] -= nm["x"]
        return d


class _ProductsWrongIndex(K._GapBoundProducts):
    """The products reading with BAC's column c+1 formed from BA's column
    c+1 instead of column c (an index shifted by one: C multiplied after A's
    new column).  (A sign error that flips a whole product cannot show: the
    reading takes its moduli.)"""

    def _step_acd(self, alpha, omega):
        c = self.c
        before = self.M["BA"][:c + 1].copy()
        super()._step_acd(alpha, omega)
        self.M["BAC"][:c + 1] += omega * before - omega * self.M["BA"][:c + 1]


class _ProductsDroppedPath(K._GapBoundProducts):
    """The products reading without the BPA product (the P path of the z
    gap into the s gap)."""

    def _value(self):
        keep = self.M["BPA"].copy()
        self.M["BPA"][:] = 0.0
        f = super()._value()
        self.M["BPA"][:] = keep
        return f


@pytest.mark.parametrize("planted,reading", [(_DroppedTerm, "nested"),
                                             (_WrongCoefficient, "nested"),
                                             (_ProductsWrongIndex, "products"),
                                             (_ProductsDroppedPath, "products")])
def test_planted_mistake_breaks_agreement(monkeypatch, planted, reading):
    name = "_GapBound" if reading == "nested" else "_GapBoundProducts"
    monkeypatch.setattr(K, name, planted)
    p, A, ops, res, nM = _run("tp2_50", False, maxit=60, reading=reading)
    fm = _matrix_form(ops, res, p.n, nM, reading)
    rel = np.abs(fm - np.array(res.fr)) / fm
    assert rel.max() > 1e-6, rel.max()


def test_both_readings_dominate_exact_gap():
    """Section 3.6's bound in both readings is at least the residual gap
    ||(b - A x_i) - r_i|| evaluated exactly; the products reading (moduli of
    the products of eq:all_error_matrices) never exceeds the nested one
    (products of moduli, eq:DDr_bound as printed)."""
    p = convdiff2d_c1(6)
    A = p.scipy_csr()
    d = 1.0 / A.diagonal()
    ops = Float64Ops(A, d)
    res = pipelined_bicgstab(ops, p.b, tol=0.0, maxit=20, rr_mode="auto", rr_tau=1e300,
                             record=True)
    errs = gaps.pipelined_local_errors(A, p.b, res.snapshots)
    exact = np.array([gaps.exact_norm(e["Dr1"]) for e in errs])
    nested = _matrix_form(ops, res, p.n, ops.norm_bound_M(), "nested")
    products = _matrix_form(ops, res, p.n, ops.norm_bound_M(), "products")
    assert np.all(exact <= products) and np.all(products <= nested * (1 + 1e-12))
    assert np.all(exact > 0)


def test_derived_bounds_reproduce_printed_constants():
    """The generic rounding model applied to the trees of Algorithm 2's lines
    gives the printed constants of eq:errbounds1 and eq:errbounds4 (2, 3, 2
    for x; 1, 2 for r, q, u, y) on unit norms and scalars, and the operator
    terms of eq:errbounds2-3 scale with mu sqrt(N) ||A|| and sqrt(N) ||M^-1||."""
    keys = ("x", "g", "u", "q", "y", "r", "s", "k", "l", "w", "z", "m", "t", "n", "v")
    norms = {k: 1.0 for k in keys}
    norms.update({k + "_p": 1.0 for k in ("g", "s", "l", "z", "n", "v")})
    sc = dict(alpha=1.0, beta=1.0, omega=1.0, wp=1.0)
    d = GM.derived_local_bounds(norms, sc, nA=1.0, nM=1.0, mu=1, N=1, eps=1.0)
    assert d["x"] == 7.0 and d["r"] == 3.0 and d["q"] == 3.0 and d["u"] == 3.0 and d["y"] == 3.0
    assert d["g"] == 8.0 and d["s"] == 8.0
    # l: |m| + 3|b l'| + 4|b wp n'| plus the two M^-1 products (sqrt(N) ||M^-1|| each)
    d2 = GM.derived_local_bounds(norms, sc, nA=1.0, nM=3.0, mu=1, N=4, eps=1.0)
    assert d2["l"] == 8.0 + 2 * 2 * 3.0
