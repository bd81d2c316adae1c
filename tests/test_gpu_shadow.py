"""A caller shadow vector (pbcg_opts.rhat, an option outside the paper) on
the GPU against the oracle with the same vector.

* Scalar traces (alpha, omega, beta, ||r||) to 1e-10 and the vectors
  element-wise to 1e-12, for the CSR, stencil and DIA5 operators, Algorithm
  1 and Algorithm 2 with periodic replacement.  A random shadow vector makes
  (rhat, r_i) a sum with cancellation from the first iteration, so the
  rounding-order drift of the scalars grows faster than with r_0: the trace
  is compared over the iterations in which the oracle against itself with
  correctly rounded dots (``math.fsum``) stays within 1e-12 (``_horizon``,
  between 2 and 8).
* FP32 storage: the stored vectors bit for bit after a few iterations
  (the shadow vector is rounded to FP32 on both sides).
* rhat = r_0 passed explicitly is the default, bit for bit; the shadow
  vector survives a restart (the 3x3 system on which r_0 breaks down
  converges without one when another vector is given).
* The 2048^2 coefficient-field operator with its constant source: the
  interior column sums of the operator vanish, so (r_0, r_i) with r_0 = b
  depends on the boundary values of x_i alone and decays long before r_i;
  Algorithm 1 with r_0 stops with the true residual above the tolerance,
  with a random shadow vector it converges.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp

from gpu_util import dev, history_buffer, host, oracle_ops, rel, split_history
from oracle import STATUS, Float64Ops, classic_bicgstab, pipelined_bicgstab
from oracle.mixed import pipelined_bicgstab_lowprec
from workloads import convdiff2d_c1, inverse_problem_c5, poisson2d_c2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Solver():
    from paper_1809_01948_amd.solver import Solver as S
    return S


def _shadow(n, seed=56):
    return np.random.default_rng(seed).standard_normal(n)


class _FsumOps(Float64Ops):
    """The oracle's arithmetic with correctly rounded dot products."""

    def dot(self, v, w):
        return math.fsum(np.asarray(v) * np.asarray(w))


def _horizon(A, b, dinv, method, rh, kw, cap=8):
    runs = []
    for cls in (Float64Ops, _FsumOps):
        ops = cls(A, dinv)
        if method == "pipelined":
            runs.append(pipelined_bicgstab(ops, b, tol=0.0, maxit=cap + 1, rhat=rh, **kw))
        else:
            runs.append(classic_bicgstab(ops, b, tol=0.0, maxit=cap + 1, rhat=rh))
    a, f = runs
    n = min(a.iterations, f.iterations)
    d = np.zeros(n)
    for x, y in ((a.alpha, f.alpha), (a.omega, f.omega), (a.rnorm, f.rnorm), (a.beta, f.beta)):
        d = np.maximum(d, rel(x[:n], y[:n]))
    bad = np.nonzero(d > 1e-12)[0]
    return max(2, min(cap, int(bad[0]) if len(bad) else n))


_CASES = [
    ("c1-csr", lambda: convdiff2d_c1(32), "csr", "none"),
    ("c1-stencil-jacobi", lambda: convdiff2d_c1(32), "stencil", "jacobi"),
    ("poisson64-stencil", lambda: poisson2d_c2(64), "stencil", "jacobi"),
    ("dia5-48", lambda: inverse_problem_c5(48, sigma=1.0, with_csr=True), "dia5", "jacobi"),
]


@pytest.mark.parametrize("name,make,form,pc", _CASES, ids=[c[0] for c in _CASES])
@pytest.mark.parametrize("method", ["pipelined", "classic"])
def test_shadow_trace_and_vectors(Solver, name, make, form, pc, method):
    p = make()
    A, ops = oracle_ops(p, pc)
    rh = _shadow(p.n)
    k = _horizon(A, p.b, ops.dinv, method, rh, dict(rr_period=4, rr_tau=0.0))
    print(f"{name} {method}: trace horizon {k} iterations", flush=True)
    if method == "pipelined":
        ref = pipelined_bicgstab(ops, p.b, tol=0.0, maxit=k, rr_period=4, rr_tau=0.0,
                                 record=True, rhat=rh)
    else:
        ref = classic_bicgstab(ops, p.b, tol=0.0, maxit=k, record=True, rhat=rh)
    S = Solver.from_problem(p, form=form, precond=pc)
    hist = history_buffer(k)
    kw = dict(rr_period=4, rr_tau=1e-300) if method == "pipelined" else {}
    x, st = S.solve(dev(p.b), tol=0.0, maxit=k, history=hist, method=method, rhat=dev(rh), **kw)
    assert st["iterations"] == k
    rn, al, om, be = split_history(hist, k)
    assert np.all(rel(al, ref.alpha) <= 1e-10)
    assert np.all(rel(om, ref.omega) <= 1e-10)
    assert np.all(rel(rn, ref.rnorm) <= 1e-10)
    assert np.all(rel(be[:k - 1], ref.beta[:k - 1]) <= 1e-10)
    # the vectors are sums of scalar-times-vector terms; the scalars agree to
    # ~1e-12 over the horizon, so each vector to 1e-12 of its largest term
    # (random shadow vectors give large alpha_0 = (rhat, r_0)/(rhat, w_0)):
    # x_{i+1} = x_i + alpha_i g_i + omega_i u_i (g, u preconditioned)
    def amax(v):
        return float(np.max(np.abs(np.asarray(v, dtype=float))))
    term_x, term = 0.0, 0.0
    for j, snap in enumerate(ref.snapshots):
        term_x = max(term_x, amax(snap["x1"]), abs(ref.alpha[j]) * amax(snap["g"]),
                     abs(ref.omega[j]) * amax(snap["u"]))
        sc = [1.0, abs(ref.alpha[j]), abs(ref.omega[j])]
        if method == "pipelined":
            sc += [abs(ref.alpha[j] * ref.omega[j]), abs(snap["beta"]),
                   abs(snap["beta"] * snap["omega_prev"])]
        vmax = max(amax(v) for v in snap.values() if isinstance(v, np.ndarray))
        term = max(term, max(sc) * vmax)
    assert np.max(np.abs(host(x) - ref.x)) <= 1e-12 * term_x
    assert np.array_equal(host(S.get_vector("rhat")), rh)
    if method == "pipelined":
        # a replacement recomputes r = b - A x (and w, s, z from it and g):
        # the difference in x carries over to the replaced vectors times
        # ||A||_inf (times ||A M^-1||_inf for the ones a further product makes)
        sn = ref.snapshots[-1]
        nA = float(np.max(np.asarray(abs(A).sum(axis=1)).ravel()))
        if pc == "jacobi":
            nA *= float(np.max(np.abs(1.0 / A.diagonal())))
        floor = 1e-12 * term * max(nA, 1.0) ** 2
        for vname, want in {"r": sn["r1"], "w": sn["w1"], "s": sn["s"], "z": sn["z"]}.items():
            got = host(S.get_vector(vname))
            assert np.max(np.abs(got - want)) <= floor, vname
    S.close()


@pytest.mark.parametrize("method", ["pipelined", "classic"])
def test_shadow_r0_is_the_default(Solver, method):
    p = convdiff2d_c1(32)
    S = Solver.from_problem(p, form="csr", precond="jacobi")
    kw = dict(rr_period=20) if method == "pipelined" else {}
    x0, st0 = S.solve(dev(p.b), tol=1e-10, maxit=500, method=method, **kw)
    x1, st1 = S.solve(dev(p.b), tol=1e-10, maxit=500, method=method, rhat=dev(p.b), **kw)
    assert st0["iterations"] == st1["iterations"] and st0["status"] == st1["status"] == 0
    assert np.array_equal(host(x0), host(x1))
    S.close()


@pytest.mark.parametrize("k", [1, 6])
def test_shadow_mixed_vectors_bitwise(Solver, k):
    p = poisson2d_c2(64)
    A = p.scipy_csr()
    rh = _shadow(p.n)
    ref = pipelined_bicgstab_lowprec(A, p.b, jacobi=True, tol=0.0, maxit=k, record=True, rhat=rh)
    sn = ref.snapshots[-1]
    S = Solver.from_problem(p, form="stencil", precision="mixed", precond="jacobi")
    x, st = S.solve(dev(p.b), tol=0.0, maxit=k, rhat=dev(rh))
    assert st["iterations"] == k
    assert np.array_equal(host(S.get_vector("rhat")), rh.astype(np.float32).astype(np.float64))
    for name, want in {"r": sn["r1"], "k": sn["k1"], "w": sn["w1"], "g": sn["g"], "s": sn["s"],
                       "l": sn["l"], "z": sn["z"], "v": sn["v"]}.items():
        got = host(S.get_vector(name))
        assert np.array_equal(got, want.astype(np.float64)), name
    S.close()


def test_shadow_avoids_the_exact_breakdown(Solver):
    """The 3x3 system on which (r_0, r_1) = 0 exactly: with the shadow vector
    (1, 1, 1) no breakdown and no restart, A^-1 b = (3/4, 1/4, -1) in 3
    iterations as in the oracle; the vector is kept across a restart that a
    breaking-down vector forces."""
    Abd = np.array([[-2.0, -2.0, -2.0], [-2.0, -2.0, -1.0], [-2.0, 2.0, -1.0]])
    bbd = np.array([0.0, -1.0, 0.0])
    A = sp.csr_matrix(Abd)
    ones = np.ones(3)
    ref = pipelined_bicgstab(Float64Ops(A), bbd, tol=1e-14, maxit=10, rhat=ones)
    S = Solver.from_csr(A.indptr, A.indices, A.data, precond="none")
    x, st = S.solve(dev(bbd), tol=1e-14, maxit=10, rhat=dev(ones))
    assert st["status"] == 0 and st["restarts"] == 0
    assert st["iterations"] == ref.iterations == 3
    assert np.allclose(host(x), [0.75, 0.25, -1.0], rtol=0, atol=1e-14)
    # (1, 2, 3) is orthogonal to A r_0: the first alpha-denominator vanishes,
    # and a restart keeps the same vector, so it breaks down again
    bad = np.array([1.0, 2.0, 3.0])
    refb = pipelined_bicgstab(Float64Ops(A), bbd, tol=1e-14, maxit=10, rhat=bad, restarts=1)
    x, st = S.solve(dev(bbd), tol=1e-14, maxit=10, rhat=dev(bad), restarts=1)
    assert st["status"] == refb.status == STATUS["BREAKDOWN_RHO"]
    assert st["iterations"] == refb.iterations == 0
    S.close()


def test_c5_full_size_shadow_vector(Solver):
    """The 2048^2 coefficient-field operator, b = h^2 1, Jacobi, tolerance
    1e-6: Algorithm 1 with r_0 ends with the true residual above the
    tolerance (its (r_0, r_i) decays with the boundary values of x_i); with a
    random shadow vector it converges."""
    import torch
    p = inverse_problem_c5(2048)
    S = Solver.from_problem(p, form="dia5", precond="jacobi")
    b = torch.from_numpy(p.b).cuda()
    x0, st0 = S.solve(b, tol=1e-6, maxit=20000, method="classic")
    x1, st1 = S.solve(b, tol=1e-6, maxit=20000, method="classic",
                      rhat=torch.from_numpy(_shadow(p.n)).cuda())
    print(f"c5 2048^2 classic: r_0 {st0['status_name']} {st0['iterations']} its "
          f"true {st0['rel_res_true']:.3g}; random shadow {st1['status_name']} "
          f"{st1['iterations']} its true {st1['rel_res_true']:.3g}", flush=True)
    assert st0["status"] != 0
    assert st1["status"] == 0 and st1["rel_res_true"] <= 1e-6
    S.close()
