"""The n/v refresh on residual replacement (pbcg_opts.rr_nv, an option
outside the paper) on the GPU against the oracle with the same option.

* Traces (alpha, omega, beta, ||r||) to 1e-10 with replacement every 4
  iterations (every 2 on the 3D operator, whose horizon is short), over the
  iterations in which the oracle against itself with
  correctly rounded dots stays within 1e-12, and x to 1e-12 of its largest
  term; operators: CSR with a Jacobi vector (the products read M^-1 z and
  M^-1 w that the phase kernels write), the 2D stencil (products fused into
  the phase kernels), DIA5 (fused), the 3D stencil (plane-marching product),
  and the single-workgroup solve.
* After a replacement in the last iteration the stored v is A M^-1 of the
  stored (replaced) z; also for the transposed (adjoint) solve, against the
  oracle on A^T.
* FP32 storage: the stored vectors bit for bit after the refresh and a few
  more iterations, and the trace over its horizon (the FP32 oracle with two
  summation orders of the dot products).
* Captured graphs: a handle that solves without the option, then with it,
  then without it again gives the bits of a fresh handle each time (the
  option is part of the graph cache key).
"""

import math

import numpy as np
import pytest

from gpu_util import dev, history_buffer, host, oracle_ops, rel, split_history
from oracle import STATUS, Float64Ops, pipelined_bicgstab
from oracle.mixed import pipelined_bicgstab_lowprec
from workloads import convdiff2d_c1, convdiff3d_c3, inverse_problem_c5, poisson2d_c2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Solver():
    from paper_1809_01948_amd.solver import Solver as S
    return S


class _FsumOps(Float64Ops):
    """The oracle's arithmetic with correctly rounded dot products."""

    def dot(self, v, w):
        return math.fsum(np.asarray(v) * np.asarray(w))


def _horizon(A, b, dinv, kw, cap=24):
    a, f = (pipelined_bicgstab(cls(A, dinv), b, tol=0.0, maxit=cap + 1, **kw)
            for cls in (Float64Ops, _FsumOps))
    n = min(a.iterations, f.iterations)
    d = np.zeros(n)
    for x, y in ((a.alpha, f.alpha), (a.omega, f.omega), (a.rnorm, f.rnorm), (a.beta, f.beta)):
        d = np.maximum(d, rel(x[:n], y[:n]))
    bad = np.nonzero(d > 1e-12)[0]
    return max(2, min(cap, int(bad[0]) if len(bad) else n))


_CASES = [
    ("c1-csr-jacobi", lambda: convdiff2d_c1(32), "csr", "jacobi", False),
    ("c1-stencil-jacobi", lambda: convdiff2d_c1(32), "stencil", "jacobi", False),
    ("dia5-48", lambda: inverse_problem_c5(48, sigma=1.0, with_csr=True), "dia5", "jacobi", False),
    ("3d7-16", lambda: convdiff3d_c3(16, with_csr=True), "stencil", "jacobi", False),
    ("c1-csr-single-kernel", lambda: convdiff2d_c1(32), "csr", "jacobi", True),
]


@pytest.mark.parametrize("name,make,form,pc,single", _CASES, ids=[c[0] for c in _CASES])
def test_nv_refresh_trace(Solver, name, make, form, pc, single):
    p = make()
    A, ops = oracle_ops(p, pc)
    P = 2 if name.startswith("3d") else 4
    kw = dict(rr_period=P, rr_tau=0.0, rr_nv=True)
    k = _horizon(A, p.b, ops.dinv, kw)
    k -= k % P                               # end on a replacement
    assert k >= P
    print(f"{name}: trace horizon {k} iterations", flush=True)
    ref = pipelined_bicgstab(ops, p.b, tol=0.0, maxit=k, record=True, **kw)
    S = Solver.from_problem(p, form=form, precond=pc)
    hist = history_buffer(k)
    x, st = S.solve(dev(p.b), tol=0.0, maxit=k, history=hist, rr_period=P, rr_tau=1e-300,
                    rr_nv=True, single_kernel=single)
    assert st["single_kernel"] == (1 if single else 0)
    assert st["iterations"] == k and st["status"] == STATUS["MAXIT"]
    assert st["replacements"] == ref.replacements == k // P
    assert st["spmvs"] == 3 + 2 * k + 5 * st["replacements"] + 1
    rn, al, om, be = split_history(hist, k)
    assert np.all(rel(al, ref.alpha) <= 1e-10)
    assert np.all(rel(om, ref.omega) <= 1e-10)
    assert np.all(rel(rn, ref.rnorm) <= 1e-10)
    assert np.all(rel(be[:k - 1], ref.beta[:k - 1]) <= 1e-10)

    def amax(v):
        return float(np.max(np.abs(np.asarray(v, dtype=float))))
    term_x = max(max(amax(sn["x1"]), abs(ref.alpha[j]) * amax(sn["g"]),
                     abs(ref.omega[j]) * amax(sn["u"])) for j, sn in enumerate(ref.snapshots))
    assert np.max(np.abs(host(x) - ref.x)) <= 1e-12 * term_x
    # the last iteration replaced z: the stored v is A M^-1 of the stored z
    z = host(S.get_vector("z"))
    v = host(S.get_vector("v"))
    want = A @ (ops.dinv * z)
    assert np.max(np.abs(v - want)) <= 1e-13 * np.max(np.abs(want))
    # and it is the oracle's refreshed v (z agrees to the trace's accuracy)
    rep = ref.snapshots[-1]["rep"]
    assert np.max(np.abs(v - rep["v"])) <= 1e-9 * np.max(np.abs(rep["v"]))
    S.close()


@pytest.mark.parametrize("name,make,form", [
    ("c1-csr-jacobi", lambda: convdiff2d_c1(32), "csr"),
    ("dia5-48", lambda: inverse_problem_c5(48, sigma=1.0, with_csr=True), "dia5")],
    ids=["c1-csr-jacobi", "dia5-48"])
def test_nv_refresh_transposed_trace(Solver, name, make, form):
    """The adjoint solve A^T x = b with the refresh against the oracle on
    A^T (same Jacobi diagonal), replacement every 4 iterations."""
    import scipy.sparse as sp
    p = make()
    A = sp.csr_matrix(p.scipy_csr().T)
    dinv = 1.0 / A.diagonal()
    kw = dict(rr_period=4, rr_tau=0.0, rr_nv=True)
    k = _horizon(A, p.b, dinv, kw)
    k -= k % 4
    assert k >= 4
    print(f"{name} transposed: trace horizon {k} iterations", flush=True)
    ref = pipelined_bicgstab(Float64Ops(A, dinv), p.b, tol=0.0, maxit=k, **kw)
    S = Solver.from_problem(p, form=form, precond="jacobi")
    hist = history_buffer(k)
    x, st = S.solve(dev(p.b), tol=0.0, maxit=k, history=hist, rr_period=4, rr_tau=1e-300,
                    rr_nv=True, transpose=True)
    assert st["iterations"] == k and st["replacements"] == ref.replacements == k // 4
    rn, al, om, be = split_history(hist, k)
    assert np.all(rel(al, ref.alpha) <= 1e-10)
    assert np.all(rel(om, ref.omega) <= 1e-10)
    assert np.all(rel(rn, ref.rnorm) <= 1e-10)
    z = host(S.get_vector("z"))
    v = host(S.get_vector("v"))
    want = A @ (dinv * z)
    assert np.max(np.abs(v - want)) <= 1e-13 * np.max(np.abs(want))
    S.close()


@pytest.mark.parametrize("k", [10, 14])
def test_nv_refresh_fp32_storage_vectors_bitwise(Solver, k):
    """Poisson 64^2, Jacobi, FP32 storage, replacement every 10 with the
    refresh: after the replacement in iteration 9 (k = 10) and four more
    iterations (k = 14) every stored vector, v included, equals the FP32
    oracle's bit for bit."""
    p = poisson2d_c2(64)
    A = p.scipy_csr()
    ref = pipelined_bicgstab_lowprec(A, p.b, jacobi=True, tol=0.0, maxit=k, rr_period=10,
                                     rr_nv=True, record=True)
    sn = ref.snapshots[-1]
    S = Solver.from_problem(p, form="stencil", precision="mixed", precond="jacobi")
    x, st = S.solve(dev(p.b), tol=0.0, maxit=k, rr_period=10, rr_nv=True)
    assert st["replacements"] == ref.replacements == 1
    for name, key in (("z", "z"), ("v", "v"), ("w", "w1"), ("r", "r1"), ("k", "k1"), ("s", "s"),
                      ("l", "l"), ("g", "g")):
        got = host(S.get_vector(name))
        assert np.array_equal(got, sn[key].astype(np.float64)), name
    S.close()


def test_nv_refresh_fp32_storage_trace(Solver):
    """The same solve through two replacements (iterations 9 and 19): the
    scalar trace over the iterations in which the FP32 oracle with BLAS dot
    products and with correctly rounded ones agree to 1e-12 (after the
    second replacement the refreshed trajectory amplifies rounding-order
    differences faster than the plain one)."""
    p = poisson2d_c2(64)
    A = p.scipy_csr()
    its = 22
    kw = dict(jacobi=True, tol=0.0, maxit=its, rr_period=10, rr_nv=True)
    ref = pipelined_bicgstab_lowprec(A, p.b, **kw)
    fs = pipelined_bicgstab_lowprec(A, p.b, dot_order="fsum", **kw)
    d = np.maximum(rel(ref.alpha, fs.alpha), rel(ref.omega, fs.omega))
    bad = np.nonzero(d > 1e-12)[0]
    h = int(bad[0]) if len(bad) else its
    print(f"fp32 refresh trace horizon {h}", flush=True)
    assert h >= 12                            # past the first replacement
    S = Solver.from_problem(p, form="stencil", precision="mixed", precond="jacobi")
    hist = history_buffer(its)
    x, st = S.solve(dev(p.b), tol=0.0, maxit=its, rr_period=10, rr_nv=True, history=hist)
    assert st["replacements"] == ref.replacements == 2
    rn, al, om, be = split_history(hist, its)
    assert np.all(rel(al[:h], ref.alpha[:h]) <= 1e-10)
    assert np.all(rel(om[:h], ref.omega[:h]) <= 1e-10)
    assert np.all(rel(rn[:h], ref.rnorm[:h]) <= 1e-10)
    S.close()


def test_nv_refresh_graph_cache(Solver):
    p = convdiff2d_c1(32)
    b = dev(p.b)
    kw = dict(tol=1e-10, maxit=2000, rr_period=10, use_graph=True)
    S = Solver.from_problem(p, form="csr", precond="jacobi")
    runs = [S.solve(b, **kw), S.solve(b, rr_nv=True, **kw), S.solve(b, **kw)]
    S.close()
    fresh = []
    for nv in (False, True):
        F = Solver.from_problem(p, form="csr", precond="jacobi")
        fresh.append(F.solve(b, rr_nv=nv, **kw))
        F.close()
    for (x, st), (xf, sf) in ((runs[0], fresh[0]), (runs[2], fresh[0]), (runs[1], fresh[1])):
        assert st["status"] == sf["status"] == 0
        for key in ("iterations", "replacements", "spmvs", "rel_res_true"):
            assert st[key] == sf[key], key
        assert np.array_equal(host(x), host(xf))
    # the option took effect: one more product per replacement
    for (x, st), nv in ((runs[0], False), (runs[1], True)):
        assert st["replacements"] > 0
        assert st["spmvs"] == 3 + 2 * st["iterations"] + (5 if nv else 4) * st["replacements"] + 1
    assert not np.array_equal(host(runs[0][0]), host(runs[1][0]))
