"""The adjoint rule of the oracle against central finite differences."""

import numpy as np
import scipy.sparse as sp

from oracle import Float64Ops, pipelined_bicgstab
from oracle.adjoint import dense_adjoint_grads, grad_on_pattern, kappa_gradient
from workloads import dia5_from_kappa, dia5_to_csr, kappa_field_c5, random_banded_c4


def _loss_dense(Ad, b, c):
    return float(c @ np.linalg.solve(Ad, b))


def test_grad_b_and_values_vs_finite_differences():
    p = random_banded_c4(N=60, nnz_row=7, band=10, seed=3, xseed=4)
    A = p.scipy_csr()
    c = np.random.default_rng(9).standard_normal(p.n)
    x, lam, gb, gv = dense_adjoint_grads(A, p.b, c)
    Ad = A.toarray()
    h = 1e-6
    fd_b = np.array([(_loss_dense(Ad, p.b + h * e, c) - _loss_dense(Ad, p.b - h * e, c)) / (2 * h)
                     for e in np.eye(p.n)])
    assert np.linalg.norm(fd_b - gb) <= 1e-7 * np.linalg.norm(gb)
    rows = np.repeat(np.arange(p.n), np.diff(A.indptr))
    fd_v = np.empty(A.nnz)
    for kk in range(A.nnz):
        Ap = Ad.copy()
        Ap[rows[kk], A.indices[kk]] += h
        Am = Ad.copy()
        Am[rows[kk], A.indices[kk]] -= h
        fd_v[kk] = (_loss_dense(Ap, p.b, c) - _loss_dense(Am, p.b, c)) / (2 * h)
    assert np.linalg.norm(fd_v - gv) <= 1e-6 * np.linalg.norm(gv)
    np.testing.assert_allclose(grad_on_pattern(A.indptr, A.indices, lam, x), gv)


def test_adjoint_by_pipelined_transpose_solve():
    """The adjoint system A^T lambda = c solved by Algorithm 2 on A^T matches
    the dense adjoint."""
    p = random_banded_c4(N=400, nnz_row=9, band=20, seed=5, xseed=6)
    A = p.scipy_csr()
    c = np.random.default_rng(1).standard_normal(p.n)
    _, lam_ref, _, _ = dense_adjoint_grads(A, p.b, c)
    At = A.T.tocsr()
    res = pipelined_bicgstab(Float64Ops(At, 1.0 / At.diagonal()), c, tol=1e-13, maxit=500)
    assert res.status == 0
    assert np.linalg.norm(res.x - lam_ref) <= 1e-11 * np.linalg.norm(lam_ref)


def test_kappa_gradient_vs_finite_differences():
    n = 12
    h = 1.0 / (n + 1)
    kap = kappa_field_c5(n, seed=5, sigma=2.0)
    kap_t = kappa_field_c5(n, seed=55, sigma=2.0)
    b = np.full(n * n, h * h)

    def solve(k):
        rp, col, val = dia5_to_csr((n, n), dia5_from_kappa(k, h))
        Ad = sp.csr_matrix((val, col, rp), shape=(n * n, n * n)).toarray()
        return Ad, np.linalg.solve(Ad, b)

    _, u_t = solve(kap_t)

    def loss(k):
        _, u = solve(k)
        return float(np.sum((u - u_t) ** 2))

    Ad, u = solve(kap)
    lam = np.linalg.solve(Ad.T, 2.0 * (u - u_t))
    g = kappa_gradient(lam, u, (n, n))
    eps = 1e-6
    fd = np.zeros((n, n))
    for iy in range(n):
        for ix in range(n):
            kp = kap.copy()
            kp[iy, ix] += eps
            km = kap.copy()
            km[iy, ix] -= eps
            fd[iy, ix] = (loss(kp) - loss(km)) / (2 * eps)
    assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g)
