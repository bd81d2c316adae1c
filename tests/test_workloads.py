"""The seeded generators produce the shapes and structure the workloads
state (grid sizes, nnz, symmetry, dominance, FP32-exact values)."""

import numpy as np
import pytest
import scipy.sparse as sp

from workloads import (Stencil, convdiff2d_c1, convdiff3d_c3, dia5_from_kappa,
                       dia5_to_csr, inverse_problem_c5, kappa_field_c5,
                       poisson2d_c2, random_banded_c4, stencil_to_csr,
                       tp2_unsymmetric)


def test_c1_shape_and_exact_solution():
    p = convdiff2d_c1(32)
    assert p.n == 1024 and p.nnz == 4992
    A = p.scipy_csr()
    assert abs(A - A.T).max() > 0          # unsymmetric
    np.testing.assert_allclose(A @ p.x_exact, p.b, rtol=0, atol=1e-15)
    assert np.all(np.diff(p.col[p.rowptr[5]:p.rowptr[6]]) > 0)


def test_c2_shape():
    p = poisson2d_c2(1000)
    assert p.n == 1_000_000 and p.nnz == 4_996_000
    assert p.b.min() >= -1 and p.b.max() <= 1
    assert np.array_equal(p.b, np.random.default_rng(2).uniform(-1, 1, p.n))


def test_c3_stencil_small():
    p = convdiff3d_c3(10, with_csr=True)
    assert p.nnz == 7 * 1000 - 6 * 100
    co = p.stencil.coef
    assert (co["C"], co["E"], co["W"], co["N"], co["S"], co["U"], co["D"]) == (6, 4, -6, 1.5, -3.5, -0.5, -1.5)
    for v in co.values():
        assert float(np.float32(v)) == v
    A = p.scipy_csr()
    np.testing.assert_allclose(A @ p.x_exact, p.b, rtol=0, atol=1e-15)
    assert convdiff3d_c3(200).n == 8_000_000


def test_c4_structure_small():
    p = random_banded_c4(N=20000, nnz_row=27, band=500, seed=4)
    assert p.nnz == 27 * 20000
    A = p.scipy_csr()
    rows = np.repeat(np.arange(p.n), 27)
    assert np.all(np.abs(p.col - rows) <= 500)
    c = p.col.reshape(p.n, 27)
    assert np.all(np.diff(c, axis=1) > 0)               # distinct, sorted
    assert np.all(np.float32(p.val).astype(np.float64) == p.val)
    d = A.diagonal()
    off = np.asarray(abs(A).sum(axis=1)).ravel() - np.abs(d)
    np.testing.assert_allclose(d, 1.2 * off, rtol=1e-6)
    np.testing.assert_allclose(A @ p.x_exact, p.b)


def test_c5_dia5_matches_csr_and_faces():
    n = 16
    h = 1.0 / (n + 1)
    kap = kappa_field_c5(n, seed=5, sigma=3.0)
    assert kap.shape == (n, n) and np.all(kap > 0)
    dia = dia5_from_kappa(kap, h)
    rp, col, val = dia5_to_csr((n, n), dia)
    A = sp.csr_matrix((val, col, rp), shape=(n * n, n * n))
    assert A.nnz == 5 * n * n - 4 * n
    # symmetric part of the diffusion: A + A^T has zero skew apart from convection
    S = (A - A.T).toarray()
    assert np.allclose(np.abs(S[S != 0]), h)
    # row sums equal the boundary-face coefficients (interior rows sum to 0)
    rs = np.asarray(A.sum(axis=1)).ravel().reshape(n, n)
    assert np.allclose(rs[1:-1, 1:-1], 0.0, atol=1e-13)
    # so do the interior column sums (the convection terms cancel pairwise):
    # with the constant b the shadow residual r_0 = b gives
    # (r_0, r_i) = h^2 (1^T b - c^T x_i), c = A^T 1 nonzero on the boundary only
    cs = np.asarray(A.sum(axis=0)).ravel().reshape(n, n)
    assert np.allclose(cs[1:-1, 1:-1], 0.0, atol=1e-13)
    assert np.all(np.abs(cs[0, :]) > 1e-3)
    p = inverse_problem_c5(64)
    assert p.dia5.shape == (5, 64 * 64) and np.allclose(p.b, p.extra["h"] ** 2)


def test_stencil_csr_roundtrip_3d_ordering():
    st = Stencil("3d7", (3, 4, 5), {k: float(i + 1) for i, k in enumerate("DSWCENU")})
    rp, col, val = stencil_to_csr(st)
    A = sp.csr_matrix((val, col, rp))
    # interior point (1, 1, 1): p = 1 + 3*1 + 12*1 = 16
    row = A.getrow(16)
    assert list(row.indices) == [4, 13, 15, 16, 17, 19, 28]
    assert list(row.data) == [1, 2, 3, 4, 5, 6, 7]


def test_tp2_normalised():
    p = tp2_unsymmetric(30)
    A = p.scipy_csr()
    s = np.linalg.norm(A.toarray(), 2)
    assert abs(s - 1.0) < 1e-3          # power-iteration estimate of ||A||_2
