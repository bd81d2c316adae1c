"""Reverse-mode rule of the linear solve x = A^-1 b (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper contains no differentiation; this module states the textbook rule
that the differentiable solve is checked against.  For x = A^-1 b and a loss
L(x):

* the adjoint lambda solves A^T lambda = dL/dx;
* dL/db = lambda;
* dL/dA = -lambda x^T, so for a stored entry (i, j) of the sparsity pattern
  dL/da_ij = -lambda_i x_j  (from d(A^-1) = -A^-1 (dA) A^-1).

For the coefficient-field operator -div(kappa grad u) + c.grad u assembled
with face coefficients (the mean of the two node values, the node's own
value on a boundary face), a face f between nodes p and q enters
A(p,p), A(q,q) with +c_f and A(p,q), A(q,p) with -c_f, hence
dL/dc_f = -(lambda_p - lambda_q)(x_p - x_q); a boundary face of p enters
A(p,p) only: dL/dc_f = -lambda_p x_p.  Each interior face passes half of its
gradient to each of its two nodes, a boundary face all of it to its node.

Pins: central finite differences of the dense solve (tests).
"""

from __future__ import annotations

import numpy as np


def dense_solve(A, b):
    """x = A^-1 b by LAPACK LU (numpy.linalg.solve)."""
    import scipy.sparse as sp
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    return np.linalg.solve(Ad, b)


def dense_adjoint_grads(A, b, dLdx):
    """Dense reference: returns (x, lambda, grad_b, grad_val) where grad_val
    follows the CSR pattern of ``A`` (stored order)."""
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    Ad = A.toarray()
    x = np.linalg.solve(Ad, b)
    lam = np.linalg.solve(Ad.T, dLdx)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    grad_val = -lam[rows] * x[A.indices]
    return x, lam, lam.copy(), grad_val


def grad_on_pattern(rowptr, col, lam, x):
    """dL/da_ij = -lambda_i x_j for every stored entry (CSR order)."""
    rows = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    return -lam[rows] * x[np.asarray(col)]


def kappa_gradient(lam, x, shape):
    """dL/dkappa for the face-mean assembly described in the module docstring.

    ``lam`` and ``x`` are flattened in lexicographic order ``p = ix + nx*iy``;
    ``shape`` is (ny, nx).  Returns an array of ``shape``."""
    ny, nx = shape
    L = np.asarray(lam).reshape(ny, nx)
    X = np.asarray(x).reshape(ny, nx)
    g = np.zeros((ny, nx))
    # interior faces in x: between (iy, ix) and (iy, ix+1)
    fx = -(L[:, :-1] - L[:, 1:]) * (X[:, :-1] - X[:, 1:])
    g[:, :-1] += 0.5 * fx
    g[:, 1:] += 0.5 * fx
    # interior faces in y: between (iy, ix) and (iy+1, ix)
    fy = -(L[:-1, :] - L[1:, :]) * (X[:-1, :] - X[1:, :])
    g[:-1, :] += 0.5 * fy
    g[1:, :] += 0.5 * fy
    # boundary faces: west/east columns and south/north rows
    own = -L * X
    g[:, 0] += own[:, 0]
    g[:, -1] += own[:, -1]
    g[0, :] += own[0, :]
    g[-1, :] += own[-1, :]
    return g
