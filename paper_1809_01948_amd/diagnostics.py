"""Error-propagation diagnostics of a p-BiCGStab run (host-side analysis).

Section 3.3 writes the gaps between true and recursively computed
quantities as local rounding errors multiplied by *error propagation
matrices* built from the iteration's scalars (eq:all_matrices), and points
to the column maximum norms of the products listed in eq:all_error_matrices
as the indicator of lost stability.  This module builds those matrices from
the alpha_i, omega_i, beta_{i+1} a solve records in its history buffer
(``Solver.solve(..., history=...)``) and returns the column maximum norms.

Pure NumPy on the host; dense matrices of order i (a few thousand at most).
"""

from __future__ import annotations

import numpy as np


def propagation_matrices(alpha, omega, beta):
    """The matrices of eq:all_matrices for i iterations.

    alpha[j], omega[j]: the scalars of iteration j = 0..i-1; beta[j]: beta_{j+1},
    formed at the end of iteration j (beta_0 = 0 is not used).  Returns a dict
    of (i x i) arrays A, B, E, P, C, D, O, U (index k of the paper's
    subscripts runs over the columns)."""
    a = np.asarray(alpha, dtype=np.float64)
    w = np.asarray(omega, dtype=np.float64)
    bt = np.asarray(beta, dtype=np.float64)
    i = len(a)
    if len(w) != i or len(bt) < i - 1:
        raise ValueError("alpha, omega need i entries and beta at least i - 1")
    # beta_j for j = 1..i-1 (the paper's B uses beta_1 .. beta_{i-1} for order i)
    b = np.concatenate([[0.0], bt[: i - 1]])          # b[j] = beta_j, b[0] unused
    # products beta_{r+1} ... beta_c for r < c (empty product 1 on the diagonal)
    Bm = np.zeros((i, i))
    for r in range(i):
        Bm[r, r] = 1.0
        p = 1.0
        for c in range(r + 1, i):
            p *= b[c]
            Bm[r, c] = p
    U = np.triu(np.ones((i, i)))
    Am = np.zeros((i, i))
    Cm = np.zeros((i, i))
    Dm = np.zeros((i, i))
    Pm = np.zeros((i, i))
    for r in range(i):
        Am[r, r + 1:] = -a[r]
        Cm[r, r + 1:] = -w[r]
        Dm[r, r + 1:] = w[r] * a[r]
        Pm[r, r + 1:] = -w[r] * Bm[r, r + 1:]
    Em = Bm.copy()
    Em[0, :] = 0.0
    Om = np.zeros((i, i))
    for r in range(1, i):
        Om[r, r] = -w[r - 1]
    return dict(A=Am, B=Bm, E=Em, P=Pm, C=Cm, D=Dm, O=Om, U=U)


PRODUCTS = ("U", "OU", "BA", "UEA", "BAEA", "BPA", "UC", "BAC", "BD")


def column_max_norms(alpha, omega, beta):
    """Column maximum norms of the nine products of eq:all_error_matrices,
    each an array of length i.  Column k of a product holds the factors that
    multiply the local rounding errors of iterations 0..k in the gap of
    iteration k (eq:matrix_expr), so its maximum modulus is the largest
    amplification any earlier local error has reached by then."""
    M = propagation_matrices(alpha, omega, beta)
    A, B, E, P, C, D, O, U = (M[k] for k in "ABEPCDOU")
    prods = {
        "U": U,
        "OU": O @ U,
        "BA": B @ A,
        "UEA": U @ E @ A,
        "BAEA": B @ A @ E @ A,
        "BPA": B @ P @ A,
        "UC": U @ C,
        "BAC": B @ A @ C,
        "BD": B @ D,
    }
    return {k: np.max(np.abs(v), axis=0) for k, v in prods.items()}


def from_history(hist, iterations):
    """(alpha, omega, beta) from a solve's history buffer (rows ||r_{i+1}||,
    alpha_i, omega_i, beta_{i+1}) for its first `iterations` rows."""
    h = np.asarray(hist, dtype=np.float64).reshape(-1, 4)[:iterations]
    return h[:, 1], h[:, 2], h[:, 3]
