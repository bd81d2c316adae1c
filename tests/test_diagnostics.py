"""Error-propagation diagnostics (Section 3.3, eq:all_matrices and
eq:all_error_matrices), against closed forms of the propagation matrices."""

import numpy as np

from paper_1809_01948_amd.diagnostics import column_max_norms, from_history, propagation_matrices


def test_matrices_for_constant_scalars():
    a, w, b, i = 0.7, 0.3, 0.5, 6
    M = propagation_matrices([a] * i, [w] * i, [b] * i)
    for r in range(i):
        for c in range(i):
            if c < r:
                assert M["B"][r, c] == 0 and M["A"][r, c] == 0
            else:
                assert np.isclose(M["B"][r, c], b ** (c - r))
            if c > r:
                assert M["A"][r, c] == -a and M["C"][r, c] == -w
                assert np.isclose(M["D"][r, c], w * a)
                assert np.isclose(M["P"][r, c], -w * b ** (c - r))
    assert np.all(M["E"][0] == 0) and np.allclose(M["E"][1:], M["B"][1:])
    assert np.allclose(np.diag(M["O"]), [0] + [-w] * (i - 1))
    assert np.allclose(M["U"], np.triu(np.ones((i, i))))


def test_column_norms_closed_forms():
    """BA with constant scalars: (BA)[r, c] = -a (1 + b + ... + b^(c-1-r)) for
    r < c, so its column maximum is a (1 - b^c) / (1 - b) (r = 0)."""
    a, w, b, i = 0.7, 0.3, 0.5, 8
    n = column_max_norms([a] * i, [w] * i, [b] * i)
    k = np.arange(i)
    assert np.allclose(n["BA"], a * (1 - b ** k) / (1 - b))
    assert np.allclose(n["U"], 1.0)
    assert np.allclose(n["OU"], np.where(k == 0, 0.0, w))
    # UC[r, c] = -(c - r) w summed over the rows above: column max at r = 0
    assert np.allclose(n["UC"], w * k)
    # beta = 0: B = I, so BD = D and BA = A
    n0 = column_max_norms([a] * i, [w] * i, [0.0] * i)
    assert np.allclose(n0["BA"], np.where(k == 0, 0.0, a))
    assert np.allclose(n0["BD"], np.where(k == 0, 0.0, w * a))


def test_amplification_grows_with_large_beta():
    n = column_max_norms([1.0] * 10, [1.0] * 10, [3.0] * 10)
    assert n["BA"][-1] > 1e3 and np.all(np.diff(n["BA"]) > 0)


def test_from_history_layout():
    rows = np.array([[1.0, 0.5, 0.2, 0.9], [0.8, 0.4, 0.3, 0.7], [0.6, 0.0, 0.0, 0.0]])
    a, w, b = from_history(rows.ravel(), 2)
    assert list(a) == [0.5, 0.4] and list(w) == [0.2, 0.3] and list(b) == [0.9, 0.7]


def test_paper_tp2_amplification_is_large():
    """Section 3.3: on the paper's problems the entries of the propagation
    products reach several orders of magnitude above one (here TP2 on a
    200 x 200 grid, 150 iterations of the FP64 oracle)."""
    from oracle import Float64Ops, pipelined_bicgstab
    from workloads import tp2_unsymmetric
    p = tp2_unsymmetric(200)
    r = pipelined_bicgstab(Float64Ops(p.scipy_csr()), p.b, tol=0.0, maxit=150)
    n = column_max_norms(r.alpha, r.omega, r.beta)
    assert n["U"].max() == 1.0
    assert n["BA"].max() > 1e2 and n["BAEA"].max() > 1e4 and n["BAC"].max() > 1e4
