"""Sliced-ELL products with a Jacobi vector read a copy of their input that
the phase kernels (and the replacement) have already multiplied by the
Jacobi vector, instead of gathering dinv_j beside every z_j.  The copy holds
the same products dinv_j * z_j that the gathering form computes, so whole
solves agree bit for bit with the gathering form (selected with
PBCG_PREMULT=0 when the solver is created): periodic and automated
replacement, FP32 storage, the transposed operator, a ragged row count.
"""

import numpy as np
import pytest

from gpu_util import dev, history_buffer, host, solver_env
from workloads import random_banded_c4

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Solver():
    from paper_1809_01948_amd.solver import Solver as S
    return S


_CASES = [
    # name, rows, precision, solve kwargs
    ("fp64-P10", 20000, "fp64", dict(tol=0.0, maxit=40, rr_period=10)),
    ("fp64-auto", 20000, "fp64", dict(tol=1e-12, maxit=300, rr_auto=True)),
    ("mixed-P7", 20000, "mixed", dict(tol=0.0, maxit=30, rr_period=7)),
    ("fp64-transpose", 20000, "fp64", dict(tol=1e-12, maxit=300, transpose=True, rr_period=25)),
    ("fp64-ragged", 20011, "fp64", dict(tol=0.0, maxit=25, rr_period=5)),
    ("mixed-ragged-auto", 20011, "mixed", dict(tol=1e-8, maxit=200, rr_auto=True)),
]


@pytest.mark.parametrize("name,rows,prec,sk", _CASES, ids=[c[0] for c in _CASES])
def test_premultiplied_equals_gathering(Solver, name, rows, prec, sk):
    p = random_banded_c4(rows, band=300)
    out = {}
    for pre in (1, 0):
        with solver_env(PBCG_PREMULT=pre):
            S = Solver.from_problem(p, form="csr", precision=prec, precond="jacobi")
        hist = history_buffer(sk["maxit"])
        x, st = S.solve(dev(p.b), history=hist, **sk)
        vecs = {v: host(S.get_vector(v)) for v in ("r", "w", "z", "v", "t", "g", "s", "l", "k")}
        out[pre] = (host(x), st, host(hist), vecs)
        S.close()
    (xa, sa, ha, va), (xb, sb, hb, vb) = out[1], out[0]
    print(name, sa["status_name"], sa["iterations"], sa["replacements"])
    assert sa["iterations"] == sb["iterations"] and sa["status"] == sb["status"]
    assert sa["replacements"] == sb["replacements"]
    assert sa["iterations"] > 0
    assert np.array_equal(xa, xb)
    assert np.array_equal(ha, hb)
    for v in va:
        assert np.array_equal(va[v], vb[v]), v


def test_premultiplied_kernel_timing(Solver):
    """The timing entry points run the products on the pre-multiplied copy."""
    p = random_banded_c4(20000, band=300)
    S = Solver.from_problem(p, form="csr", precision="fp64", precond="jacobi")
    S.solve(dev(p.b), tol=0.0, maxit=10, rr_period=5)
    for k in ("spmv1", "spmv2", "spmv_bare", "iteration"):
        assert S.time_kernel(k, reps=3) > 0.0
    S.close()


# The sliced-ELL iteration products stage each block's column window of
# their input in LDS (banded matrices: the window of 1024 rows spans the band
# plus the rows); the rows are summed in the same order as the gathering
# kernel, so solves agree bit for bit with PBCG_SELL_LDS=0.  The last case's
# window (the whole 40000-row range) exceeds the LDS of a block, so it takes
# the gathering kernel either way.
_LDS_CASES = _CASES + [
    ("fp64-gather-input", 20000, "fp64", dict(tol=0.0, maxit=30, rr_period=10)),
    ("fp64-wide-window", 40000, "fp64", dict(tol=0.0, maxit=10, rr_period=5)),
]


@pytest.mark.parametrize("name,rows,prec,sk", _LDS_CASES, ids=[c[0] for c in _LDS_CASES])
def test_lds_window_equals_global_gathers(Solver, name, rows, prec, sk):
    band = 40000 if name == "fp64-wide-window" else 300
    p = random_banded_c4(rows, band=band)
    pre = 0 if name == "fp64-gather-input" else 1
    out = {}
    for lds in (1, 0):
        with solver_env(PBCG_SELL_LDS=lds, PBCG_PREMULT=pre):
            S = Solver.from_problem(p, form="csr", precision=prec, precond="jacobi")
        hist = history_buffer(sk["maxit"])
        x, st = S.solve(dev(p.b), history=hist, **sk)
        # (t of the stopping iteration is not compared: its product is skipped
        # once the GLRED 2 final has stopped the solve -- entirely here, by the
        # blocks that start after the final in the fused form)
        vecs = {v: host(S.get_vector(v)) for v in ("r", "w", "z", "v")}
        out[lds] = (host(x), st, host(hist), vecs)
        S.close()
    (xa, sa, ha, va), (xb, sb, hb, vb) = out[1], out[0]
    print(name, sa["status_name"], sa["iterations"], sa["replacements"])
    assert sa["iterations"] == sb["iterations"] and sa["status"] == sb["status"]
    assert sa["iterations"] > 0
    assert np.array_equal(xa, xb)
    assert np.array_equal(ha, hb)
    for v in va:
        assert np.array_equal(va[v], vb[v]), v


# Windows of changing shape: the cycle matrix alternates three row-block
# patterns (band below the diagonal, band above it, narrow), so the windows
# a block stages in turn start below, inside and past one another and differ
# in length.  Few blocks (PBCG_LDS_BLOCKS) make every block stage several
# windows; the products are the gathering kernel's bit for bit.

_TILE = 1024


def _cycle_matrix(n, k=8, reach=3000, seed=21):
    """Row i in row block t reads k distinct columns of [i - lo_t, i + hi_t]
    besides its diagonal, (lo_t, hi_t) = (reach, 10), (10, reach), (10, 10)
    for t mod 3 = 0, 1, 2; values standard normal, the diagonal 1.5 times
    the row's absolute sum."""
    import scipy.sparse as sp
    from workloads.generators import Problem
    rng = np.random.default_rng(seed)
    rows = np.arange(n, dtype=np.int64)
    t = rows // _TILE
    lo = np.where(t % 3 == 0, reach, 10)
    hi = np.where(t % 3 == 1, reach, 10)
    a = np.maximum(0, rows - lo)
    b = np.minimum(n - 1, rows + hi)
    W = b - a
    draws = np.sort(rng.integers(0, (W - k + 1)[:, None], size=(n, k)), axis=1)
    c = a[:, None] + draws + np.arange(k)[None, :]
    c = c + (c >= rows[:, None])
    off = rng.standard_normal((n, k))
    diag = 1.5 * np.abs(off).sum(axis=1)
    A = sp.csr_matrix((np.concatenate([off, diag[:, None]], axis=1).ravel(),
                       np.concatenate([c, rows[:, None]], axis=1).ravel(),
                       np.arange(n + 1) * (k + 1)), shape=(n, n))
    A.sort_indices()
    x = np.random.default_rng(seed + 1).uniform(-1, 1, n)
    return Problem(name=f"cycle_{n}", n=n, b=A @ x, x0=np.zeros(n),
                   rowptr=A.indptr.astype(np.int32), col=A.indices.astype(np.int32),
                   val=A.data, x_exact=x, precond="jacobi")


def _windows(A):
    """First column and end of each 1024-row block's window (its columns and
    its rows)."""
    n = A.shape[0]
    out = []
    for t in range((n + _TILE - 1) // _TILE):
        r0, r1 = t * _TILE, min(n, (t + 1) * _TILE)
        cols = A.indices[A.indptr[r0]:A.indptr[r1]]
        out.append((min(r0, int(cols.min())), max(r1 - 1, int(cols.max())) + 1))
    return out


_SHAPE_CASES = [
    # name, precision, blocks, solve kwargs
    ("cycle-fp64-auto", "fp64", 8, dict(tol=1e-12, maxit=200, rr_auto=True)),
    ("cycle-fp64-transpose", "fp64", 8, dict(tol=0.0, maxit=30, rr_period=10, transpose=True)),
    ("cycle-mixed", "mixed", 16, dict(tol=0.0, maxit=30, rr_period=10)),
]


@pytest.mark.parametrize("name,prec,blocks,sk", _SHAPE_CASES, ids=[c[0] for c in _SHAPE_CASES])
def test_lds_windows_of_changing_shape(Solver, name, prec, blocks, sk):
    import scipy.sparse as sp
    p = _cycle_matrix(61_447)
    A = p.scipy_csr()
    w = _windows(A)
    # every window fits a block's LDS (160 KB), so the LDS product runs
    assert max(h - l for l, h in w) * 8 <= 160 * 1024
    # and consecutive windows start below, inside and past one another
    starts = [(w[t + 1][0] < w[t][0], w[t][0] <= w[t + 1][0] < w[t][1], w[t + 1][0] >= w[t][1])
              for t in range(len(w) - 1)]
    assert all(any(s[k] for s in starts) for k in range(3))
    out = {}
    for lds in (1, 0):
        with solver_env(PBCG_LDS_BLOCKS=blocks, PBCG_SELL_LDS=lds):
            S = Solver.from_problem(p, form="csr", precision=prec, precond="jacobi")
        hist = history_buffer(sk["maxit"])
        x, st = S.solve(dev(p.b), history=hist, **sk)
        vecs = {v: host(S.get_vector(v)) for v in ("r", "w", "z", "v")}
        out[lds] = (host(x), st, host(hist), vecs)
        S.close()
    (xa, sa, ha, va), (xb, sb, hb, vb) = out[1], out[0]
    print(name, sa["status_name"], sa["iterations"], sa["replacements"])
    assert sa["iterations"] > 0 and sa["status_name"] in ("CONVERGED", "MAXIT")
    assert sa["iterations"] == sb["iterations"] and sa["status"] == sb["status"]
    assert np.array_equal(xa, xb)
    assert np.array_equal(ha, hb)
    for v in va:
        assert np.array_equal(va[v], vb[v]), v
    P = sk.get("rr_period", 0)
    if prec == "fp64" and sa["status_name"] == "MAXIT" and P and sa["iterations"] % P:
        # the last product: v = A M^-1 z of the stored z
        Ao = sp.csr_matrix(A.T) if sk.get("transpose") else A
        want = Ao @ (va["z"] / A.diagonal())
        assert np.max(np.abs(va["v"] - want)) <= 1e-13 * np.max(np.abs(want))
