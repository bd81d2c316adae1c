"""Local rounding errors and true-vs-recursive gaps, evaluated exactly (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Given the per-iteration snapshots of a double precision run of
``oracle.krylov`` (``record=True``), every stored double is converted to an
exact rational and the quantities of the analysis are evaluated without any
rounding:

* the local rounding errors of the recurrences, defined as in eq:auxrec
  (pipelined) and eq:auxrec0 (classic): the stored result minus the exact
  value of the bracketed formula applied to the stored inputs, e.g.
  delta^g_i = g_i - (k_i + beta_i (g_{i-1} - omega_{i-1} l_{i-1}));
* the errors of the explicitly computed products of eq:auxvars2 (and
  eq:auxvars01): e^t_i = t_i - A m_i, e^v_i = v_i - A n_i
  (e^s = s - A g, e^y = y - A u for the classic method);
* the gaps eq:res_gap and eq:DsDwDz: Delta^r_i = (b - A x_i) - r_i,
  Delta^s_i = A g_i - s_i, Delta^w_i = A k_i - w_i, Delta^z_i = A l_i - z_i.

With these, the gap recurrences eq:Dr, eq:Ds, eq:Dw, eq:Dz and the 4x4
system eq:system / eq:local hold *exactly*, once the explicit SPMV errors are
kept as separate terms (the paper folds them into the local error bounds;
see ``pipelined_gap_residuals``).  The norms of the local errors obey the
bounds eq:errbounds1-4 with epsilon the unit roundoff (see
``pipelined_error_bounds``).
"""

from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def to_exact(a):
    """Exact rational copy of a float64 vector."""
    return np.array([Fraction(float(x)) for x in np.asarray(a, dtype=np.float64)],
                    dtype=object)


class ExactMatrix:
    """A sparse matrix with exact rational entries (rows of (col, value))."""

    def __init__(self, A):
        import scipy.sparse as sp
        A = sp.csr_matrix(A)
        self.n = A.shape[0]
        self.rows = []
        for i in range(self.n):
            lo, hi = A.indptr[i], A.indptr[i + 1]
            self.rows.append([(int(A.indices[j]), Fraction(float(A.data[j])))
                              for j in range(lo, hi)])

    def __matmul__(self, v):
        out = np.empty(self.n, dtype=object)
        for i, row in enumerate(self.rows):
            acc = Fraction(0)
            for j, a in row:
                acc += a * v[j]
            out[i] = acc
        return out


def exact_norm(v) -> float:
    """2-norm of an exact vector, rounded to float at the very end."""
    acc = Fraction(0)
    for a in v:
        acc += a * a
    return math.sqrt(float(acc))


def _F(s):
    return Fraction(float(s))


def _zeros(n):
    return np.array([Fraction(0)] * n, dtype=object)


# -----------------------------------------------------------------------------
# pipelined BiCGStab (Algorithm 2)
# -----------------------------------------------------------------------------

def pipelined_local_errors(A, b, snaps):
    """Exact local errors and gaps of each recorded iteration of Algorithm 2.

    Returns one dict per snapshot with exact vectors
    d_g, d_s, d_l, d_z, d_q, d_u, d_y, d_x, d_r, d_k, d_w (eq:auxrec),
    e_t = t_i - A m_i, e_v = v_i - A n_i (eq:auxvars2),
    Dr, Dw (at i, inputs), Ds, Dz (at i, after the i-th updates),
    Dr1, Dw1 (at i+1, before any replacement of that iteration), and the
    exact scalars alpha, beta, omega, omega_prev.
    """
    Ax = ExactMatrix(A)
    n = Ax.n
    bx = to_exact(b)
    out = []
    prev = None
    for sn in snaps:
        E = {k: to_exact(sn[k]) for k in ("x", "r", "k", "w", "m", "t", "g", "s", "l", "z",
                                          "q", "u", "y", "n", "v", "x1", "r1", "k1", "w1")}
        al, be, om, omp = _F(sn["alpha"]), _F(sn["beta"]), _F(sn["omega"]), _F(sn["omega_prev"])
        if prev is None:
            gp = sp_ = lp = zp = np_ = vp = _zeros(n)
        else:
            gp, sp_, lp, zp, np_, vp = (prev[k] for k in ("g", "s", "l", "z", "n", "v"))
        d = {}
        d["d_g"] = E["g"] - (E["k"] + be * (gp - omp * lp))
        d["d_s"] = E["s"] - (E["w"] + be * (sp_ - omp * zp))
        d["d_l"] = E["l"] - (E["m"] + be * (lp - omp * np_))
        d["d_z"] = E["z"] - (E["t"] + be * (zp - omp * vp))
        d["d_q"] = E["q"] - (E["r"] - al * E["s"])
        d["d_u"] = E["u"] - (E["k"] - al * E["l"])
        d["d_y"] = E["y"] - (E["w"] - al * E["z"])
        d["d_x"] = E["x1"] - ((E["x"] + al * E["g"]) + om * E["u"])
        d["d_r"] = E["r1"] - (E["q"] - om * E["y"])
        d["d_k"] = E["k1"] - (E["u"] - om * (E["m"] - al * E["n"]))
        d["d_w"] = E["w1"] - (E["y"] - om * (E["t"] - al * E["v"]))
        d["e_t"] = E["t"] - (Ax @ E["m"])
        d["e_v"] = E["v"] - (Ax @ E["n"])
        d["Dr"] = (bx - Ax @ E["x"]) - E["r"]
        d["Dw"] = (Ax @ E["k"]) - E["w"]
        d["Ds"] = (Ax @ E["g"]) - E["s"]
        d["Dz"] = (Ax @ E["l"]) - E["z"]
        d["Dr1"] = (bx - Ax @ E["x1"]) - E["r1"]
        d["Dw1"] = (Ax @ E["k1"]) - E["w1"]
        d.update(alpha=al, beta=be, omega=om, omega_prev=omp, replaced=sn["replaced"], i=sn["i"])
        d["_ev_prev"] = None if prev is None else prev["_d"]["e_v"]
        d["_Ds_prev"] = _zeros(n) if prev is None else prev["_d"]["Ds"]
        d["_Dz_prev"] = _zeros(n) if prev is None else prev["_d"]["Dz"]
        d["_Ax"] = Ax
        out.append(d)
        E["_d"] = d
        prev = E
    return out


def pipelined_gap_residuals(errs):
    """For each iteration, the exact residual of the gap recurrences.

    Returned per iteration (as max-abs Fractions, all must be 0):

    * ``Dr``: eq:Dr,
      Dr_{i+1} = Dr_i - a Ds_i - w Dw_i + w a Dz_i - A dx - dr - w A du - dq + w dy.
    * ``Ds``: eq:Ds,
      Ds_i = Dw_i + b Ds_{i-1} - b w_{i-1} Dz_{i-1} + A dg - ds.
    * ``Dw``: eq:Dw with the explicit SPMV errors kept,
      Dw_{i+1} = Dw_i - a Dz_i + A dk - dw + A du - dy + w e^t_i - w a e^v_i.
    * ``Dz``: eq:Dz with the explicit SPMV errors kept,
      Dz_i = b Dz_{i-1} + A dl - dz - e^t_i + b w_{i-1} e^v_{i-1}.
    * ``system``: eq:system with eq:local (the e^t, e^v terms added to the
      local contributions in the same way).

    Iterations with a replacement are skipped for the (i+1)-quantities.
    """
    res = []
    for d in errs:
        Ax = d["_Ax"]
        a, bb, w, wp = d["alpha"], d["beta"], d["omega"], d["omega_prev"]
        n = len(d["Dr"])
        evp = d["_ev_prev"] if d["_ev_prev"] is not None else _zeros(n)
        Dsp, Dzp = d["_Ds_prev"], d["_Dz_prev"]
        r = {}
        lhs = d["Ds"]
        rhs = d["Dw"] + bb * Dsp - bb * wp * Dzp + (Ax @ d["d_g"]) - d["d_s"]
        r["Ds"] = max(abs(v) for v in (lhs - rhs))
        eps_z = (Ax @ d["d_l"]) - d["d_z"] - d["e_t"] + bb * wp * evp
        lhs = d["Dz"]
        rhs = bb * Dzp + eps_z
        r["Dz"] = max(abs(v) for v in (lhs - rhs))
        if not d["replaced"]:
            lhs = d["Dr1"]
            rhs = (d["Dr"] - a * d["Ds"] - w * d["Dw"] + w * a * d["Dz"] - (Ax @ d["d_x"])
                   - d["d_r"] - w * (Ax @ d["d_u"]) - d["d_q"] + w * d["d_y"])
            r["Dr"] = max(abs(v) for v in (lhs - rhs))
            lhs = d["Dw1"]
            rhs = (d["Dw"] - a * d["Dz"] + (Ax @ d["d_k"]) - d["d_w"] + (Ax @ d["d_u"])
                   - d["d_y"] + w * d["e_t"] - w * a * d["e_v"])
            r["Dw"] = max(abs(v) for v in (lhs - rhs))
            # eq:system: [Dr1, Ds, Dw1, Dz] = Mat [Dr, Ds_prev, Dw, Dz_prev] + eps
            eps_s = (Ax @ d["d_g"]) - d["d_s"]
            eps_w = (-a * eps_z + (Ax @ d["d_k"]) - d["d_y"] - d["d_w"] + (Ax @ d["d_u"])
                     + w * d["e_t"] - w * a * d["e_v"])
            eps_r = (-(Ax @ d["d_x"]) - w * (Ax @ d["d_u"]) + w * d["d_y"] - d["d_r"]
                     - d["d_q"] - a * eps_s + w * a * eps_z)
            row1 = d["Dr"] - a * bb * Dsp - (a + w) * d["Dw"] + a * bb * (w + wp) * Dzp + eps_r
            row2 = bb * Dsp + d["Dw"] - bb * wp * Dzp + eps_s
            row3 = d["Dw"] - a * bb * Dzp + eps_w
            row4 = bb * Dzp + eps_z
            r["system"] = max(max(abs(v) for v in (d["Dr1"] - row1)),
                              max(abs(v) for v in (d["Ds"] - row2)),
                              max(abs(v) for v in (d["Dw1"] - row3)),
                              max(abs(v) for v in (d["Dz"] - row4)))
        res.append(r)
    return res


def pipelined_error_bounds(A, errs, snaps, dinv=None, eps=2.0 ** -53):
    """Norms of the local errors and the bounds eq:errbounds1-4.

    mu is the maximum number of nonzeros per row of A, mu~ that of M^-1
    (1 for the identity or a Jacobi diagonal), ||A|| and ||M^-1|| are
    2-norms.  Returns a list (per iteration) of dicts name -> (norm, bound).
    The SPMV bound of Section 2, ||e^t|| <= mu sqrt(N) ||A|| ||m|| eps, is
    included as ``e_t`` and ``e_v``.
    """
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    N = A.shape[0]
    mu = int(np.max(np.diff(A.indptr)))
    mut = 1
    nA = float(np.linalg.norm(A.toarray(), 2))
    nM = 1.0 if dinv is None else float(np.max(np.abs(dinv)))
    smu, smut = mu * math.sqrt(N), mut * math.sqrt(N)
    nrm = np.linalg.norm
    out = []
    prev = None
    for d, sn in zip(errs, snaps):
        a, b, w, wp = abs(sn["alpha"]), abs(sn["beta"]), abs(sn["omega"]), abs(sn["omega_prev"])
        if prev is None:
            gp = sp_ = lp = zp = np_ = vp = np.zeros(N)
        else:
            gp, sp_, lp, zp, np_, vp = (prev[k] for k in ("g", "s", "l", "z", "n", "v"))
        k, wv, m, t, r = sn["k"], sn["w"], sn["m"], sn["t"], sn["r"]
        g, s, l, z, q, u, y, nn, v, x = (sn[c] for c in ("g", "s", "l", "z", "q", "u", "y",
                                                         "n", "v", "x"))
        B = {}
        B["d_g"] = nrm(k) + 3 * b * nrm(gp) + 4 * b * wp * nrm(lp)
        B["d_x"] = 2 * nrm(x) + 3 * a * nrm(g) + 2 * w * nrm(u)
        B["d_s"] = nrm(wv) + 3 * b * nrm(sp_) + 4 * b * wp * nrm(zp)
        B["d_r"] = nrm(q) + 2 * w * nrm(y)
        B["d_l"] = (nrm(m) + smut * nM * nrm(wv) + 3 * b * nrm(lp) + 4 * b * wp * nrm(np_)
                    + smut * nM * b * wp * nrm(zp))
        B["d_z"] = (nrm(t) + smu * nA * nrm(m) + smut * nA * nM * nrm(wv) + 3 * b * nrm(zp)
                    + 4 * b * wp * nrm(vp) + smu * nA * b * wp * nrm(np_)
                    + smut * nA * nM * b * wp * nrm(zp))
        B["d_k"] = (nrm(u) + 3 * w * nrm(m) + smut * nM * w * nrm(wv) + 4 * w * a * nrm(nn)
                    + smut * nM * w * a * nrm(z))
        B["d_w"] = (nrm(y) + 3 * w * nrm(t) + smu * nA * w * nrm(m) + smut * nA * nM * w * nrm(wv)
                    + 4 * w * a * nrm(v) + smu * nA * w * a * nrm(nn)
                    + smut * nA * nM * w * a * nrm(z))
        B["d_q"] = nrm(r) + 2 * a * nrm(s)
        B["d_u"] = nrm(k) + 2 * a * nrm(l)
        B["d_y"] = nrm(wv) + 2 * a * nrm(z)
        B["e_t"] = smu * nA * nrm(m)
        B["e_v"] = smu * nA * nrm(nn)
        out.append({key: (exact_norm(d[key]), bound * eps) for key, bound in B.items()})
        prev = sn
    return out


# -----------------------------------------------------------------------------
# classic BiCGStab (Algorithm 1)
# -----------------------------------------------------------------------------

def classic_local_errors(A, b, snaps, dinv=None):
    """Exact local errors of eq:auxrec0 and the classic gap identity.

    Per iteration: d_x, d_r, d_q, e_s = s - A g, e_y = y - A u, Dr (at i),
    Dr1 (at i+1) and ``identity`` = max-abs of
    Dr1 - (Dr + a e_s + w e_y - A dx - dr - dq), which must be exactly 0
    (eq:classic_nomatrix with the explicit SPMV errors kept: the classic gap
    is a plain accumulation of local errors, no amplification)."""
    Ax = ExactMatrix(A)
    bx = to_exact(b)
    out = []
    for sn in snaps:
        E = {k: to_exact(sn[k]) for k in ("x", "r", "g", "s", "q", "u", "y", "x1", "r1")}
        a, w = _F(sn["alpha"]), _F(sn["omega"])
        d = {}
        d["d_x"] = E["x1"] - ((E["x"] + a * E["g"]) + w * E["u"])
        d["d_r"] = E["r1"] - (E["q"] - w * E["y"])
        d["d_q"] = E["q"] - (E["r"] - a * E["s"])
        d["e_s"] = E["s"] - Ax @ E["g"]
        d["e_y"] = E["y"] - Ax @ E["u"]
        d["Dr"] = (bx - Ax @ E["x"]) - E["r"]
        d["Dr1"] = (bx - Ax @ E["x1"]) - E["r1"]
        rhs = d["Dr"] + a * d["e_s"] + w * d["e_y"] - (Ax @ d["d_x"]) - d["d_r"] - d["d_q"]
        d["identity"] = max(abs(v) for v in (d["Dr1"] - rhs))
        out.append(d)
    return out
