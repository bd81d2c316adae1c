"""The residual-gap bound f^r evaluated a second way: error propagation
matrices and a generic first-order rounding analysis (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

``oracle.krylov`` computes the bound f^r of eq:DDr_bound with a running
recursion, one iteration at a time, from local error bounds typed in from
eq:errbounds1-4.  This module evaluates the same quantity without sharing any
of that code, so that a wrong coefficient or a dropped term in either shows
up as a disagreement:

* the local error bounds are *derived*, not typed in: each recurrence of
  eq:auxrec is written down as an expression tree (the algorithm's own
  lines), and the standard first-order rounding model of Section 2 (every
  multiplication and addition contributes the modulus of its exact result
  times epsilon, an explicit product by A or M^-1 contributes
  mu sqrt(N) ||op|| ||input|| epsilon, and every error is carried to the
  result multiplied by the moduli of the scalars and operator norms it
  passes through) is applied to the tree (``derived_local_bounds``);
* the propagation of the local errors into the residual gap follows the
  matrix form of Section 3.3: the error propagation matrices of
  eq:all_matrices are built explicitly from the recorded alpha, beta and
  omega, and the column sums of eq:matrix_expr are formed
  (``bound_from_matrices``).

Two readings of "summing the moduli of the entries in the i-th column"
(Section 3.6) are available:

``nested``    each gap norm ||Delta^s_j||, ||Delta^w_j||, ||Delta^z_j|| is
              bounded first and enters eq:DDr_bound with the moduli of its
              coefficients; in matrix form the moduli of the propagation
              matrices are multiplied (|B||A| instead of |BA|).  This is
              eq:DDr_bound exactly as printed, and it is the reading the
              running recursion evaluates.
``products``  the moduli of the entries of the nine products of
              eq:all_error_matrices, each times the bound of the local error
              group it multiplies.  Never larger than ``nested``.

Initial gaps (Section 3.2): ||Delta^r_0|| <= ((mu sqrt(N) + 1) ||A|| ||x_0||
+ ||b||) eps, ||Delta^w_0|| <= mu sqrt(N) ||A|| ||k_0|| eps,
||Delta^s_0|| <= mu sqrt(N) ||A|| ||g_0|| eps and
||Delta^z_0|| <= mu sqrt(N) ||A|| ||l_0|| eps; they form column 0 of the
Theta matrices of eq:thetas, and iteration 0's s and z (where beta_0 = 0
makes g_0 = k_0, s_0 = w_0, l_0 = m_0, z_0 = t_0) contribute no further
local error.  A replacement (eq:rr) starts a new system whose column 0 holds
the bounds of the recomputation's own rounding.
"""

from __future__ import annotations

import math

import numpy as np


# -----------------------------------------------------------------------------
# expression trees of the recurrences (eq:auxrec) and the first-order model
# -----------------------------------------------------------------------------

class _V:
    """A stored vector (a leaf)."""

    def __init__(self, name):
        self.name = name


class _P:
    """An explicitly computed product ``op @ child``, stored as ``name``;
    ``op`` is "A" (mu nonzeros per row) or "M" (M^-1, mu~ = 1 per row)."""

    def __init__(self, op, name, child):
        self.op, self.name, self.child = op, name, child


class _S:
    """Scalar times a vector expression."""

    def __init__(self, scalar, child):
        self.scalar, self.child = scalar, child


class _Add:
    """Sum or difference of two vector expressions (same rounding model)."""

    def __init__(self, a, b):
        self.a, self.b = a, b


# Algorithm 2's lines as written (eq:auxrec); names ending in "_p" are
# iteration i-1 values, "wp" is omega_{i-1}.
def _prec(src, dst):
    return _P("M", dst, _V(src))


def _spmv_prec(src, mid, dst):
    return _P("A", dst, _P("M", mid, _V(src)))


RECURRENCES = {
    "g": _Add(_V("k"), _S("beta", _Add(_V("g_p"), _S("wp", _V("l_p"))))),
    "s": _Add(_V("w"), _S("beta", _Add(_V("s_p"), _S("wp", _V("z_p"))))),
    "l": _Add(_prec("w", "m"), _S("beta", _Add(_V("l_p"), _S("wp", _prec("z_p", "n_p"))))),
    "z": _Add(_spmv_prec("w", "m", "t"),
              _S("beta", _Add(_V("z_p"), _S("wp", _spmv_prec("z_p", "n_p", "v_p"))))),
    "x": _Add(_Add(_V("x"), _S("alpha", _V("g"))), _S("omega", _V("u"))),
    "r": _Add(_V("q"), _S("omega", _V("y"))),
    "k": _Add(_V("u"), _S("omega", _Add(_prec("w", "m"), _S("alpha", _prec("z", "n"))))),
    "w": _Add(_V("y"), _S("omega", _Add(_spmv_prec("w", "m", "t"),
                                        _S("alpha", _spmv_prec("z", "n", "v"))))),
    "q": _Add(_V("r"), _S("alpha", _V("s"))),
    "u": _Add(_V("k"), _S("alpha", _V("l"))),
    "y": _Add(_V("w"), _S("alpha", _V("z"))),
}


class _Model:
    def __init__(self, norms, scalars, nA, nM, cmu, cmut, eps):
        self.nv, self.sc, self.eps = norms, scalars, eps
        self.opnorm = {"A": nA, "M": nM}
        self.opmu = {"A": cmu, "M": cmut}     # mu sqrt(N) and mu~ sqrt(N) (or estimates)

    def mag(self, e):
        """Upper bound of the norm of the value of expression e."""
        if isinstance(e, (_V, _P)):
            return self.nv[e.name]
        if isinstance(e, _S):
            return abs(self.sc[e.scalar]) * self.mag(e.child)
        return self.mag(e.a) + self.mag(e.b)

    def err(self, e, scale=1.0):
        """First-order bound of the error of e, carried to the result with
        the factor ``scale``."""
        if isinstance(e, _V):
            return 0.0
        if isinstance(e, _P):
            own = self.opmu[e.op] * self.opnorm[e.op] * self.mag(e.child) * self.eps
            return scale * own + self.err(e.child, scale * self.opnorm[e.op])
        if isinstance(e, _S):
            c = abs(self.sc[e.scalar])
            return scale * self.mag(e) * self.eps + self.err(e.child, scale * c)
        return scale * self.mag(e) * self.eps + self.err(e.a, scale) + self.err(e.b, scale)


def derived_local_bounds(norms, scalars, nA, nM, mu, N, eps, estimate=False):
    """Bounds on ||delta^.|| of the eleven recurrences of iteration i, derived
    from their expression trees.  ``norms`` maps vector names (current ones
    and ``*_p`` of iteration i-1) to 2-norms; ``scalars`` holds alpha, beta,
    omega (iteration i) and wp (omega_{i-1})."""
    cmu = math.sqrt(mu) if estimate else mu * math.sqrt(N)
    cmut = 1.0 if estimate else math.sqrt(N)
    m = _Model(norms, scalars, nA, nM, cmu, cmut, eps)
    return {name: m.err(tree) for name, tree in RECURRENCES.items()}


# The local error groups of the four gaps, read off the gap recurrences
# eq:Dr, eq:Ds, eq:Dw and eq:Dz: (delta name, multiplied by A?, scalar).
GROUPS = {
    "R": [("x", True, None), ("r", False, None), ("u", True, "omega"), ("q", False, None),
          ("y", False, "omega")],
    "S": [("g", True, None), ("s", False, None)],
    "W": [("k", True, None), ("w", False, None), ("u", True, None), ("y", False, None)],
    "Z": [("l", True, None), ("z", False, None)],
}


def group_bounds(d, scalars, nA):
    """Bounds of the local error groups of one iteration from the bounds of
    the individual delta's."""
    out = {}
    for key, members in GROUPS.items():
        acc = 0.0
        for name, with_a, sc in members:
            c = nA if with_a else 1.0
            if sc is not None:
                c *= abs(scalars[sc])
            acc += c * d[name]
        out[key] = acc
    return out


# -----------------------------------------------------------------------------
# error propagation matrices (eq:all_matrices) and the column sums
# -----------------------------------------------------------------------------

def propagation_matrices(alpha, beta, omega):
    """The matrices of eq:all_matrices for a segment of n iterations, size
    (n+1) x (n+1).  alpha[j], omega[j] of iteration j (j < n), beta[j] = beta_j
    of iteration j (beta[0] unused)."""
    n = len(alpha)
    size = n + 1
    Am = np.zeros((size, size))
    Bm = np.zeros((size, size))
    Cm = np.zeros((size, size))
    Dm = np.zeros((size, size))
    Em = np.zeros((size, size))
    Pm = np.zeros((size, size))
    Om = np.zeros((size, size))
    Um = np.zeros((size, size))
    for j in range(size):
        for i in range(j, size):
            prod = 1.0
            for k in range(j + 1, i + 1):
                prod *= beta[k] if k < len(beta) else 0.0
            Bm[j, i] = prod
            Um[j, i] = 1.0
            if j >= 1:
                Em[j, i] = prod
            if i > j and j < n:
                Am[j, i] = -alpha[j]
                Cm[j, i] = -omega[j]
                Dm[j, i] = omega[j] * alpha[j]
                Pm[j, i] = -omega[j] * prod
        if 1 <= j <= n:
            Om[j, j] = -omega[j - 1]
    return dict(A=Am, B=Bm, C=Cm, D=Dm, E=Em, P=Pm, O=Om, U=Um)


def bound_from_matrices(theta, mats, reading="nested"):
    """f^r for every column of a segment: ``theta`` maps "R", "S", "W", "Z"
    to the row vectors of local error group bounds (column 0: the initial
    gaps; R and W column j >= 1 from iteration j-1, S and Z column j >= 1
    from iteration j), ``mats`` from ``propagation_matrices``.  R's entries
    must already carry the omega factors of O (eq:matrix_expr's O U)."""
    A, B, C, D, E, P, U = (mats[k] for k in "ABCDEPU")
    tR, tS, tW, tZ = (np.asarray(theta[k], dtype=float) for k in "RSWZ")
    if reading == "nested":
        aA, aB, aC, aD, aE, aP, aU = (np.abs(M) for M in (A, B, C, D, E, P, U))
        Z = tZ @ aB
        W = tW @ aU + Z @ aA
        S = tS @ aB + W @ aE + Z @ aP
        return tR @ aU + S @ aA + W @ aC + Z @ aD
    if reading == "products":
        BA = B @ A
        prods_W = (U @ E @ A, U @ C)
        prods_Z = (BA @ E @ A, B @ P @ A, BA @ C, B @ D)
        f = tR @ np.abs(U) + tS @ np.abs(BA)
        for M in prods_W:
            f = f + tW @ np.abs(M)
        for M in prods_Z:
            f = f + tZ @ np.abs(M)
        return f
    raise ValueError(reading)


def bound_history_from_run(res, nA, nM, mu, N, nb, eps=2.0 ** -53, estimate=False,
                           reading="nested", eps_replace=None):
    """f^r_{i+1} for every iteration of a recorded run of
    ``krylov.pipelined_bicgstab(..., record=True)`` (FP64 arithmetic),
    evaluated with the propagation matrices and derived local bounds.
    Returns a list aligned with ``res.fr``.

    Each replacement (eq:rr, after the w-update of iteration i_r) starts a new
    system.  Its column 0 holds the recomputed s_{i_r}, z_{i_r} gaps, and a
    leading step with alpha = 0 (omega = omega_{i_r}) places the recomputed
    r_{i_r+1}, w_{i_r+1} gaps in column 1 of R and W: from there on the
    layout of eq:matrix_expr holds unchanged."""
    cmu = math.sqrt(mu) if estimate else mu * math.sqrt(N)
    e_r = eps if eps_replace is None else eps_replace
    keys = ("x", "g", "u", "q", "y", "r", "s", "k", "l", "w", "z", "m", "t", "n", "v")

    def nrm(v):
        return float(np.linalg.norm(np.asarray(v, dtype=float)))

    def evaluate(seg):
        n = len(seg["alpha"])
        pad = lambda row: list(row) + [0.0] * (n + 1 - len(row))
        mats = propagation_matrices(seg["alpha"], pad(seg["beta"]), seg["omega"])
        f = bound_from_matrices(dict(R=pad(seg["R"]), S=pad(seg["S"]), W=pad(seg["W"]),
                                     Z=pad(seg["Z"])), mats, reading)
        return float(f[n])

    out = []
    seg = None
    prev = {key: 0.0 for key in ("g", "s", "l", "z", "n", "v")}
    for sn in res.snapshots:
        norms = {key: nrm(sn[key]) for key in keys}
        for key in ("g", "s", "l", "z", "n", "v"):
            norms[key + "_p"] = prev[key]
        scal = {key: float(sn[src]) for key, src in
                (("alpha", "alpha"), ("beta", "beta"), ("omega", "omega"), ("wp", "omega_prev"))}
        grp = group_bounds(derived_local_bounds(norms, scal, nA, nM, mu, N, eps, estimate),
                           scal, nA)
        if seg is None:        # Algorithm 2's start: Section 3.2's initial gaps
            seg = dict(alpha=[scal["alpha"]], omega=[scal["omega"]], beta=[0.0],
                       R=[((cmu + 1.0) * nA * norms["x"] + nb) * eps, grp["R"]],
                       W=[cmu * nA * norms["k"] * eps, grp["W"]],
                       S=[cmu * nA * norms["g"] * eps], Z=[cmu * nA * norms["l"] * eps])
        else:
            for key, val in (("alpha", scal["alpha"]), ("omega", scal["omega"]),
                             ("beta", scal["beta"]), ("R", grp["R"]), ("W", grp["W"]),
                             ("S", grp["S"]), ("Z", grp["Z"])):
                seg[key].append(val)
        f = evaluate(seg)
        prev = {key: norms[key] for key in ("g", "s", "l", "z", "n", "v")}
        if sn.get("replaced"):
            rep = sn["rep"]
            seg = dict(alpha=[0.0], omega=[scal["omega"]], beta=[0.0],
                       R=[0.0, ((cmu + 1.0) * nA * nrm(sn["x1"]) + nb) * e_r],
                       W=[0.0, cmu * nA * nrm(rep["k"]) * e_r],
                       S=[cmu * nA * norms["g"] * e_r], Z=[cmu * nA * nrm(rep["l"]) * e_r])
            f = evaluate(seg)
            prev.update(s=nrm(rep["s"]), l=nrm(rep["l"]), z=nrm(rep["z"]))
        out.append(f)
    return out
