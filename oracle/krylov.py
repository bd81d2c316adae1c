"""Classic and pipelined preconditioned BiCGStab, step by step (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Both solvers follow the paper's listings in their order of operations:

* ``classic_bicgstab``   -- Algorithm 1 (Section 2.1).
* ``pipelined_bicgstab`` -- Algorithm 2 (Section 3), with the auxiliary
  quantities of eq:auxvars, and the periodic residual replacement of
  Section 3.6 (eq:rr, performed right after the w-update of the iteration).

Every vector expression is written with the brackets of eq:auxrec0 /
eq:auxrec and is evaluated left to right with one rounding per operation
(NumPy never contracts into fused multiply-adds), which is the
floating-point model of Section 2.

Readings of points the paper leaves open (each is listed in the design doc):

* The preconditioner is applied on the right exactly as the listings do:
  r = b - A x is the unpreconditioned residual and x is updated with
  M^-1-preconditioned directions.  M^-1 is either the identity or the
  Jacobi diagonal ``dinv`` (elementwise product).
* In iteration 0 the listing refers to g, s, l, z, n, v and omega of
  iteration -1; they are taken as zero (beta_0 = 0 makes the terms vanish).
* Stopping: ||r_i|| <= tol * ||b|| on the recursively computed residual
  (Section 3.5 keeps the unpreconditioned residual norm); (r, r) is
  reduced together with the second global reduction.  A recursive
  convergence is confirmed by the true residual ||b - A x||; if that fails
  and residual replacement is enabled, a replacement is performed and the
  iteration continues, otherwise the solve reports TRUE_RES_NOT_MET.
* Periodic replacement: in iteration i, after the w-update, when
  (i+1) mod P == 0 and the last reduced ||r_i|| >= tau * ||r_0|| (tau =
  sqrt(eps), eps = unit roundoff 2^-53), recompute r, k, w from x_{i+1}
  and s, l, z from g_i (the six quantities of eq:rr; n and v are not
  recomputed, the shadow residual r_0 is never replaced).
* Scalars are evaluated left to right as printed:
  beta = ((alpha/omega) * rho') / rho and
  alpha' = rho' / ((rw + beta*rs) - (beta*omega)*rz).
* Breakdowns: rho' = 0 or a zero alpha-denominator -> BREAKDOWN_RHO;
  omega = 0 (including (y, y) = 0, where omega is set to 0 and the update
  x + alpha g, r = q is still performed) -> BREAKDOWN_OMEGA unless that
  update meets the tolerance; a non-finite reduction -> NONFINITE.

Pins: exact-rational equality of the classic and pipelined iterates with and
without replacement (the abstract and Section 3: identical iterates in exact
arithmetic); agreement with SciPy's textbook BiCGStab; the dense LU solution
at convergence; the local error bounds eq:errbounds1-4 and the exact gap
identities eq:Dr-eq:Dz (``oracle.gaps``); a hand-derived 2x2 iteration
(tests/golden).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from fractions import Fraction
from typing import Optional

import numpy as np

# Status codes (numerically the same as the solver library's; declared here
# independently so the oracle imports nothing from the library).
STATUS = {
    "CONVERGED": 0,
    "MAXIT": 1,
    "BREAKDOWN_RHO": 2,
    "BREAKDOWN_OMEGA": 3,
    "NONFINITE": 4,
    "TRUE_RES_NOT_MET": 5,
}


# A recursive convergence whose true residual misses the tolerance is
# followed by a replacement and more iterations at most this many times per
# solve; the next failure ends the solve with TRUE_RES_NOT_MET (the attainable
# accuracy is then above the tolerance, e.g. with FP32 recurrences).
MAX_FORCED_REPLACEMENTS = 3


def unit_roundoff(dtype=np.float64) -> float:
    """Unit roundoff u = 2^-(p) of a binary format with p-bit significand
    (the epsilon of Section 2 read as u; 2^-53 for double)."""
    return float(np.finfo(dtype).eps) / 2.0


# -----------------------------------------------------------------------------
# arithmetic backends
# -----------------------------------------------------------------------------

class Float64Ops:
    """IEEE double arithmetic.

    SPMV is SciPy's CSR product (each row summed sequentially in stored
    column order, one rounding per multiply and per add), PREC is the
    elementwise product with ``dinv`` (or a copy for M = I), DOTPR is
    ``numpy.dot``."""

    exact = False

    def __init__(self, A, dinv: Optional[np.ndarray] = None):
        import scipy.sparse as sp
        self.A = sp.csr_matrix(A)
        self.n = self.A.shape[0]
        self.dinv = None if dinv is None else np.asarray(dinv, dtype=np.float64)

    def spmv(self, v):
        return self.A @ v

    def prec(self, v):
        return v.copy() if self.dinv is None else self.dinv * v

    def norm_bound_A(self):
        """Upper bound sqrt(||A||_1 ||A||_inf) of ||A||_2."""
        absA = abs(self.A)
        n1 = float(np.max(np.asarray(absA.sum(axis=0)).ravel()))
        ninf = float(np.max(np.asarray(absA.sum(axis=1)).ravel()))
        return math.sqrt(n1 * ninf)

    def max_row_nnz(self):
        return int(np.max(np.diff(self.A.indptr)))

    def norm_bound_M(self):
        return 1.0 if self.dinv is None else float(np.max(np.abs(self.dinv)))

    def dot(self, v, w):
        return float(np.dot(v, w))

    def norm(self, v):
        return math.sqrt(self.dot(v, v))

    def zeros(self):
        return np.zeros(self.n)

    def copy(self, v):
        return np.array(v, dtype=np.float64, copy=True)

    def finite(self, *vals):
        return all(math.isfinite(float(a)) for a in vals)

    def zero(self):
        return 0.0

    def scalar_sqrt(self, s):
        return math.sqrt(s)


class BlockJacobiOps(Float64Ops):
    """IEEE double arithmetic with a block-Jacobi preconditioner (a block
    preconditioner of the kind Section 4.1 names as keeping the overlap; the
    paper's experiments use ICC(0) on one block per rank).

    M is the block diagonal of A with consecutive blocks of ``bs`` rows and
    columns (the last one ragged); PREC multiplies each block of the vector
    by the inverse of its diagonal block (NumPy/LAPACK inverse, then a
    matrix-vector product).  With bs = 1 this is the Jacobi preconditioner,
    with bs = N the exact inverse (M = A)."""

    def __init__(self, A, bs: int):
        import scipy.sparse as sp
        super().__init__(A, None)
        if bs < 1:
            raise ValueError("block size must be >= 1")
        self.bs = bs
        self.blocks = []
        for lo in range(0, self.n, bs):
            hi = min(self.n, lo + bs)
            blk = sp.csr_matrix(self.A[lo:hi, lo:hi]).toarray()
            self.blocks.append((lo, hi, np.linalg.inv(blk)))

    def prec(self, v):
        out = np.empty(self.n)
        for lo, hi, inv in self.blocks:
            out[lo:hi] = inv @ v[lo:hi]
        return out

    def norm_bound_M(self):
        return max(float(np.max(np.abs(inv).sum(axis=1))) for _, _, inv in self.blocks)


class ExactOps:
    """Exact rational arithmetic for tiny systems (vectors are NumPy object
    arrays of ``fractions.Fraction``).  Norms used by stopping tests are
    converted to float; everything that enters an iterate stays exact."""

    exact = True

    def __init__(self, A, dinv=None):
        import scipy.sparse as sp
        A = sp.csr_matrix(A)
        self.n = A.shape[0]
        self.rows = []
        for i in range(self.n):
            lo, hi = A.indptr[i], A.indptr[i + 1]
            self.rows.append([(int(A.indices[j]), Fraction(float(A.data[j])))
                              for j in range(lo, hi)])
        self.dinv = None if dinv is None else self.vec(dinv)

    def vec(self, a):
        return np.array([x if isinstance(x, Fraction) else Fraction(float(x)) for x in a],
                        dtype=object)

    def spmv(self, v):
        out = np.empty(self.n, dtype=object)
        for i, row in enumerate(self.rows):
            acc = Fraction(0)
            for j, a in row:
                acc += a * v[j]
            out[i] = acc
        return out

    def prec(self, v):
        return v.copy() if self.dinv is None else self.dinv * v

    def dot(self, v, w):
        acc = Fraction(0)
        for a, b in zip(v, w):
            acc += a * b
        return acc

    def norm(self, v):
        return math.sqrt(float(self.dot(v, v)))

    def zeros(self):
        return np.array([Fraction(0)] * self.n, dtype=object)

    def copy(self, v):
        return self.vec(v)

    def finite(self, *vals):
        return True

    def zero(self):
        return Fraction(0)


# -----------------------------------------------------------------------------
# results
# -----------------------------------------------------------------------------

@dataclass
class SolveResult:
    x: np.ndarray
    status: int
    iterations: int
    replacements: int = 0
    rnorm0: float = 0.0
    bnorm: float = 0.0
    alpha: list = field(default_factory=list)     # alpha_i used in iteration i
    omega: list = field(default_factory=list)     # omega_i of iteration i
    beta: list = field(default_factory=list)      # beta_{i+1} formed at the end of iteration i
    rnorm: list = field(default_factory=list)     # ||r_{i+1}|| after iteration i
    rr_iters: list = field(default_factory=list)  # iterations i in which a replacement ran
    restarts: int = 0                             # restarts after breakdowns (option)
    fr: list = field(default_factory=list)        # f^r_{i+1} after iteration i (automated mode)
    true_rel_res: Optional[float] = None
    snapshots: list = field(default_factory=list)

    @property
    def status_name(self):
        return {v: k for k, v in STATUS.items()}[self.status]


def _finish(res, x, status, its, ops, b):
    res.x = x
    res.status = status
    res.iterations = its
    if not ops.exact and res.bnorm > 0:
        res.true_rel_res = ops.norm(b - ops.spmv(x)) / res.bnorm
    return res


# -----------------------------------------------------------------------------
# Algorithm 1: classic preconditioned BiCGStab
# -----------------------------------------------------------------------------

def classic_bicgstab(ops, b, x0=None, *, tol=1e-10, maxit=1000, record=False, rhat=None):
    """Algorithm 1 (classic preconditioned BiCGStab), Section 2.1.

    Three global reductions per iteration: (r0, s_i); (q_i, y_i), (y_i, y_i);
    (r0, r_{i+1}) together with (r_{i+1}, r_{i+1}) for the stopping test.
    No residual replacement (Section 4.3 performs none for the classic
    method).  ``rhat`` (not in the paper, default r_0): the fixed vector
    the dots are taken against in place of r_0."""
    b = ops.copy(b)
    x = ops.zeros() if x0 is None else ops.copy(x0)
    r = b - ops.spmv(x)                       # r_0 := b - A x_0
    rhat = ops.copy(r) if rhat is None else ops.copy(rhat)   # the shadow residual
    p = ops.copy(r)                           # p_0 := r_0
    rho = ops.dot(rhat, r)                    # (r_0, r_i)
    nb = ops.norm(b)
    rn0 = ops.norm(r)
    res = SolveResult(x=x, status=STATUS["MAXIT"], iterations=0, rnorm0=rn0, bnorm=nb)
    if nb == 0:
        return _finish(res, ops.zeros(), STATUS["CONVERGED"], 0, ops, b)
    if rn0 <= tol * nb:
        return _finish(res, x, STATUS["CONVERGED"], 0, ops, b)
    for i in range(maxit):
        g = ops.prec(p)                       # g_i := M^-1 p_i
        s = ops.spmv(g)                       # s_i := A g_i
        sig = ops.dot(rhat, s)                # GLRED 1: (r_0, s_i)
        if not ops.finite(sig):
            return _finish(res, x, STATUS["NONFINITE"], i, ops, b)
        if sig == 0:
            return _finish(res, x, STATUS["BREAKDOWN_RHO"], i, ops, b)
        alpha = rho / sig                     # alpha_i
        q = r - alpha * s                     # q_i := r_i - alpha_i s_i
        u = ops.prec(q)                       # u_i := M^-1 q_i
        y = ops.spmv(u)                       # y_i := A u_i
        sig1 = ops.dot(q, y)                  # GLRED 2: (q_i, y_i), (y_i, y_i)
        sig2 = ops.dot(y, y)
        if not ops.finite(sig1, sig2):
            return _finish(res, x, STATUS["NONFINITE"], i, ops, b)
        omega = sig1 / sig2 if sig2 != 0 else ops.zero()
        x_in, r_in = x, r
        x = (x + alpha * g) + omega * u       # x_{i+1}
        r = q - omega * y                     # r_{i+1}
        rho_new = ops.dot(rhat, r)            # GLRED 3: (r_0, r_{i+1}) and ||r_{i+1}||
        rr = ops.dot(r, r)
        if not ops.finite(rho_new, rr):
            return _finish(res, x, STATUS["NONFINITE"], i + 1, ops, b)
        rn = math.sqrt(float(rr))
        res.alpha.append(alpha)
        res.omega.append(omega)
        res.rnorm.append(rn)
        if record:
            res.snapshots.append(dict(i=i, alpha=alpha, omega=omega, x=x_in, r=r_in, p=p,
                                      g=g, s=s, q=q, u=u, y=y, x1=ops.copy(x),
                                      r1=ops.copy(r)))
        if rn <= tol * nb:
            tr = ops.norm(b - ops.spmv(x))
            st = STATUS["CONVERGED"] if tr <= tol * nb else STATUS["TRUE_RES_NOT_MET"]
            return _finish(res, x, st, i + 1, ops, b)
        if omega == 0:
            return _finish(res, x, STATUS["BREAKDOWN_OMEGA"], i + 1, ops, b)
        if rho_new == 0:
            return _finish(res, x, STATUS["BREAKDOWN_RHO"], i + 1, ops, b)
        beta = ((alpha / omega) * rho_new) / rho          # beta_i
        res.beta.append(beta)
        p = r + beta * (p - omega * s)                    # p_{i+1}
        rho = rho_new
    return _finish(res, x, STATUS["MAXIT"], maxit, ops, b)


# -----------------------------------------------------------------------------
# Algorithm 2: preconditioned pipelined BiCGStab, with residual replacement
# -----------------------------------------------------------------------------

class _GapBound:
    """Running bound f^r on the residual gap (Section 3.6, eq:DDr_bound).

    The local rounding errors of iteration i are bounded with
    eq:errbounds1-4 (epsilon = `eps`, mu = max nonzeros per row of A,
    mu~ = 1 for a diagonal M^-1, ||A|| and ||M^-1|| upper bounds); the gap
    norms ||Delta^s_i||, ||Delta^w_i||, ||Delta^z_i|| are bounded the same
    way from eq:DDs, eq:DDw, eq:DDz, i.e. by the triangle inequality applied
    to eq:Ds, eq:Dw, eq:Dz one iteration at a time, and f^r accumulates them
    as eq:DDr_bound does.  (This is the printed bound with the moduli of the
    coefficients of each of its sums: products of the moduli of the error
    propagation matrices of eq:all_matrices.  ``oracle.gapbound_matrix``
    evaluates the same number from those matrices.)

    Initial gaps as in Section 3.2: ||Delta^r_0|| <= ((mu sqrt(N) + 1) ||A||
    ||x_0|| + ||b||) eps, ||Delta^w_0|| <= mu sqrt(N) ||A|| ||k_0|| eps,
    ||Delta^s_0|| <= mu sqrt(N) ||A|| ||g_0|| eps and ||Delta^z_0|| <=
    mu sqrt(N) ||A|| ||l_0|| eps; iteration 0's s_0 = w_0 and z_0 = t_0
    (beta_0 = 0) add no local error of their own.  A replacement restarts
    the bounds from the same expressions evaluated for the explicit
    recomputation (x_{i+1}, k_{i+1}, g_i, l_i), in the arithmetic of the
    recomputation (epsilon ``eps_replace``)."""

    def __init__(self, N, mu, nA, nM, eps, nb, estimate=False, eps_replace=None):
        self.N, self.mu, self.nA, self.nM, self.eps, self.nb = N, mu, nA, nM, eps, nb
        self.eps_r = eps if eps_replace is None else eps_replace
        # worst-case factors of eq:errbounds1-4, or their square-root estimates
        # (the typical size of accumulated rounding errors, Section 3.6)
        self.cmu = math.sqrt(mu) if estimate else mu * math.sqrt(N)    # mu sqrt(N)
        self.cmut = 1.0 if estimate else math.sqrt(N)                   # mu~ sqrt(N), mu~ = 1
        self.smu = self.cmu * nA
        self.smut = self.cmut * nM

    def start(self, nx, nk):
        """f^r_0 and ||Delta^w_0|| for r_0 = b - A x_0, w_0 = A k_0; the
        initial s and z gaps are set by the first ``step``."""
        e = self.eps
        self.f = ((self.cmu + 1.0) * self.nA * nx + self.nb) * e
        self.dw = self.smu * nk * e
        self.ds_prev = self.dz_prev = 0.0
        self.first = True
        self.prev = dict(g=0.0, s=0.0, l=0.0, z=0.0, n=0.0, v=0.0)
        return self.f

    def local_bounds(self, a, b, w, wp, nm):
        """eq:errbounds1-4 for iteration i (without the factor epsilon).
        ``nm`` holds the norms of the iteration-i vectors; the iteration i-1
        ones are kept from the previous step; a, b, w, wp are |alpha_i|,
        |beta_i|, |omega_i|, |omega_{i-1}|."""
        nA, smu, smut = self.nA, self.smu, self.smut
        P = self.prev
        return dict(
            x=2 * nm["x"] + 3 * a * nm["g"] + 2 * w * nm["u"],
            r=nm["q"] + 2 * w * nm["y"],
            q=nm["r"] + 2 * a * nm["s"],
            u=nm["k"] + 2 * a * nm["l"],
            y=nm["w"] + 2 * a * nm["z"],
            g=nm["k"] + 3 * b * P["g"] + 4 * b * wp * P["l"],
            s=nm["w"] + 3 * b * P["s"] + 4 * b * wp * P["z"],
            l=(nm["m"] + smut * nm["w"] + 3 * b * P["l"] + 4 * b * wp * P["n"]
               + smut * b * wp * P["z"]),
            z=(nm["t"] + smu * nm["m"] + smut * nA * nm["w"] + 3 * b * P["z"]
               + 4 * b * wp * P["v"] + smu * b * wp * P["n"] + smut * nA * b * wp * P["z"]),
            k=(nm["u"] + 3 * w * nm["m"] + smut * w * nm["w"] + 4 * w * a * nm["n"]
               + smut * w * a * nm["z"]),
            w_=(nm["y"] + 3 * w * nm["t"] + smu * w * nm["m"] + smut * nA * w * nm["w"]
                + 4 * w * a * nm["v"] + smu * w * a * nm["n"] + smut * nA * w * a * nm["z"]),
        )

    def step(self, a, b, w, wp, nm):
        """Advance over iteration i.  `nm` holds the norms of the iteration-i
        vectors x, g, u, q, y, r, s, k, l, w, z, m, t, n, v; a, b, w, wp are
        alpha_i, beta_i, omega_i, omega_{i-1} (their moduli are used).
        Returns f^r_{i+1}."""
        a, b, w, wp = abs(a), abs(b), abs(w), abs(wp)
        e, nA = self.eps, self.nA
        d = {key: val * e for key, val in self.local_bounds(a, b, w, wp, nm).items()}
        if self.first:          # Delta^s_0 and Delta^z_0: the initial gaps
            ds = self.smu * nm["g"] * e
            dz = self.smu * nm["l"] * e
            self.first = False
        else:
            dz = b * self.dz_prev + nA * d["l"] + d["z"]                            # eq:Dz
            ds = self.dw + b * self.ds_prev + b * wp * self.dz_prev + nA * d["g"] + d["s"]  # eq:Ds
        f = (self.f + a * ds + w * self.dw + w * a * dz + nA * d["x"] + d["r"]      # eq:Dr
             + w * nA * d["u"] + d["q"] + w * d["y"])
        dw = self.dw + a * dz + nA * d["k"] + d["w_"] + nA * d["u"] + d["y"]      # eq:Dw
        self.f, self.dw, self.ds_prev, self.dz_prev = f, dw, ds, dz
        self.prev = dict(g=nm["g"], s=nm["s"], l=nm["l"], z=nm["z"], n=nm["n"], v=nm["v"])
        return f

    def reset(self, nx, nk, ng, nl, ns=None, nz=None):
        """After a replacement (eq:rr) from x_{i+1} and g_i: the errors of the
        explicit recomputation, in the arithmetic of the recomputation
        (epsilon ``eps_replace``).  The next iteration's local bounds use the
        replaced s_i, l_i, z_i (norms ``ns``, ``nl``, ``nz``)."""
        e = self.eps_r
        self.f = ((self.cmu + 1.0) * self.nA * nx + self.nb) * e
        self.dw = self.smu * nk * e
        self.ds_prev = self.smu * ng * e
        self.dz_prev = self.smu * nl * e
        self.first = False
        self.prev["l"] = nl
        if ns is not None:
            self.prev["s"] = ns
        if nz is not None:
            self.prev["z"] = nz
        return self.f


class _GapBoundProducts(_GapBound):
    """The other reading of Section 3.6's computation of f^r: the moduli of
    the entries of the nine products of eq:all_error_matrices (column i),
    each times the bound of the local error group it multiplies, summed over
    the columns (the sources j of the errors).  ``_GapBound`` takes the
    printed eq:DDr_bound instead, where each gap norm is bounded first and
    the moduli of the propagation matrices are multiplied; this reading keeps
    the signs inside each product and is never larger.

    The products are those of eq:matrix_expr: the residual gap collects the
    R errors through U; the S errors through BA; the W errors through UEA
    and UC; the Z errors through BAEA, BPA, BAC and BD (A, B, C, D, E, P, U
    of eq:all_matrices, built from the signed alpha, beta, omega).  Column c
    of every partial product is kept as a vector over the sources and moved
    to column c+1 with the recursions the matrices obey:

    * a product ending in A, C or D gains, in column c+1, its left factor's
      column c times -alpha_c, -omega_c or omega_c alpha_c;
    * one ending in E, B or P is scaled by beta_{c+1} and gains the left
      factor's column c+1 (E, B) or column c times -omega_c (P);
    * U accumulates: every source enters with coefficient 1.

    The A/C/D step needs alpha_c, omega_c only (so f^r_{c+1} is known at the
    end of iteration c); the E/B/P step waits for beta_{c+1}, which the next
    iteration brings.  Column 0 holds the initial gaps (Section 3.2); R and W
    sources of iteration c sit in column c+1, S and Z sources in column c.
    A replacement starts a new system whose column 0 holds the recomputed s
    and z gaps, with alpha_0 = 0 and the recomputed r and w gaps in column 1.
    The local error bounds are the same as ``_GapBound``'s."""

    _PRODUCTS = ("B", "BA", "BD", "BAC", "BAE", "BAEA", "BP", "BPA", "U", "UE", "UEA", "UC")

    def _segment(self):
        cap = 64
        self.M = {k: np.zeros(cap) for k in self._PRODUCTS}
        self.th = {k: np.zeros(cap) for k in "RSWZ"}
        self.M["B"][0] = 1.0
        self.M["U"][0] = 1.0
        self.c = 0                                     # current column (sources 0..c)

    def _grow(self):
        if self.c + 2 <= len(self.M["B"]):
            return
        for d in (self.M, self.th):
            for k in d:
                d[k] = np.concatenate([d[k], np.zeros(len(d[k]))])

    def _step_acd(self, alpha, omega):
        """Column c -> c+1 of the products that end in A, C, D or U."""
        M, c = self.M, self.c
        self._grow()
        sl = slice(0, c + 1)
        old_ba = M["BA"][sl].copy()
        M["BA"][sl] -= alpha * M["B"][sl]
        M["BD"][sl] += omega * alpha * M["B"][sl]
        M["BAC"][sl] -= omega * old_ba
        M["BAEA"][sl] -= alpha * M["BAE"][sl]
        M["BPA"][sl] -= alpha * M["BP"][sl]
        M["UEA"][sl] -= alpha * M["UE"][sl]
        M["UC"][sl] -= omega * M["U"][sl]
        M["U"][c + 1] = 1.0                            # the new source row c+1

    def _step_ebp(self, beta, omega_prev):
        """Column c -> c+1 of the products that end in B, E or P (after
        ``_step_acd`` moved the A/U products to column c+1)."""
        M, c = self.M, self.c
        sl = slice(0, c + 1)
        M["BP"][sl] = beta * (M["BP"][sl] - omega_prev * M["B"][sl])
        M["B"][sl] *= beta
        M["B"][c + 1] = 1.0
        sl1 = slice(0, c + 2)
        M["BAE"][sl1] = beta * M["BAE"][sl1] + M["BA"][sl1]
        M["UE"][sl1] = beta * M["UE"][sl1] + M["U"][sl1]
        self.c = c + 1

    def _value(self):
        M, th, n = self.M, self.th, self.c + 2       # sources 0..c+1 of column c+1
        a = np.abs
        f = (np.sum(th["R"][:n])
             + np.sum(th["S"][:n] * a(M["BA"][:n]))
             + np.sum(th["W"][:n] * (a(M["UEA"][:n]) + a(M["UC"][:n])))
             + np.sum(th["Z"][:n] * (a(M["BAEA"][:n]) + a(M["BPA"][:n]) + a(M["BAC"][:n])
                                     + a(M["BD"][:n]))))
        return float(f)

    def start(self, nx, nk):
        e = self.eps
        self._segment()
        self.th["R"][0] = ((self.cmu + 1.0) * self.nA * nx + self.nb) * e
        self.th["W"][0] = self.smu * nk * e
        self.first = True
        self.pending = False
        self.prev = dict(g=0.0, s=0.0, l=0.0, z=0.0, n=0.0, v=0.0)
        self.f = float(self.th["R"][0])
        return self.f

    def step(self, a, b, w, wp, nm):
        e, nA = self.eps, self.nA
        d = {key: val * e for key, val in
             self.local_bounds(abs(a), abs(b), abs(w), abs(wp), nm).items()}
        if self.first:          # Delta^s_0 and Delta^z_0: the initial gaps
            self.th["S"][0] = self.smu * nm["g"] * e
            self.th["Z"][0] = self.smu * nm["l"] * e
            self.first = False
        else:
            if self.pending:    # column c of the B/E/P products needs beta_c
                self._step_ebp(b, wp)
            c = self.c
            self.th["S"][c] = nA * d["g"] + d["s"]
            self.th["Z"][c] = nA * d["l"] + d["z"]
        self._step_acd(a, w)
        c = self.c
        self.th["R"][c + 1] = (nA * d["x"] + d["r"] + abs(w) * nA * d["u"] + d["q"]
                               + abs(w) * d["y"])
        self.th["W"][c + 1] = nA * d["k"] + d["w_"] + nA * d["u"] + d["y"]
        self.pending = True
        self.f = self._value()
        self.prev = dict(g=nm["g"], s=nm["s"], l=nm["l"], z=nm["z"], n=nm["n"], v=nm["v"])
        return self.f

    def reset(self, nx, nk, ng, nl, ns=None, nz=None):
        e = self.eps_r
        self._segment()
        self.th["S"][0] = self.smu * ng * e
        self.th["Z"][0] = self.smu * nl * e
        self._step_acd(0.0, 0.0)                       # the leading step: alpha = 0
        self.th["R"][1] = ((self.cmu + 1.0) * self.nA * nx + self.nb) * e
        self.th["W"][1] = self.smu * nk * e
        self.first = False
        self.pending = True
        self.prev["l"] = nl
        if ns is not None:
            self.prev["s"] = ns
        if nz is not None:
            self.prev["z"] = nz
        self.f = self._value()
        return self.f


def pipelined_bicgstab(ops, b, x0=None, *, tol=1e-10, maxit=1000, rr_period=0,
                       rr_tau=None, rr_mode="periodic", rr_eps=None, rr_estimate=False,
                       rr_reading="nested", restarts=0, record=False, rhat=None,
                       rr_nv=False):
    """Algorithm 2 (preconditioned p-BiCGStab), Section 3, with residual
    replacement (Section 3.6, eq:rr):

    * ``rr_mode="periodic"``: every ``rr_period`` iterations while
      ||r_i|| >= tau ||r_0|| (tau = sqrt(eps) by default);
    * ``rr_mode="auto"``: the automated strategy -- the running bound f^r of
      eq:DDr_bound (``_GapBound``, epsilon = ``rr_eps``, default the unit
      roundoff) and the criterion eq:criterion: replace in step i when
      f^r_{i-1} <= tau ||r_{i-1}|| and f^r_i > tau ||r_i||, tau = sqrt(eps);
      with ``rr_estimate`` the square-root estimate of the bound (Section
      3.6 suggests it as a less pessimistic alternative); ``rr_reading``
      "nested" evaluates eq:DDr_bound as printed (``_GapBound``), "products"
      the moduli of the products of eq:all_error_matrices
      (``_GapBoundProducts``).

    Two global reductions per iteration, each overlapped (on parallel
    hardware) by one PREC + SPMV: (q_i, y_i), (y_i, y_i) with
    n_i = M^-1 z_i, v_i = A n_i; and (r0, r_{i+1}), (r0, w_{i+1}),
    (r0, s_i), (r0, z_i) -- plus (r_{i+1}, r_{i+1}) for the stopping test --
    with m_{i+1} = M^-1 w_{i+1}, t_{i+1} = A m_{i+1}.  In automated mode the
    norms entering the bound are reduced with the second global reduction
    (Section 3.6: no extra synchronisation).

    ``restarts`` (not in the paper, default 0): after a rho' = 0 or zero
    alpha-denominator breakdown in iteration i, up to this many times, the
    method starts again from x_{i+1}: the initialisation of Algorithm 2 is
    repeated with x_0 := x_{i+1} (new r_0 = b - A x_{i+1}, which is also the
    new shadow residual), the iteration count continues.

    ``rhat`` (not in the paper, default r_0): a fixed shadow vector that
    replaces r_0 in every dot (r_0, .) of the algorithm, also after a
    restart.  BiCGStab admits any such vector with (rhat, r_0) != 0; r_0
    itself breaks down when the operator's column sums vanish and r_0 is a
    constant vector, since (1, b - A x_i) then depends on the boundary
    values of x_i alone and tends to zero long before r_i does.

    ``rr_nv`` (not in the paper, default False): a replacement also
    recomputes n_i := M^-1 z_i and v_i := A n_i from the replaced z_i, the
    definitions eq:auxvars gives them; the next iteration's l and z
    recurrences then combine n_i, v_i and z_i of the same z_i.  By default
    only the six quantities of eq:rr are recomputed and n_i, v_i keep the
    values computed from the recursive z_i before the replacement."""
    auto = rr_mode == "auto"
    rhat_in = None if rhat is None else ops.copy(rhat)
    if rr_mode not in ("periodic", "auto"):
        raise ValueError(rr_mode)
    eps = unit_roundoff() if rr_eps is None else rr_eps
    tau = math.sqrt(eps if auto else unit_roundoff()) if rr_tau is None else rr_tau
    b = ops.copy(b)
    x = ops.zeros() if x0 is None else ops.copy(x0)

    def initialise(x):
        """The two lines before the loop of Algorithm 2."""
        r = b - ops.spmv(x)                   # r_0 := b - A x_0
        # shadow residual r_0 (never replaced), or the caller's fixed vector
        rhat = ops.copy(r) if rhat_in is None else rhat_in
        k = ops.prec(r)                       # k_0 := M^-1 r_0
        w = ops.spmv(k)                       # w_0 := A k_0
        m = ops.prec(w)                       # m_0 := M^-1 w_0
        t = ops.spmv(m)                       # t_0 := A m_0
        rho = ops.dot(rhat, r)                # (r_0, r_0)
        den = ops.dot(rhat, w)                # (r_0, w_0)
        return r, rhat, k, w, m, t, rho, den

    r, rhat, k, w, m, t, rho, den = initialise(x)
    nb = ops.norm(b)
    rn0 = ops.norm(r)
    rn = rn0
    res = SolveResult(x=x, status=STATUS["MAXIT"], iterations=0, rnorm0=rn0, bnorm=nb)
    if nb == 0:
        return _finish(res, ops.zeros(), STATUS["CONVERGED"], 0, ops, b)
    if rn0 <= tol * nb:
        return _finish(res, x, STATUS["CONVERGED"], 0, ops, b)
    if not ops.finite(rho, den):
        return _finish(res, x, STATUS["NONFINITE"], 0, ops, b)
    if den == 0:
        return _finish(res, x, STATUS["BREAKDOWN_RHO"], 0, ops, b)
    alpha = rho / den                         # alpha_0
    beta = ops.zero()                         # beta_0 := 0
    omega_prev = ops.zero()                   # omega_{-1} (taken as 0)
    g, s, l, z, n, v = (ops.zeros() for _ in range(6))   # iteration -1 values (taken as 0)
    gb = None
    rr_next = False
    forced = 0                                # replacements forced by a failed confirmation
    if auto:
        cls = {"nested": _GapBound, "products": _GapBoundProducts}[rr_reading]
        gb = cls(ops.n, ops.max_row_nnz(), ops.norm_bound_A(), ops.norm_bound_M(), eps, nb,
                 estimate=rr_estimate)
        f_cur = gb.start(ops.norm(x), ops.norm(k))
        f_ok_prev = f_cur <= tau * rn0

    def replace(x, g):
        """eq:rr: explicit recomputation of r, k, w (from x) and s, l, z (from g)."""
        r_ = b - ops.spmv(x)
        k_ = ops.prec(r_)
        w_ = ops.spmv(k_)
        s_ = ops.spmv(g)
        l_ = ops.prec(s_)
        z_ = ops.spmv(l_)
        return r_, k_, w_, s_, l_, z_

    for i in range(maxit):
        # recurrences for the auxiliary vectors (each uses iteration i-1 values)
        g_new = k + beta * (g - omega_prev * l)        # g_i
        s_new = w + beta * (s - omega_prev * z)        # s_i
        l_new = m + beta * (l - omega_prev * n)        # l_i
        z_new = t + beta * (z - omega_prev * v)        # z_i
        g, s, l, z = g_new, s_new, l_new, z_new
        q = r - alpha * s                              # q_i
        u = k - alpha * l                              # u_i
        y = w - alpha * z                              # y_i
        sig1 = ops.dot(q, y)                           # GLRED 1 begins: (q_i, y_i), (y_i, y_i)
        sig2 = ops.dot(y, y)
        n = ops.prec(z)                                # n_i := M^-1 z_i   (overlaps GLRED 1)
        v = ops.spmv(n)                                # v_i := A n_i
        if not ops.finite(sig1, sig2):                 # GLRED 1 ends
            return _finish(res, x, STATUS["NONFINITE"], i, ops, b)
        omega = sig1 / sig2 if sig2 != 0 else ops.zero()   # omega_i
        if auto:   # norms of the iteration-i vectors (reduced with GLRED 2)
            nm = {key: ops.norm(vec) for key, vec in
                  (("x", x), ("g", g), ("u", u), ("q", q), ("y", y), ("r", r), ("s", s),
                   ("k", k), ("l", l), ("w", w), ("z", z), ("m", m), ("t", t), ("n", n),
                   ("v", v))}
        x_new = (x + alpha * g) + omega * u            # x_{i+1}
        r_new = q - omega * y                          # r_{i+1}
        k_new = u - omega * (m - alpha * n)            # k_{i+1}
        w_new = y - omega * (t - alpha * v)            # w_{i+1}
        snap = None
        if record:
            snap = dict(i=i, alpha=alpha, beta=beta, omega=omega, omega_prev=omega_prev,
                        x=x, r=r, k=k, w=w, m=m, t=t, g=g, s=s, l=l, z=z, q=q, u=u, y=y,
                        n=n, v=v, x1=x_new, r1=r_new, k1=k_new, w1=w_new, replaced=False)
        x, r, k, w = x_new, r_new, k_new, w_new
        replaced = False
        if auto:
            f_next = gb.step(float(alpha), float(beta), float(omega), float(omega_prev), nm)
        due = (rr_next if auto else
               (rr_period > 0 and (i + 1) % rr_period == 0 and rn >= tau * rn0))
        if due:
            r, k, w, s, l, z = replace(x, g)           # eq:rr, right after the w-update
            if rr_nv:
                n = ops.prec(z)                        # n_i, v_i of the replaced z_i
                v = ops.spmv(n)
            res.replacements += 1
            res.rr_iters.append(i)
            replaced = True
            if snap is not None:
                snap["rep"] = dict(r=r, k=k, w=w, s=s, l=l, z=z, n=n, v=v)
            if auto:
                f_next = gb.reset(ops.norm(x), ops.norm(k), ops.norm(g), ops.norm(l),
                                  ops.norm(s), ops.norm(z))
        rho_new = ops.dot(rhat, r)                     # GLRED 2 begins: (r0, r_{i+1}),
        rw = ops.dot(rhat, w)                          #   (r0, w_{i+1}), (r0, s_i),
        rs = ops.dot(rhat, s)                          #   (r0, z_i) and (r_{i+1}, r_{i+1})
        rz = ops.dot(rhat, z)
        rr = ops.dot(r, r)
        if not ops.finite(rho_new, rw, rs, rz, rr):
            return _finish(res, x, STATUS["NONFINITE"], i + 1, ops, b)
        rn = math.sqrt(float(rr))
        if rn <= tol * nb:
            tr = ops.norm(b - ops.spmv(x))
            if tr <= tol * nb:
                res.alpha.append(alpha)
                res.omega.append(omega)
                res.rnorm.append(rn)
                if auto:
                    res.fr.append(f_next)
                if snap is not None:
                    snap["replaced"] = replaced
                    res.snapshots.append(snap)
                return _finish(res, x, STATUS["CONVERGED"], i + 1, ops, b)
            if (rr_period <= 0 and not auto) or forced >= MAX_FORCED_REPLACEMENTS:
                res.alpha.append(alpha)
                res.omega.append(omega)
                res.rnorm.append(rn)
                if auto:
                    res.fr.append(f_next)
                return _finish(res, x, STATUS["TRUE_RES_NOT_MET"], i + 1, ops, b)
            r, k, w, s, l, z = replace(x, g)           # confirm failed: replace and go on
            if rr_nv:
                n = ops.prec(z)
                v = ops.spmv(n)
            forced += 1
            res.replacements += 1
            res.rr_iters.append(i)
            replaced = True
            if snap is not None:
                snap["rep"] = dict(r=r, k=k, w=w, s=s, l=l, z=z)
            if auto:
                f_next = gb.reset(ops.norm(x), ops.norm(k), ops.norm(g), ops.norm(l),
                                  ops.norm(s), ops.norm(z))
            rho_new = ops.dot(rhat, r)
            rw = ops.dot(rhat, w)
            rs = ops.dot(rhat, s)
            rz = ops.dot(rhat, z)
            rr = ops.dot(r, r)
            rn = math.sqrt(float(rr))
        if auto:   # eq:criterion for step i+1
            f_ok = f_next <= tau * rn
            rr_next = f_ok_prev and not f_ok
            f_ok_prev = f_ok
            res.fr.append(f_next)
        res.alpha.append(alpha)
        res.omega.append(omega)
        res.rnorm.append(rn)
        if snap is not None:
            snap["replaced"] = replaced
            res.snapshots.append(snap)
        if omega == 0:
            return _finish(res, x, STATUS["BREAKDOWN_OMEGA"], i + 1, ops, b)
        m = ops.prec(w)                                # m_{i+1} := M^-1 w_{i+1} (overlaps GLRED 2)
        t = ops.spmv(m)                                # t_{i+1} := A m_{i+1}
        breakdown = rho_new == 0 or rho == 0           # GLRED 2 ends
        if not breakdown:
            beta = ((alpha / omega) * rho_new) / rho   # beta_{i+1}
            den = (rw + beta * rs) - (beta * omega) * rz
            breakdown = den == 0
        if breakdown:
            if res.restarts >= restarts:
                return _finish(res, x, STATUS["BREAKDOWN_RHO"], i + 1, ops, b)
            # start again from x_{i+1} (not in the paper; see the docstring)
            res.restarts += 1
            res.beta.append(ops.zero())
            r, rhat, k, w, m, t, rho, den = initialise(x)
            rn0 = ops.norm(r)
            rn = rn0
            if rn0 <= tol * nb:
                return _finish(res, x, STATUS["CONVERGED"], i + 1, ops, b)
            if not ops.finite(rho, den):
                return _finish(res, x, STATUS["NONFINITE"], i + 1, ops, b)
            if den == 0:
                return _finish(res, x, STATUS["BREAKDOWN_RHO"], i + 1, ops, b)
            alpha = rho / den
            beta = ops.zero()
            omega_prev = ops.zero()
            g, s, l, z, n, v = (ops.zeros() for _ in range(6))
            if auto:
                f_cur = gb.start(ops.norm(x), ops.norm(k))
                f_ok_prev = f_cur <= tau * rn0
                rr_next = False
            continue
        res.beta.append(beta)
        alpha = rho_new / den                          # alpha_{i+1}
        rho = rho_new
        omega_prev = omega
    return _finish(res, x, STATUS["MAXIT"], maxit, ops, b)
