"""Pipelined BiCGStab with low-precision vector storage (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper analyses one working precision.  The FP32-storage form of the
method checked here is this build's own definition (no passage of the
paper covers it); it is Algorithm 2 (Section 3) in the order of
``krylov.pipelined_bicgstab``, with every quantity's precision spelled out:

* the matrix is rounded once to the storage type (A_s = fl_s(A)); the
  Jacobi diagonal is 1 / fl_s(a_ii), divided in the storage type;
* the recurrence vectors r0, r, k, w, m, t, g, s, l, z, n, v, q, u, y are
  storage-type arrays and every vector line is evaluated in the storage
  type, one rounding per operation, with the FP64 scalars alpha, beta,
  omega rounded to the storage type first;
* SPMVs of storage vectors (v = A n, t = A m and the initial w_0, t_0)
  accumulate in the storage type over A_s in ascending column order;
* x and b are FP64; x_{i+1} = (x_i + alpha_i g_i) + omega_i u_i is an FP64
  update with FP64 scalars and the storage vectors widened;
* dot products widen both operands to FP64 and accumulate in FP64; the
  scalars are FP64;
* the residual replacement (eq:rr) forms r = b - A_s x, s = A_s g, w = A_s k,
  z = A_s l with FP64 accumulation (A_s widened) and rounds each result to
  the storage type; k = M^-1 r and l = M^-1 s in the storage type;
* the automated criterion (Section 3.6) uses the bound with the storage
  type's unit roundoff for the recurrences, the FP64 one for the restart
  after an FP64 replacement, and tau = sqrt of the former.

With ``store=np.float64`` every line reduces to ``krylov.pipelined_bicgstab``
on ``Float64Ops`` and the two give bitwise identical results (a pin in
tests/test_oracle_mixed.py).
"""

from __future__ import annotations

import math

import numpy as np

from .krylov import MAX_FORCED_REPLACEMENTS, STATUS, SolveResult, _GapBound, _GapBoundProducts


def pipelined_bicgstab_lowprec(A, b, *, jacobi=False, store=np.float32, x0=None, tol=1e-10,
                               maxit=1000, rr_period=0, rr_tau=None, rr_mode="periodic",
                               rr_estimate=None, record=False, dot_order="blas", rhat=None,
                               rr_reading="nested", rr_nv=False):
    """Algorithm 2 with `store`-precision vectors (see the module docstring).

    A: scipy CSR (FP64 values, rounded here to `store`); b, x0: FP64.
    ``dot_order``: "blas" (numpy.dot) or "fsum" (the correctly rounded sum of
    the products, ``math.fsum``) -- two summation orders of the same dot
    products, for measuring how fast rounding-order differences grow.
    ``rhat``: a fixed shadow vector in place of r_0 (not in the paper; see
    krylov.pipelined_bicgstab), stored in the storage precision.
    ``rr_nv``: a replacement also recomputes n_i and v_i from the replaced
    z_i (not in the paper; see krylov.pipelined_bicgstab), with the
    storage-type PREC and SPMV of the iteration.
    Returns a ``krylov.SolveResult`` (x in FP64)."""
    S = np.dtype(store).type
    f64 = np.float64
    A_s = A.astype(S)                      # A rounded once to the storage type
    A_w = A_s.astype(f64)                  # the same values, widened
    b = np.asarray(b, dtype=f64)
    n = A.shape[0]
    diag = A.diagonal()
    dinv = (S(1) / diag.astype(S)) if jacobi else None

    def prec(v):                           # M^-1 v in the storage type
        return v if dinv is None else dinv * v

    def spmv(v):                           # storage-type SPMV
        return A_s @ v

    def spmv_wide(v):                      # FP64-accumulated SPMV of A_s
        return A_w @ np.asarray(v, dtype=f64)

    if dot_order == "blas":
        def dot(u, v):
            return float(np.dot(np.asarray(u, dtype=f64), np.asarray(v, dtype=f64)))
    elif dot_order == "fsum":
        def dot(u, v):
            return math.fsum(np.asarray(u, dtype=f64) * np.asarray(v, dtype=f64))
    else:
        raise ValueError(dot_order)

    def norm(v):
        return math.sqrt(dot(v, v))

    eps_s = float(np.finfo(S).eps) / 2.0   # unit roundoff of the storage type
    eps_64 = 2.0 ** -53
    auto = rr_mode == "auto"
    estimate = (S is not f64) if rr_estimate is None else rr_estimate
    tau = rr_tau if rr_tau is not None else math.sqrt(eps_s if auto else eps_64)

    x = np.zeros(n) if x0 is None else np.array(x0, dtype=f64)
    r = (b - spmv_wide(x)).astype(S)       # r_0 = b - A x_0 (FP64), stored
    rhat = r.copy() if rhat is None else np.asarray(rhat, dtype=f64).astype(S)
    k = prec(r)                            # k_0 = M^-1 r_0
    w = spmv(prec(r))                      # w_0 = A k_0
    m = prec(w)                            # m_0 = M^-1 w_0
    t = spmv(prec(w))                      # t_0 = A m_0
    zero = np.zeros(n, dtype=S)
    g, s, l, z, nv, v = zero, zero, zero, zero, zero, zero
    rho = dot(rhat, r)
    rw = dot(rhat, w)
    nb = norm(b)
    rn0 = norm(r)
    rn = rn0
    res = SolveResult(x=x, status=-1, iterations=0, rnorm0=rn0, bnorm=nb)
    if nb == 0:
        res.x = np.zeros(n)
        return _done(res, res.x, STATUS["CONVERGED"], 0, A_w, b)
    if rn0 <= tol * nb:
        return _done(res, x, STATUS["CONVERGED"], 0, A_w, b)
    if rw == 0:
        return _done(res, x, STATUS["BREAKDOWN_RHO"], 0, A_w, b)
    alpha = rho / rw
    beta = 0.0
    omega_prev = 0.0
    forced = 0                             # replacements forced by a failed confirmation
    if auto:
        absA = abs(A)
        nA = math.sqrt(float(absA.sum(axis=0).max()) * float(absA.sum(axis=1).max()))
        nM = float(np.max(np.abs(1.0 / diag))) if jacobi else 1.0
        mu = int(np.max(np.diff(A.indptr)))
        cls = {"nested": _GapBound, "products": _GapBoundProducts}[rr_reading]
        gb = cls(n, mu, nA, nM, eps_s, nb, estimate=estimate, eps_replace=eps_64)
        f_next = gb.start(norm(x), norm(k))
        f_ok_prev = f_next <= tau * rn0
        rr_next = False

    def replace(x, g):
        """eq:rr with FP64 accumulation, results rounded to the storage type."""
        r_ = (b - spmv_wide(x)).astype(S)
        k_ = prec(r_)
        w_ = spmv_wide(k_).astype(S)
        s_ = spmv_wide(g).astype(S)
        l_ = prec(s_)
        z_ = spmv_wide(l_).astype(S)
        return r_, k_, w_, s_, l_, z_

    for i in range(maxit):
        a_s, b_s, wp_s = S(alpha), S(beta), S(omega_prev)
        g = k + b_s * (g - wp_s * l)                       # g_i
        s = w + b_s * (s - wp_s * z)                       # s_i
        l = m + b_s * (l - wp_s * nv)                      # l_i
        z = t + b_s * (z - wp_s * v)                       # z_i
        q = r - a_s * s                                    # q_i
        u = k - a_s * l                                    # u_i
        y = w - a_s * z                                    # y_i
        sig1 = dot(q, y)
        sig2 = dot(y, y)
        nv = prec(z)                                       # n_i
        v = spmv(nv)                                       # v_i = A n_i
        if not (math.isfinite(sig1) and math.isfinite(sig2)):
            return _done(res, x, STATUS["NONFINITE"], i, A_w, b)
        omega = sig1 / sig2 if sig2 != 0 else 0.0
        om_s = S(omega)
        if auto:
            nm = {key: norm(vec) for key, vec in
                  (("x", x), ("g", g), ("u", u), ("q", q), ("y", y), ("r", r), ("s", s),
                   ("k", k), ("l", l), ("w", w), ("z", z), ("m", m), ("t", t), ("n", nv),
                   ("v", v))}
        x = (x + alpha * g.astype(f64)) + omega * u.astype(f64)     # x_{i+1}, FP64
        r = q - om_s * y                                   # r_{i+1}
        k = u - om_s * (m - a_s * nv)                      # k_{i+1}
        w = y - om_s * (t - a_s * v)                       # w_{i+1}
        replaced = False
        if auto:
            f_next = gb.step(alpha, beta, omega, omega_prev, nm)
        due = (rr_next if auto else
               (rr_period > 0 and (i + 1) % rr_period == 0 and rn >= tau * rn0))
        if due:
            r, k, w, s, l, z = replace(x, g)
            if rr_nv:
                nv = prec(z)
                v = spmv(nv)
            res.replacements += 1
            res.rr_iters.append(i)
            replaced = True
            if auto:
                f_next = gb.reset(norm(x), norm(k), norm(g), norm(l), norm(s), norm(z))
        rho_new = dot(rhat, r)
        rw = dot(rhat, w)
        rs = dot(rhat, s)
        rz = dot(rhat, z)
        rr = dot(r, r)
        if not all(math.isfinite(c) for c in (rho_new, rw, rs, rz, rr)):
            return _done(res, x, STATUS["NONFINITE"], i + 1, A_w, b)
        rn = math.sqrt(rr)
        snap = None
        if record:
            snap = dict(i=i, x1=x.copy(), r1=r.copy(), k1=k.copy(), w1=w.copy(), g=g.copy(),
                        s=s.copy(), l=l.copy(), z=z.copy(), v=v.copy(), replaced=replaced)
        if rn <= tol * nb:
            tr = norm(b - spmv_wide(x))
            if tr <= tol * nb or (rr_period <= 0 and not auto) or forced >= MAX_FORCED_REPLACEMENTS:
                res.alpha.append(alpha)
                res.omega.append(omega)
                res.rnorm.append(rn)
                if auto:
                    res.fr.append(f_next)
                if snap is not None:
                    res.snapshots.append(snap)
                st = "CONVERGED" if tr <= tol * nb else "TRUE_RES_NOT_MET"
                return _done(res, x, STATUS[st], i + 1, A_w, b)
            r, k, w, s, l, z = replace(x, g)           # confirmation failed: replace, go on
            if rr_nv:
                nv = prec(z)
                v = spmv(nv)
            forced += 1
            res.replacements += 1
            res.rr_iters.append(i)
            if auto:
                f_next = gb.reset(norm(x), norm(k), norm(g), norm(l), norm(s), norm(z))
            rho_new = dot(rhat, r)
            rw = dot(rhat, w)
            rs = dot(rhat, s)
            rz = dot(rhat, z)
            rn = norm(r)
        if auto:
            f_ok = f_next <= tau * rn
            rr_next = f_ok_prev and not f_ok
            f_ok_prev = f_ok
            res.fr.append(f_next)
        res.alpha.append(alpha)
        res.omega.append(omega)
        res.rnorm.append(rn)
        if snap is not None:
            res.snapshots.append(snap)
        if omega == 0:
            return _done(res, x, STATUS["BREAKDOWN_OMEGA"], i + 1, A_w, b)
        m = prec(w)                                        # m_{i+1}
        t = spmv(m)                                        # t_{i+1}
        if rho_new == 0 or rho == 0:
            return _done(res, x, STATUS["BREAKDOWN_RHO"], i + 1, A_w, b)
        beta = ((alpha / omega) * rho_new) / rho
        den = (rw + beta * rs) - (beta * omega) * rz
        if den == 0:
            return _done(res, x, STATUS["BREAKDOWN_RHO"], i + 1, A_w, b)
        res.beta.append(beta)
        alpha = rho_new / den
        rho = rho_new
        omega_prev = omega
    return _done(res, x, STATUS["MAXIT"], maxit, A_w, b)


def _done(res, x, status, its, A_w, b):
    res.x = x
    res.status = status
    res.iterations = its
    if res.bnorm > 0:
        res.true_rel_res = float(np.linalg.norm(b - A_w @ x)) / res.bnorm
    return res
