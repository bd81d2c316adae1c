"""Python face of the HIP library: a Solver handle and differentiable solves.

Argument marshalling only -- every step of a solve runs in the library's
kernels.  Device vectors are torch CUDA float64 tensors; torch provides the
device memory and the stream (``torch.cuda.current_stream()``), nothing else.
"""

from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_vec(t: torch.Tensor, n: int, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return t.contiguous()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_PRECISION = {"fp64": L.FP64, "mixed": L.MIXED}
_PRECOND = {"none": L.PC_NONE, None: L.PC_NONE, "jacobi": L.PC_JACOBI}


def _pc_code(precond) -> int:
    """'none', 'jacobi' or 'block<b>' (block-Jacobi with blocks of b rows,
    CSR only: PBCG_PC_BLOCK_JACOBI(b))."""
    if isinstance(precond, str) and precond.startswith("block"):
        return L.PC_BLOCK_JACOBI_BASE | int(precond[len("block"):])
    return _PRECOND[precond]
_KIND = {"2d5": L.ST_2D5, "3d7": L.ST_3D7, "dia5": L.ST_DIA5}


def workspace_bytes(fmt: str, n: int, nnz: int = 0, width: int = 0, precision="fp64",
                    precond="jacobi", with_transpose=True) -> int:
    """pbicgstab_workspace_bytes for a format 'csr', '2d5', '3d7' or 'dia5'."""
    code = L.CSR if fmt == "csr" else _KIND[fmt]
    nb = L.load().pbicgstab_workspace_bytes(code, n, nnz, width, _PRECISION[precision],
                                            _pc_code(precond), 1 if with_transpose else 0)
    if nb == 0:
        msg = L.load().pbicgstab_last_error()
        raise L.PbcgError(-1, msg.decode() if msg else "invalid workspace query")
    return int(nb)


def _workspace(nbytes: int) -> torch.Tensor:
    """Caller-owned device workspace: a uint8 CUDA tensor (torch's caching
    allocator returns blocks aligned far beyond the 256 bytes required)."""
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace tensor is not 256-byte aligned")
    return ws


class Solver:
    """A matrix living on the GPU, ready for (pipelined) BiCGStab solves.

    Create with :meth:`from_csr` or :meth:`from_stencil` (NumPy or torch
    input; the arrays are handed to the library as device tensors).  The
    handle's device data lives in a uint8 torch tensor this object owns
    (``workspace``), sized by pbicgstab_workspace_bytes.
    """

    def __init__(self, handle, n: int, kind: str, precision: str, precond: str, dims=None,
                 nnz: int = 0, workspace: Optional[torch.Tensor] = None):
        self._h = handle
        self.n = n
        self.kind = kind
        self.precision = precision
        self.precond = precond
        self.dims = dims
        self.nnz = nnz
        self.workspace = workspace

    # ---- construction -------------------------------------------------
    @classmethod
    def from_csr(cls, rowptr, col, val, precision="fp64", precond="jacobi",
                 with_transpose=True, workspace: Optional[torch.Tensor] = None):
        lib = L.load()
        torch.cuda.init()
        rp = torch.as_tensor(np.ascontiguousarray(rowptr, dtype=np.int32)
                             if not isinstance(rowptr, torch.Tensor) else rowptr,
                             dtype=torch.int32).cuda().contiguous()
        cl = torch.as_tensor(np.ascontiguousarray(col, dtype=np.int32)
                             if not isinstance(col, torch.Tensor) else col,
                             dtype=torch.int32).cuda().contiguous()
        vl = torch.as_tensor(np.ascontiguousarray(val, dtype=np.float64)
                             if not isinstance(val, torch.Tensor) else val,
                             dtype=torch.float64).cuda().contiguous()
        n = rp.numel() - 1
        nnz = cl.numel()
        if isinstance(precond, str) and precond.startswith("block"):
            with_transpose = False          # block-Jacobi handles have no transpose
        # slice-width bound of the sliced-ELL layouts: longest row (and column)
        rows = torch.diff(rp.to(torch.int64))
        width = int(rows.max()) if n > 0 else 0
        if with_transpose and nnz > 0:
            width = max(width, int(torch.bincount(cl.to(torch.int64), minlength=n).max()))
        if workspace is None:
            workspace = _workspace(workspace_bytes("csr", n, nnz, width, precision, precond,
                                                   with_transpose))
        h = ctypes.c_void_p()
        L.check(lib.pbicgstab_create_csr(
            ctypes.byref(h), n, nnz, _ptr(rp), _ptr(cl), _ptr(vl), _PRECISION[precision],
            _pc_code(precond), _ptr(workspace), workspace.numel(), _stream()))
        return cls(h, n, "csr", precision, precond, nnz=nnz, workspace=workspace)

    @classmethod
    def from_stencil(cls, kind, dims, coef, precision="fp64", precond="jacobi",
                     with_transpose=True, workspace: Optional[torch.Tensor] = None):
        """kind: '2d5' (coef S,W,C,E,N), '3d7' (D,S,W,C,E,N,U) or 'dia5'
        (coef array (5, N) in the order S, W, C, E, N)."""
        lib = L.load()
        torch.cuda.init()
        dims_a = np.ascontiguousarray(dims, dtype=np.int64)
        n = int(np.prod(dims_a))
        if kind == "dia5":
            coef_t = torch.as_tensor(np.ascontiguousarray(coef, dtype=np.float64).reshape(-1)
                                     if not isinstance(coef, torch.Tensor) else coef.reshape(-1),
                                     dtype=torch.float64).cuda().contiguous()
            coef_p = _ptr(coef_t)
        else:
            coef_a = np.ascontiguousarray(coef, dtype=np.float64).reshape(-1)
            coef_p = coef_a.ctypes.data_as(ctypes.c_void_p)
        if workspace is None:
            workspace = _workspace(workspace_bytes(kind, n, 0, 0, precision, precond,
                                                   with_transpose))
        h = ctypes.c_void_p()
        L.check(lib.pbicgstab_create_stencil(
            ctypes.byref(h), _KIND[kind], dims_a.ctypes.data_as(ctypes.c_void_p), coef_p,
            _PRECISION[precision], _PRECOND[precond], _ptr(workspace), workspace.numel(),
            _stream()))
        nn = ctypes.c_int64()
        L.check(lib.pbicgstab_info(h, None, ctypes.byref(nn), None))
        return cls(h, n, kind, precision, precond, dims=tuple(int(d) for d in dims_a),
                   nnz=nn.value, workspace=workspace)

    @classmethod
    def from_problem(cls, prob, form="csr", precision="fp64", precond=None):
        """From a workloads.Problem: form 'csr', 'stencil' or 'dia5'."""
        pc = precond if precond is not None else prob.precond
        if form == "csr":
            return cls.from_csr(prob.rowptr, prob.col, prob.val, precision, pc)
        if form == "stencil":
            st = prob.stencil
            return cls.from_stencil(st.kind, st.dims, st.coef_vector(), precision, pc)
        if form == "dia5":
            return cls.from_stencil("dia5", prob.dims, prob.dia5, precision, pc)
        raise ValueError(form)

    # ---- solves ---------------------------------------------------------
    def _opts(self, tol, maxit, rr_period, rr_tau, check_every, transpose, history, gap_every,
              gap_history, use_graph, rr_auto=False, rr_eps=0.0, bound_history=None,
              restarts=0, single_kernel=False, rr_nv=False):
        o = L.Opts()
        L.load().pbicgstab_default_opts(ctypes.byref(o))
        o.tol = tol
        o.maxit = maxit
        o.rr_period = rr_period
        o.rr_tau = rr_tau
        o.check_every = check_every
        o.transpose = 1 if transpose else 0
        if history is not None:
            o.history = history.data_ptr()
            o.history_len = history.numel() // 4
        o.gap_every = gap_every
        if gap_history is not None:
            o.gap_history = gap_history.data_ptr()
            o.gap_len = gap_history.numel()
        o.use_graph = 1 if use_graph else 0
        o.stream = torch.cuda.current_stream().cuda_stream
        if rr_auto in (False, None, 0):
            o.rr_auto = 0
        elif rr_auto == "bound":
            o.rr_auto = 1
        elif rr_auto == "estimate":
            o.rr_auto = 2
        elif rr_auto == "products":
            o.rr_auto = 3
        elif rr_auto == "products-estimate":
            o.rr_auto = 4
        else:   # True: the worst-case bound in FP64, the estimate with FP32 recurrences
            o.rr_auto = 1 if self.precision == "fp64" else 2
        o.rr_eps = rr_eps
        if bound_history is not None:
            o.bound_history = bound_history.data_ptr()
            o.bound_len = bound_history.numel()
        o.restarts = restarts
        o.single_kernel = 1 if single_kernel else 0
        o.rr_nv = 1 if rr_nv else 0
        return o

    def solve(self, b: torch.Tensor, x0: Optional[torch.Tensor] = None, *, tol=1e-10,
              maxit=10000, rr_period=0, rr_tau=0.0, check_every=0, transpose=False,
              history: Optional[torch.Tensor] = None, gap_every=0,
              gap_history: Optional[torch.Tensor] = None, use_graph=False,
              method="pipelined", out: Optional[torch.Tensor] = None, rr_auto=False,
              rr_eps=0.0, bound_history: Optional[torch.Tensor] = None, restarts=0,
              rhat: Optional[torch.Tensor] = None, single_kernel=False, rr_nv=False):
        """Solve A x = b (A^T x = b with transpose).  Returns (x, stats dict).

        method: 'pipelined' (Algorithm 2 with residual replacement: every
        ``rr_period`` iterations, or automated with ``rr_auto``) or 'classic'
        (Algorithm 1).  ``rr_auto``: False, True (the bound in FP64, its
        estimate with FP32 storage), 'bound', 'estimate' (eq:DDr_bound as
        printed), 'products', 'products-estimate' (the moduli of the products
        of the error propagation matrices; the binding allocates the state
        the library needs).  ``rhat``: a fixed shadow vector in place of r_0
        (not in the paper; None keeps r_0).  ``single_kernel``: run the whole
        solve as one kernel in one workgroup when the system allows it (FP64,
        at most 2048 rows, no or periodic replacement, or up to 1024 rows the
        automated one -- not the 'products' readings; stats
        ``single_kernel`` says whether it did).  ``rr_nv``: every replacement
        also recomputes n = M^-1 z and v = A n from the replaced z (not in the
        paper, which replaces the six quantities of eq:rr only)."""
        lib = L.load()
        b = _dev_vec(b, self.n, "b")
        rhat = None if rhat is None else _dev_vec(rhat, self.n, "rhat")
        if out is None:
            out = torch.zeros_like(b) if x0 is None else _dev_vec(x0, self.n, "x0").clone()
        elif x0 is not None:
            out.copy_(x0)
        for t, nm in ((history, "history"), (gap_history, "gap_history"),
                      (bound_history, "bound_history")):
            if t is not None and (not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous()):
                raise TypeError(f"{nm} must be a contiguous CUDA float64 tensor")
        o = self._opts(tol, maxit, rr_period, rr_tau, check_every, transpose, history, gap_every,
                       gap_history, use_graph, rr_auto, rr_eps, bound_history, restarts,
                       single_kernel, rr_nv)
        if rhat is not None:
            o.rhat = rhat.data_ptr()
        state = None
        if o.rr_auto >= 3:      # the products reading's per-iteration state
            state = torch.empty(16 * (maxit + 2), dtype=torch.float64, device=b.device)
            o.bound_state = state.data_ptr()
            o.bound_state_len = state.numel()
        st = L.Stats()
        fn = lib.pbicgstab_solve if method == "pipelined" else lib.classic_bicgstab_solve
        code = fn(self._h, _ptr(b), _ptr(out), ctypes.byref(o), ctypes.byref(st))
        L.check(code)
        return out, st.as_dict()

    def apply(self, x: torch.Tensor, transpose=False) -> torch.Tensor:
        x = _dev_vec(x, self.n, "x")
        y = torch.empty_like(x)
        L.check(L.load().pbicgstab_apply(self._h, _ptr(x), _ptr(y), 1 if transpose else 0,
                                         _stream()))
        return y

    def grad_values(self, lam: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
        lam = _dev_vec(lam, self.n, "lambda")
        x = _dev_vec(x, self.n, "x")
        size = {"csr": self.nnz, "dia5": 5 * self.n, "2d5": 5, "3d7": 7}[self.kind]
        g = torch.empty(size, dtype=torch.float64, device=x.device)
        L.check(L.load().pbicgstab_grad_values(self._h, _ptr(lam), _ptr(x), _ptr(g), _stream()))
        return g

    def update_values(self, values: torch.Tensor):
        if values.is_cuda:
            v = values.detach().to(torch.float64).contiguous()
            L.check(L.load().pbicgstab_update_values(self._h, _ptr(v), 1, _stream()))
        else:
            v = np.ascontiguousarray(values.detach().numpy(), dtype=np.float64)
            L.check(L.load().pbicgstab_update_values(
                self._h, v.ctypes.data_as(ctypes.c_void_p), 0, _stream()))

    def assemble_kappa(self, kappa: torch.Tensor, conv=(1.0, 0.0), h=None):
        kappa = _dev_vec(kappa.reshape(-1), self.n, "kappa")
        hh = h if h is not None else 1.0 / (self.dims[0] + 1)
        L.check(L.load().pbicgstab_dia5_assemble_kappa(self._h, _ptr(kappa), conv[0], conv[1],
                                                       hh, _stream()))

    def kappa_grad(self, lam: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
        lam = _dev_vec(lam, self.n, "lambda")
        x = _dev_vec(x, self.n, "x")
        g = torch.empty_like(x)
        L.check(L.load().pbicgstab_dia5_kappa_grad(self._h, _ptr(lam), _ptr(x), _ptr(g),
                                                   _stream()))
        return g

    VEC_IDS = {"rhat": 0, "r": 1, "g": 2, "s": 3, "l": 4, "z": 5, "k": 6, "w": 7, "t": 8,
               "v": 9, "x": 10, "dinv": 11}

    def get_vector(self, which: str, device="cuda") -> torch.Tensor:
        out = torch.empty(self.n, dtype=torch.float64, device=device)
        L.check(L.load().pbicgstab_get_vector(self._h, self.VEC_IDS[which], _ptr(out), _stream()))
        return out

    KERNELS = {"phaseA": 0, "spmv1": 1, "phaseB": 2, "spmv2": 3, "iteration": 4, "copy": 5,
               "spmv_bare": 6, "final": 7}

    def time_kernel(self, kernel: str, reps: int = 50) -> float:
        """Average duration (ms) of one launch of an iteration kernel, timed
        with HIP events on the library's stream.  Overwrites solver state."""
        ms = ctypes.c_double()
        L.check(L.load().pbicgstab_time_kernel(self._h, self.KERNELS[kernel], reps,
                                               ctypes.byref(ms), _stream()))
        return ms.value

    def device_bytes(self) -> int:
        b = ctypes.c_int64()
        L.check(L.load().pbicgstab_info(self._h, None, None, ctypes.byref(b)))
        return b.value

    def close(self):
        if self._h:
            torch.cuda.synchronize()
            L.load().pbicgstab_destroy(self._h)
            self._h = None
        self.workspace = None           # the handle no longer uses it

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SparseSolve(torch.autograd.Function):
    """x = A(values)^-1 b, differentiable in ``values`` (the stored entries,
    in the solver's value layout) and ``b``.

    backward solves the adjoint system A^T lambda = dL/dx with the same
    pipelined kernels on the transposed layout and returns
    dL/db = lambda, dL/dvalues = -lambda_i x_j on the pattern."""

    @staticmethod
    def forward(ctx, values, b, solver: Solver, opts: dict):
        if values is not None:
            solver.update_values(values)
        x, st = solver.solve(b, **opts)
        if st["status"] != 0:
            raise RuntimeError(f"forward solve did not converge: {st}")
        ctx.solver = solver
        ctx.opts = opts
        ctx.has_values = values is not None
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        opts = dict(ctx.opts)
        opts["transpose"] = not opts.get("transpose", False)
        lam, st = ctx.solver.solve(gx.contiguous().to(torch.float64), **opts)
        if st["status"] != 0:
            raise RuntimeError(f"adjoint solve did not converge: {st}")
        gvals = ctx.solver.grad_values(lam, x) if ctx.has_values else None
        return gvals, lam, None, None


class KappaSolve(torch.autograd.Function):
    """u = A(kappa)^-1 b for the coefficient-field operator of a DIA5 solver,
    differentiable in kappa (node values) and b."""

    @staticmethod
    def forward(ctx, kappa, b, solver: Solver, opts: dict, conv=(1.0, 0.0), h=None):
        solver.assemble_kappa(kappa.detach(), conv, h)
        x, st = solver.solve(b, **opts)
        if st["status"] != 0:
            raise RuntimeError(f"forward solve did not converge: {st}")
        ctx.solver = solver
        ctx.opts = opts
        ctx.shape = kappa.shape
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        opts = dict(ctx.opts)
        opts["transpose"] = True
        lam, st = ctx.solver.solve(gx.contiguous().to(torch.float64), **opts)
        if st["status"] != 0:
            raise RuntimeError(f"adjoint solve did not converge: {st}")
        gk = ctx.solver.kappa_grad(lam, x).reshape(ctx.shape)
        return gk, lam, None, None, None, None
