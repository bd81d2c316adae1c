"""Helpers shared by the GPU tests (host<->device copies, oracle set-up)."""

import contextlib
import os

import numpy as np
import scipy.sparse as sp
import torch

from oracle import Float64Ops


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def oracle_ops(prob, precond=None):
    """Oracle arithmetic for a workloads.Problem (its CSR and Jacobi diagonal)."""
    A = prob.scipy_csr()
    pc = prob.precond if precond is None else precond
    dinv = 1.0 / A.diagonal() if pc == "jacobi" else None
    return A, Float64Ops(A, dinv)


def history_buffer(rows):
    return torch.zeros(4 * rows, dtype=torch.float64, device="cuda")


def split_history(hist, its):
    h = host(hist).reshape(-1, 4)[:its]
    return h[:, 0], h[:, 1], h[:, 2], h[:, 3]


def rel(a, b):
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def csr_T(A):
    return sp.csr_matrix(A.T)


@contextlib.contextmanager
def solver_env(**values):
    """Tuning switches that a solver reads when it is created (PBCG_FUSE,
    PBCG_NBLK, ...), set for the duration of the block."""
    old = {k: os.environ.get(k) for k in values}
    os.environ.update({k: str(v) for k, v in values.items()})
    try:
        yield
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
