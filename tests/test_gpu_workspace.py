"""The ownership model of the C ABI on the GPU: every device byte of a
handle lives in the caller's workspace (a torch uint8 tensor), whose size
pbicgstab_workspace_bytes gives; too small a workspace is rejected; CSR and
DIA5 inputs are device arrays, checked after they have been read."""

import numpy as np
import pytest
import torch

from gpu_util import dev, host
from workloads import convdiff2d_c1, inverse_problem_c5, random_banded_c4

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mod():
    import paper_1809_01948_amd.solver as m
    return m


def _csr_width(p, transpose):
    w = int(np.max(np.diff(p.rowptr)))
    if transpose:
        w = max(w, int(np.max(np.bincount(p.col, minlength=p.n))))
    return w


@pytest.mark.parametrize("form", ["csr", "stencil", "dia5"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_exact_workspace_and_too_small(mod, form, precision):
    from paper_1809_01948_amd import PbcgError
    p = inverse_problem_c5(40, sigma=2.0, with_csr=True) if form == "dia5" else convdiff2d_c1(24)
    pc = "jacobi"
    if form == "csr":
        nb = mod.workspace_bytes("csr", p.n, len(p.col), _csr_width(p, True), precision, pc)
        make = lambda ws: mod.Solver.from_csr(p.rowptr, p.col, p.val, precision, pc,
                                              workspace=ws)
    elif form == "stencil":
        nb = mod.workspace_bytes("2d5", p.n, 0, 0, precision, pc)
        make = lambda ws: mod.Solver.from_stencil("2d5", p.dims, p.stencil.coef_vector(),
                                                  precision, pc, workspace=ws)
    else:
        nb = mod.workspace_bytes("dia5", p.n, 0, 0, precision, pc)
        make = lambda ws: mod.Solver.from_stencil("dia5", p.dims, p.dia5, precision, pc,
                                                  workspace=ws)
    with pytest.raises(PbcgError) as e:
        make(torch.empty(nb // 2, dtype=torch.uint8, device="cuda"))
    assert e.value.code == -4 and "workspace too small" in str(e.value)
    ws = torch.full((nb,), 0xAB, dtype=torch.uint8, device="cuda")   # not zeroed by the caller
    S = make(ws)
    assert S.device_bytes() <= nb
    x, st = S.solve(dev(p.b), tol=1e-8, maxit=40, rr_period=10)
    assert st["iterations"] >= 30, st
    # the same solve with a workspace the Solver sizes itself: bitwise the same
    S2 = make(None)
    x2, st2 = S2.solve(dev(p.b), tol=1e-8, maxit=40, rr_period=10)
    assert st2["iterations"] == st["iterations"] and st2["status"] == st["status"]
    assert np.array_equal(host(x), host(x2))
    # the transposed layout fits the reserved space (built on first use)
    y = S.apply(dev(p.b), transpose=True)
    A = p.scipy_csr()
    if precision == "fp64":
        assert np.allclose(host(y), A.T @ p.b, rtol=1e-13, atol=1e-15)
    S.close()
    S2.close()


def test_transpose_needs_reserved_space(mod):
    from paper_1809_01948_amd import PbcgError
    p = convdiff2d_c1(16)
    w = _csr_width(p, False)
    nb = mod.workspace_bytes("csr", p.n, len(p.col), w, "fp64", "none", with_transpose=False)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    S = mod.Solver.from_csr(p.rowptr, p.col, p.val, "fp64", "none", with_transpose=False,
                            workspace=ws)
    x, st = S.solve(dev(p.b), tol=1e-10, maxit=500)
    assert st["status"] == 0
    with pytest.raises(PbcgError) as e:
        S.apply(dev(p.b), transpose=True)
    assert e.value.code == -4
    S.close()


@pytest.mark.parametrize("case,msg", [
    ("rowptr0", "rowptr[0]"),
    ("decreasing", "nondecreasing"),
    ("col", "column index"),
])
def test_malformed_device_csr_is_rejected(mod, case, msg):
    from paper_1809_01948_amd import PbcgError
    rowptr, col, val = [0, 1, 2], [0, 1], [1.0, 2.0]
    if case == "rowptr0":
        rowptr = [1, 1, 2]
    elif case == "decreasing":
        rowptr, col, val = [0, 2, 1, 2], [0, 1], [1.0, 2.0]
    elif case == "col":
        col = [0, 5]
    with pytest.raises(PbcgError) as e:
        mod.Solver.from_csr(np.array(rowptr), np.array(col), np.array(val), "fp64", "none",
                            with_transpose=False)
    assert e.value.code == -1 and msg in str(e.value)


def test_large_sliced_ell_workspace(mod):
    """The 2e5-row banded random matrix (27 entries per row): the workspace
    bound from the longest row and column holds both layouts."""
    p = random_banded_c4(200_000, band=500)
    S = mod.Solver.from_problem(p, form="csr")
    x, st = S.solve(dev(p.b), tol=1e-10, maxit=200, rr_period=50)
    assert st["status"] == 0
    lam = S.apply(dev(p.b), transpose=True)
    A = p.scipy_csr()
    assert np.allclose(host(lam), A.T @ p.b, rtol=1e-13, atol=1e-13)
    assert S.device_bytes() <= S.workspace.numel()
    S.close()
