"""The plane-marching 3D 7-point product (one work item = a segment of one
grid plane over several consecutive planes, the plane below, the plane and
the plane above kept in registers) on awkward grid shapes: a single plane,
planes shorter than one segment, segments cut by the end of a plane, nx not
a multiple of the 16-byte chunk (those grids use the row-wise kernels), and
forced chunk lengths of one and three planes.  Whole solves must agree bit
for bit with the CSR form of the same operator and with the structured
product that does not march (PBCG_MARCH3D=0); with the phase kernels in
row order (PBCG_MARCH_PHASE=0), the order a CSR matrix has.  The phase
kernels' own plane march (the default for 3D grids with FP32 storage: fused
products with the planes below and above in registers) is checked bit for
bit against the separate products marching in the same order, and against
row order within a tolerance (only the dot products' summation order
differs)."""

import numpy as np
import pytest

from gpu_util import dev, host, solver_env
from workloads.generators import Stencil, _problem_from_stencil

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Solver():
    from paper_1809_01948_amd.solver import Solver as S
    return S


def _problem(dims, seed):
    coef = {"C": 6.0, "E": -1.0 + 1.5, "W": -1.0 - 1.5, "N": -1.0 + 0.75, "S": -1.0 - 0.75,
            "U": -1.0 + 0.25, "D": -1.0 - 0.25}
    st = Stencil("3d7", dims, coef)
    n = int(np.prod(dims))
    b = np.random.default_rng(seed).uniform(-1.0, 1.0, n)
    return _problem_from_stencil(f"box{dims}", st, b, None, "jacobi", 0.0, 30, 7, True)


def _solve(Solver, p, form, precision="fp64", maxit=30, **env):
    with solver_env(**env):
        S = Solver.from_problem(p, form=form, precision=precision, precond="jacobi")
    x, st = S.solve(dev(p.b), tol=0.0, maxit=maxit, rr_period=7)
    out = (host(x), st["iterations"], st["replacements"], host(S.get_vector("v")))
    S.close()
    return out


SHAPES = [(6, 5, 1), (10, 3, 7), (34, 33, 2), (200, 1, 3), (2, 2, 40), (7, 5, 9), (64, 30, 17),
          (20, 20, 20)]


@pytest.mark.parametrize("dims", SHAPES, ids=["x".join(map(str, d)) for d in SHAPES])
def test_march_equals_csr_and_rowwise(Solver, dims):
    p = _problem(dims, seed=sum(dims))
    ref = _solve(Solver, p, "csr")
    assert ref[1] > 0
    for env in ({}, {"PBCG_MARCH3D": 0}, {"PBCG_MARCH_ZLEN": 1}, {"PBCG_MARCH_ZLEN": 3}):
        got = _solve(Solver, p, "stencil", PBCG_FUSE=0, PBCG_MARCH_PHASE=0, **env)
        assert got[1:3] == ref[1:3], env
        assert np.array_equal(got[0], ref[0]), env
        assert np.array_equal(got[3], ref[3]), env


@pytest.mark.parametrize("dims", [(8, 6, 5), (36, 7, 11)], ids=["8x6x5", "36x7x11"])
def test_march_fp32_storage(Solver, dims):
    """FP32 storage (4 rows per 16-byte chunk): the separate-product iteration
    with the marching product against the one without it."""
    p = _problem(dims, seed=3)
    ref = _solve(Solver, p, "stencil", "mixed", PBCG_FUSE=0, PBCG_MARCH3D=0, PBCG_MARCH_PHASE=0)
    for env in ({}, {"PBCG_MARCH_ZLEN": 2}):
        got = _solve(Solver, p, "stencil", "mixed", PBCG_FUSE=0, PBCG_MARCH_PHASE=0, **env)
        assert got[1:3] == ref[1:3], env
        assert np.array_equal(got[0], ref[0]), env
        assert np.array_equal(got[3], ref[3]), env


PHASE_SHAPES = [(8, 6, 5), (36, 7, 11), (4, 4, 30), (64, 30, 17), (200, 2, 3)]


@pytest.mark.parametrize("dims", PHASE_SHAPES, ids=["x".join(map(str, d)) for d in PHASE_SHAPES])
def test_phase_march_fused_equals_separate(Solver, dims):
    """FP32 storage, where the 3D products are fused: the phase kernels with
    the planes in registers against separate products, both marching."""
    p = _problem(dims, seed=5)
    ref = _solve(Solver, p, "stencil", "mixed", PBCG_FUSE=0)
    for env in ({}, {"PBCG_NBLK": 8}):
        got = _solve(Solver, p, "stencil", "mixed", PBCG_FUSE=1, **env)
        sep = ref if not env else _solve(Solver, p, "stencil", "mixed", PBCG_FUSE=0, **env)
        assert got[1:3] == sep[1:3], env
        assert np.array_equal(got[0], sep[0]), env
        assert np.array_equal(got[3], sep[3]), env


@pytest.mark.parametrize("precision", ["mixed"])
def test_phase_march_close_to_row_order(Solver, precision):
    """Eight iterations, replacement at the seventh: the dot products' summation
    order differs, and on this non-normal operator such differences grow from
    iteration to iteration (after 30 iterations: 3e-3 relative in x, the FP32
    vectors rounding the scalars' differences)."""
    p = _problem((40, 24, 20), seed=7)
    a = _solve(Solver, p, "stencil", precision, maxit=8, PBCG_MARCH_PHASE=1)
    b = _solve(Solver, p, "stencil", precision, maxit=8, PBCG_MARCH_PHASE=0)
    assert a[1] == b[1] == 8 and a[2] == b[2] == 1
    tol = 1e-5
    assert np.linalg.norm(a[0] - b[0]) <= tol * np.linalg.norm(b[0])
