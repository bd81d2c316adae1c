"""Seeded problem generators (input data only; no solver arithmetic).

Every generator returns a :class:`Problem` whose arrays are plain NumPy data:
a CSR matrix (int32 ``rowptr``/``col``, float64 ``val``), optionally a
constant-coefficient :class:`Stencil` or a DIA5 coefficient array describing
the same matrix, the right-hand side ``b``, the initial guess ``x0`` and, where
the problem fixes it, the exact solution.

Grid ordering is lexicographic everywhere: ``p = ix + nx*iy (+ nx*ny*iz)``.
Neighbour names: W/E are ``p-1``/``p+1``, S/N are ``p-nx``/``p+nx`` and D/U
are ``p-nx*ny``/``p+nx*ny``.  CSR rows list their columns in ascending order,
so a stencil row is stored as (D,) S, W, C, E, N (, U).  Dirichlet boundaries:
a neighbour outside the grid has no matrix entry.

The test problems follow the paper's model problems (Section 4, Table
``tab:specs``: second-order central finite differences on a regular grid,
``b = A x_ex``, ``x0 = 0``) and the five workload shapes of the pipelined
BiCGStab benchmark (2D convection-diffusion 32^2, 2D Poisson 1000^2, 3D
convection-diffusion 200^3, random banded N=2e6, coefficient-field problem
2048^2).  The exact recipes are stated in each docstring.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# -----------------------------------------------------------------------------
# containers
# -----------------------------------------------------------------------------

_NEIGH_2D = ("S", "W", "C", "E", "N")             # ascending column order
_NEIGH_3D = ("D", "S", "W", "C", "E", "N", "U")


@dataclass
class Stencil:
    """Constant-coefficient 5-point (2D) or 7-point (3D) stencil on a grid."""

    kind: str                       # "2d5" or "3d7"
    dims: tuple                     # (nx, ny) or (nx, ny, nz)
    coef: dict                      # neighbour name -> float64 coefficient

    @property
    def n(self) -> int:
        return int(np.prod(self.dims))

    def names(self):
        return _NEIGH_2D if self.kind == "2d5" else _NEIGH_3D

    def offsets(self):
        nx = self.dims[0]
        if self.kind == "2d5":
            return (-nx, -1, 0, 1, nx)
        ny = self.dims[1]
        return (-nx * ny, -nx, -1, 0, 1, nx, nx * ny)

    def coef_vector(self):
        """Coefficients in ascending-column order as float64."""
        return np.array([self.coef[k] for k in self.names()], dtype=np.float64)


@dataclass
class Problem:
    name: str
    n: int
    b: np.ndarray
    x0: np.ndarray
    rowptr: Optional[np.ndarray] = None
    col: Optional[np.ndarray] = None
    val: Optional[np.ndarray] = None
    stencil: Optional[Stencil] = None
    dia5: Optional[np.ndarray] = None        # (5, N): S, W, C, E, N coefficients
    dims: Optional[tuple] = None
    x_exact: Optional[np.ndarray] = None
    precond: str = "none"                    # "none" | "jacobi"
    tol: float = 1e-10
    maxit: int = 10000
    rr_period: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return 0 if self.rowptr is None else int(self.rowptr[-1])

    def scipy_csr(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))


# -----------------------------------------------------------------------------
# grid helpers
# -----------------------------------------------------------------------------

def _grid_valid_masks(dims, names):
    """Boolean masks (one per neighbour name) telling whether that neighbour
    exists for each grid point."""
    n = int(np.prod(dims))
    p = np.arange(n, dtype=np.int64)
    nx = dims[0]
    ix = p % nx
    if len(dims) == 2:
        iy = p // nx
        ny = dims[1]
        iz = None
    else:
        ny = dims[1]
        iy = (p // nx) % ny
        iz = p // (nx * ny)
        nz = dims[2]
    masks = {}
    for k in names:
        if k == "C":
            masks[k] = np.ones(n, dtype=bool)
        elif k == "W":
            masks[k] = ix > 0
        elif k == "E":
            masks[k] = ix < nx - 1
        elif k == "S":
            masks[k] = iy > 0
        elif k == "N":
            masks[k] = iy < ny - 1
        elif k == "D":
            masks[k] = iz > 0
        elif k == "U":
            masks[k] = iz < nz - 1
    return masks


def _offset_of(dims, name):
    nx = dims[0]
    ny = dims[1] if len(dims) > 1 else 1
    return {"C": 0, "W": -1, "E": 1, "S": -nx, "N": nx,
            "D": -nx * ny, "U": nx * ny}[name]


def _assemble_csr(dims, names, coef_arrays):
    """CSR from per-neighbour coefficient arrays (ascending column order)."""
    n = int(np.prod(dims))
    masks = _grid_valid_masks(dims, names)
    p = np.arange(n, dtype=np.int64)
    valid = np.stack([masks[k] for k in names], axis=1)
    cols = np.stack([p + _offset_of(dims, k) for k in names], axis=1)
    vals = np.stack([np.broadcast_to(np.asarray(coef_arrays[k], dtype=np.float64), (n,))
                     for k in names], axis=1)
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = cols[valid].astype(np.int32)
    val = np.ascontiguousarray(vals[valid])
    return rowptr.astype(np.int32), col, val


def stencil_to_csr(st: Stencil):
    """CSR arrays (rowptr int32, col int32, val float64) of a stencil."""
    return _assemble_csr(st.dims, st.names(), st.coef)


def dia5_to_csr(dims, dia5):
    """CSR arrays of a 2D five-diagonal matrix given as (5, N) S, W, C, E, N."""
    arrays = {k: dia5[i] for i, k in enumerate(_NEIGH_2D)}
    return _assemble_csr(tuple(dims), _NEIGH_2D, arrays)


def _stencil_times_constant(st: Stencil, c: float):
    """b = A (c * ones) for a stencil, summed in ascending column order."""
    masks = _grid_valid_masks(st.dims, st.names())
    b = np.zeros(st.n, dtype=np.float64)
    for k in st.names():
        b += np.where(masks[k], st.coef[k] * c, 0.0)
    return b


def _problem_from_stencil(name, st, b, x_exact, precond, tol, maxit, rr_period,
                          with_csr):
    n = st.n
    prob = Problem(name=name, n=n, b=b, x0=np.zeros(n), stencil=st, dims=st.dims,
                   x_exact=x_exact, precond=precond, tol=tol, maxit=maxit,
                   rr_period=rr_period)
    if with_csr:
        prob.rowptr, prob.col, prob.val = stencil_to_csr(st)
    return prob


# -----------------------------------------------------------------------------
# the five benchmark workloads
# -----------------------------------------------------------------------------

def convdiff2d_c1(n: int = 32, conv=(1.0, 1.0), with_csr: bool = True) -> Problem:
    """2D convection-diffusion ``-Lap u + (c_x, c_y).grad u`` on the unit square.

    n x n interior points, h = 1/(n+1), homogeneous Dirichlet boundary,
    second-order central differences, the whole row scaled by h^2:
    centre 4, E/W ``-1 +/- c_x h/2``, N/S ``-1 +/- c_y h/2``.
    ``b = A * ones`` (so the exact solution is the all-ones vector),
    ``x0 = 0``, no preconditioner, tolerance 1e-10.
    """
    h = 1.0 / (n + 1)
    cx, cy = conv
    coef = {"C": 4.0, "E": -1.0 + cx * h / 2.0, "W": -1.0 - cx * h / 2.0,
            "N": -1.0 + cy * h / 2.0, "S": -1.0 - cy * h / 2.0}
    st = Stencil("2d5", (n, n), coef)
    b = _stencil_times_constant(st, 1.0)
    return _problem_from_stencil(f"convdiff2d_{n}", st, b, np.ones(n * n), "none",
                                 1e-10, 2000, 0, with_csr)


def poisson2d_c2(n: int = 1000, seed: int = 2, with_csr: bool = True) -> Problem:
    """2D Poisson, 5-point stencil [4; -1, -1, -1, -1] (h^2-scaled), n x n grid.

    ``b = default_rng(seed).uniform(-1, 1, N)``, ``x0 = 0``, Jacobi
    preconditioner (the constant diagonal 4, i.e. M^-1 = 1/4 exactly),
    tolerance 1e-10, residual replacement period 50.
    """
    coef = {"C": 4.0, "E": -1.0, "W": -1.0, "N": -1.0, "S": -1.0}
    st = Stencil("2d5", (n, n), coef)
    b = np.random.default_rng(seed).uniform(-1.0, 1.0, n * n)
    return _problem_from_stencil(f"poisson2d_{n}", st, b, None, "jacobi",
                                 1e-10, 20000, 50, with_csr)


def convdiff3d_c3(n: int = 200, conv=(10.0, 5.0, 1.0), with_csr: bool = False) -> Problem:
    """3D convection-diffusion ``-Lap u + c.grad u`` on an n^3 grid, h = 1.

    Central differences with unit cell spacing: centre 6, E/W ``-1 +/- c_x/2``,
    N/S ``-1 +/- c_y/2``, U/D ``-1 +/- c_z/2``; for c = (10, 5, 1) this is
    6; 4/-6; 1.5/-3.5; -0.5/-1.5 (all exact in FP32).  Following the paper's
    convention ``b = A x_ex`` with ``x_ex = ones/sqrt(N)``, ``x0 = 0``,
    Jacobi (the constant diagonal 6), tolerance 1e-10, replacement period 50.
    """
    cx, cy, cz = conv
    coef = {"C": 6.0, "E": -1.0 + cx / 2.0, "W": -1.0 - cx / 2.0,
            "N": -1.0 + cy / 2.0, "S": -1.0 - cy / 2.0,
            "U": -1.0 + cz / 2.0, "D": -1.0 - cz / 2.0}
    st = Stencil("3d7", (n, n, n), coef)
    N = n ** 3
    c = 1.0 / np.sqrt(N)
    b = _stencil_times_constant(st, c)
    return _problem_from_stencil(f"convdiff3d_{n}", st, b, np.full(N, c), "jacobi",
                                 1e-10, 20000, 50, with_csr)


_C4_CHUNK = 1 << 18   # rows generated per chunk (part of the recipe: fixes the draw order)


def random_banded_c4(N: int = 2_000_000, nnz_row: int = 27, band: int = 5000,
                     seed: int = 4, xseed: int = 40) -> Problem:
    """Random unsymmetric banded matrix, diagonally dominant by a factor 1.2.

    Row i holds its diagonal plus ``nnz_row - 1`` distinct off-diagonal
    columns from ``[max(0, i-band), min(N-1, i+band)] \\ {i}``.  The distinct
    set is drawn with one generator ``default_rng(seed)`` in chunks of
    ``_C4_CHUNK`` rows: ``k = nnz_row-1`` integers in ``[0, W-k]`` (W = window
    size without i) are sorted and ``0..k-1`` is added, giving k distinct
    sorted window positions.  Off-diagonal values are standard normal draws
    from the same generator, rounded to FP32; the diagonal is
    ``fl32(1.2 * sum |a_ij|)``.  Every stored value is therefore exact in
    FP32.  ``x_ex = default_rng(xseed).uniform(-1, 1, N)``, ``b = A x_ex``,
    ``x0 = 0``, Jacobi, tolerance 1e-10.
    """
    import scipy.sparse as sp

    k = nnz_row - 1
    rng = np.random.default_rng(seed)
    rowptr = np.arange(N + 1, dtype=np.int64) * nnz_row
    col = np.empty(N * nnz_row, dtype=np.int32)
    val = np.empty(N * nnz_row, dtype=np.float64)
    for r0 in range(0, N, _C4_CHUNK):
        r1 = min(N, r0 + _C4_CHUNK)
        rows = np.arange(r0, r1, dtype=np.int64)
        lo = np.maximum(0, rows - band)
        hi = np.minimum(N - 1, rows + band)
        W = hi - lo                      # window size excluding the row itself
        if np.any(W < k):
            raise ValueError("band too narrow for the requested nnz per row")
        draws = rng.integers(0, (W - k + 1)[:, None], size=(r1 - r0, k))
        draws.sort(axis=1)
        pos = draws + np.arange(k)[None, :]
        c = lo[:, None] + pos
        c = c + (c >= rows[:, None])     # skip the diagonal position
        offv = rng.standard_normal((r1 - r0, k)).astype(np.float32).astype(np.float64)
        diag = (1.2 * np.abs(offv).sum(axis=1)).astype(np.float32).astype(np.float64)
        allc = np.concatenate([c, rows[:, None]], axis=1)
        allv = np.concatenate([offv, diag[:, None]], axis=1)
        order = np.argsort(allc, axis=1, kind="stable")
        allc = np.take_along_axis(allc, order, axis=1)
        allv = np.take_along_axis(allv, order, axis=1)
        col[r0 * nnz_row:r1 * nnz_row] = allc.reshape(-1)
        val[r0 * nnz_row:r1 * nnz_row] = allv.reshape(-1)
    x_ex = np.random.default_rng(xseed).uniform(-1.0, 1.0, N)
    A = sp.csr_matrix((val, col, rowptr), shape=(N, N))
    b = A @ x_ex
    return Problem(name=f"random_banded_{N}", n=N, b=b, x0=np.zeros(N),
                   rowptr=rowptr.astype(np.int32), col=col, val=val,
                   x_exact=x_ex, precond="jacobi", tol=1e-10, maxit=5000,
                   rr_period=50)


def kappa_field_c5(n: int = 2048, seed: int = 5, sigma: float = 32.0,
                   amp: float = 0.5) -> np.ndarray:
    """Smooth log-normal coefficient field on an n x n grid.

    Standard normal draws from ``default_rng(seed)`` are filtered with a
    periodic Gaussian of standard deviation ``sigma`` cells (multiplication
    by ``exp(-2 pi^2 sigma^2 |f|^2)`` in the FFT domain), standardised to
    zero mean and unit variance, and exponentiated: ``kappa = exp(amp*g)``.
    Returned with shape (n, n) indexed ``[iy, ix]``.
    """
    g = np.random.default_rng(seed).standard_normal((n, n))
    f = np.fft.fftfreq(n)
    fy, fx = np.meshgrid(f, f, indexing="ij")
    filt = np.exp(-2.0 * np.pi ** 2 * sigma ** 2 * (fx ** 2 + fy ** 2))
    gs = np.real(np.fft.ifft2(np.fft.fft2(g) * filt))
    gs = (gs - gs.mean()) / gs.std()
    return np.exp(amp * gs)


def dia5_from_kappa(kappa: np.ndarray, h: float, conv=(1.0, 0.0)) -> np.ndarray:
    """DIA5 coefficients of ``-div(kappa grad u) + c.grad u`` (h^2-scaled).

    Face coefficients are the arithmetic mean of the two node values; a face
    on the domain boundary takes the node's own value.  Row p:
    centre ``sum of its four face values``, E ``-k_e + c_x h/2``,
    W ``-k_w - c_x h/2``, N ``-k_n + c_y h/2``, S ``-k_s - c_y h/2``; a
    neighbour outside the grid gets coefficient 0 (no entry).  Returns a
    (5, N) float64 array in the order S, W, C, E, N.
    """
    ny, nx = kappa.shape
    k = kappa
    ke = k.copy()
    ke[:, :-1] = 0.5 * (k[:, :-1] + k[:, 1:])
    kw = k.copy()
    kw[:, 1:] = 0.5 * (k[:, 1:] + k[:, :-1])
    kn = k.copy()
    kn[:-1, :] = 0.5 * (k[:-1, :] + k[1:, :])
    ks = k.copy()
    ks[1:, :] = 0.5 * (k[1:, :] + k[:-1, :])
    cx, cy = conv
    C = ke + kw + kn + ks
    E = -ke + cx * h / 2.0
    W = -kw - cx * h / 2.0
    Nn = -kn + cy * h / 2.0
    S = -ks - cy * h / 2.0
    E[:, -1] = 0.0
    W[:, 0] = 0.0
    Nn[-1, :] = 0.0
    S[0, :] = 0.0
    return np.stack([S.reshape(-1), W.reshape(-1), C.reshape(-1), E.reshape(-1),
                     Nn.reshape(-1)]).astype(np.float64)


def inverse_problem_c5(n: int = 2048, seed: int = 5, target_seed: int = 55,
                       sigma: float = 32.0, amp: float = 0.5,
                       with_csr: bool = False) -> Problem:
    """Coefficient-field problem ``-div(kappa grad u) + (1,0).grad u = 1``.

    n x n interior grid on the unit square, h = 1/(n+1), ``b = h^2 ones``,
    ``x0 = 0``, Jacobi, tolerance 1e-10.  ``extra`` carries the current field
    (``kappa``, from ``seed``) and the target field (``kappa_target``, from
    ``target_seed``); the target state ``u_target`` is the forward solution
    for ``kappa_target`` and is produced by whichever solver the caller uses.
    The loss is ``||u - u_target||^2``.
    """
    h = 1.0 / (n + 1)
    kap = kappa_field_c5(n, seed, sigma, amp)
    kap_t = kappa_field_c5(n, target_seed, sigma, amp)
    dia = dia5_from_kappa(kap, h)
    N = n * n
    prob = Problem(name=f"kappa2d_{n}", n=N, b=np.full(N, h * h), x0=np.zeros(N),
                   dia5=dia, dims=(n, n), precond="jacobi", tol=1e-10, maxit=20000,
                   rr_period=50,
                   extra={"kappa": kap, "kappa_target": kap_t, "h": h})
    if with_csr:
        prob.rowptr, prob.col, prob.val = dia5_to_csr((n, n), dia)
    return prob


# -----------------------------------------------------------------------------
# the paper's own model problems (Table tab:specs) and tiny systems
# -----------------------------------------------------------------------------

def _norm2_estimate(rowptr, col, val, n, iters=200, seed=0):
    """||A||_2 estimated by power iteration on A^T A (problem set-up only).
    Norms are correctly rounded sums (math.fsum), so the estimate -- and the
    normalised matrix -- is the same bits whatever BLAS threading is used."""
    import math

    import scipy.sparse as sp
    A = sp.csr_matrix((val, col, rowptr), shape=(n, n))
    v = np.random.default_rng(seed).standard_normal(n)
    v /= math.sqrt(math.fsum(v * v))
    s = 0.0
    for _ in range(iters):
        w = A.T @ (A @ v)
        s = math.sqrt(math.fsum(w * w))
        v = w / s
    return float(np.sqrt(s))


def tp2_unsymmetric(n: int = 1000, eps: float = 1e-3, normalize: bool = True) -> Problem:
    """Unsymmetric 2D 5-point stencil: centre 4, W/S -1, E/N (the entries
    above the diagonal) -1+eps; ``b = A ones/sqrt(N)``, ``x0 = 0``, no
    preconditioner.  With ``normalize`` the matrix is divided by a
    power-iteration estimate of its 2-norm (Section 4 rescales ||A||_2 = 1)."""
    coef = {"C": 4.0, "E": -1.0 + eps, "W": -1.0, "N": -1.0 + eps, "S": -1.0}
    st = Stencil("2d5", (n, n), coef)
    rowptr, col, val = stencil_to_csr(st)
    if normalize:
        s = _norm2_estimate(rowptr, col, val, n * n)
        val = val / s
        st = Stencil("2d5", (n, n), {k: v / s for k, v in coef.items()})
    N = n * n
    c = 1.0 / np.sqrt(N)
    b = _stencil_times_constant(st, c)
    return Problem(name=f"tp2_{n}", n=N, b=b, x0=np.zeros(N), rowptr=rowptr, col=col,
                   val=val, stencil=st, dims=(n, n), x_exact=np.full(N, c),
                   precond="none", tol=1e-13, maxit=5000, rr_period=100)


def tp3_helmholtz(n: int = 500, eps: float = 5e-4, normalize: bool = True) -> Problem:
    """Indefinite 2D Helmholtz-type stencil: centre 4-eps, neighbours -1;
    ``b = A ones/sqrt(N)``, ``x0 = 0``, no preconditioner (the timed runs of
    the paper use none)."""
    coef = {"C": 4.0 - eps, "E": -1.0, "W": -1.0, "N": -1.0, "S": -1.0}
    st = Stencil("2d5", (n, n), coef)
    rowptr, col, val = stencil_to_csr(st)
    if normalize:
        s = _norm2_estimate(rowptr, col, val, n * n)
        val = val / s
        st = Stencil("2d5", (n, n), {k: v / s for k, v in coef.items()})
    N = n * n
    c = 1.0 / np.sqrt(N)
    b = _stencil_times_constant(st, c)
    return Problem(name=f"tp3_{n}", n=N, b=b, x0=np.zeros(N), rowptr=rowptr, col=col,
                   val=val, stencil=st, dims=(n, n), x_exact=np.full(N, c),
                   precond="none", tol=1e-8, maxit=20000, rr_period=200)


def random_dense_system(n: int, seed: int, shift: float = 0.0, integer: bool = False) -> Problem:
    """A small dense unsymmetric system stored as CSR (all entries present).

    Entries are standard normal (or integers in [-3, 3] when ``integer``),
    plus ``shift`` on the diagonal; ``x_ex = default_rng(seed+1).uniform(-1,
    1, n)`` (integers in [-2, 2] when ``integer``), ``b = A x_ex``."""
    rng = np.random.default_rng(seed)
    if integer:
        M = rng.integers(-3, 4, size=(n, n)).astype(np.float64)
        x_ex = np.random.default_rng(seed + 1).integers(-2, 3, size=n).astype(np.float64)
    else:
        M = rng.standard_normal((n, n))
        x_ex = np.random.default_rng(seed + 1).uniform(-1.0, 1.0, n)
    M = M + shift * np.eye(n)
    rowptr = (np.arange(n + 1) * n).astype(np.int32)
    col = np.tile(np.arange(n, dtype=np.int32), n)
    val = M.reshape(-1).copy()
    b = M @ x_ex
    return Problem(name=f"dense_{n}_{seed}", n=n, b=b, x0=np.zeros(n), rowptr=rowptr,
                   col=col, val=val, x_exact=x_ex, precond="none", tol=1e-12,
                   maxit=200, rr_period=0)
