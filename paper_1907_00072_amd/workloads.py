"""Seeded synthetic workloads: CSR matrices and vectors.

This module only *builds inputs*.  It holds none of the solver's arithmetic
(no polynomial, no orthogonalisation, no Krylov step); the CPU oracle and the
HIP path both consume the arrays it returns, and nothing else is shared
between them.

Matrices
--------
* Finite-difference convection-diffusion  -eps*lap(u) + w.grad(u)  on the unit
  square / cube, the model problem family of the paper's parallel results
  (Section VI), discretised here with central differences instead of the
  paper's Firedrake P1 elements (those matrices are not available).
  Reading used: eps = 1/Pe; N interior points per axis; h = 1/(N+1);
  lexicographic numbering with x fastest; homogeneous Dirichlet boundary, so
  neighbours outside the grid are dropped (not stored).  The operator is
  scaled by h^2/eps, giving diagonal 2k (k = number of dimensions) and, along
  axis i, the coefficient -1 + P_i on the +x_i neighbour and -1 - P_i on the
  -x_i neighbour, with mesh Peclet number P_i = w_i * h * Pe / 2.
* 27-point random stencil: diagonal 30, every off-diagonal -1 + U(-0.3, 0.3),
  the perturbations drawn in CSR order (rows ascending, columns ascending,
  diagonal skipped).
* BiDiag1 / BiDiag2 (Section IV): upper bidiagonal test matrices with a known
  spectrum.
* The unscaled 5-point Laplacian (4, -1) on a 201 x 201 interior grid
  (Section V, n = 40401), eigenvalues in (0, 8).
* Recirculating-flow convection-diffusion (Section VI's second example):
  -eps*lap(u) + w.grad(u) = 0 on [-1, 1]^2 with w = (2y(1-x^2), -2x(1-y^2)),
  u = 1 on the boundary x = 1 and 0 on the others; central differences on an
  N x N interior grid (h = 2/(N+1)), scaled by h^2/eps, so the diagonal is 4
  and the neighbours along axis a carry -1 +- w_a(x, y) h / (2 eps) at the
  row's own grid point; the boundary values go to the right-hand side.

Every CSR array is returned as numpy ``int32`` row_ptr / col_ind (columns
sorted ascending inside each row) and ``float64`` values.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "CSR", "Problem", "convection_diffusion", "stencil27_random", "bidiag1",
    "bidiag2", "laplacian5", "uniform", "normal", "config", "CONFIG_NAMES",
    "random_csr", "recirculating_flow", "ILU_WORKLOAD", "EX1_WORKLOAD", "permutation",
    "permuted",
]


@dataclass
class CSR:
    """A square sparse matrix in CSR form (host numpy arrays)."""

    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col_ind: np.ndarray  # int32[nnz]
    vals: np.ndarray     # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals, self.col_ind, self.row_ptr),
                             shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        for i in range(self.n):
            lo, hi = self.row_ptr[i], self.row_ptr[i + 1]
            d[i, self.col_ind[lo:hi]] += self.vals[lo:hi]
        return d


@dataclass
class Problem:
    """One workload: matrix, right-hand side and solver parameters."""

    name: str
    A: CSR
    b: np.ndarray
    v0: np.ndarray
    m: int
    d: int
    tol: float
    x_star: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)


# ----------------------------------------------------------------- vectors
def uniform(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """n doubles ~ U(lo, hi) from numpy's PCG64 ``default_rng(seed)``."""
    return np.random.default_rng(seed).uniform(lo, hi, int(n))


def normal(n: int, seed: int) -> np.ndarray:
    """n doubles ~ N(0, 1) from numpy's PCG64 ``default_rng(seed)``."""
    return np.random.default_rng(seed).standard_normal(int(n))


# ---------------------------------------------------------------- matrices
def _stencil_csr(dims, offsets, coeffs):
    """CSR of a constant-coefficient stencil on an N^k grid, x fastest.

    ``offsets`` is a list of per-axis displacement tuples (dx, dy[, dz]) in
    ascending order of the resulting column offset; ``coeffs`` the matching
    values.  Neighbours that fall outside the grid are dropped.
    """
    dims = tuple(int(s) for s in dims)
    n = int(np.prod(dims))
    k = len(dims)
    strides = [1]
    for s in dims[:-1]:
        strides.append(strides[-1] * s)
    idx = np.arange(n, dtype=np.int64)
    coord = []
    for ax in range(k):
        coord.append((idx // strides[ax]) % dims[ax])
    ncol = len(offsets)
    valid = np.ones((n, ncol), dtype=bool)
    cols = np.empty((n, ncol), dtype=np.int32)
    for c, disp in enumerate(offsets):
        off = 0
        for ax in range(k):
            dd = disp[ax]
            if dd:
                nb = coord[ax] + dd
                valid[:, c] &= (nb >= 0) & (nb < dims[ax])
                off += dd * strides[ax]
        cols[:, c] = (idx + off).astype(np.int32, copy=False) if off else idx.astype(np.int32)
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    col_ind = cols[valid]
    vals = np.broadcast_to(np.asarray(coeffs, dtype=np.float64), (n, ncol))[valid]
    return CSR(n, row_ptr.astype(np.int32), np.ascontiguousarray(col_ind, dtype=np.int32),
               np.ascontiguousarray(vals, dtype=np.float64))


def convection_diffusion(N: int, dim: int, peclet: float, wind) -> CSR:
    """Central-difference convection-diffusion on an N^dim interior grid.

    Scaled by h^2/eps with eps = 1/Pe, so the diagonal is 2*dim and the
    +-x_i neighbours carry -1 +- P_i, P_i = wind_i * h * Pe / 2.
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    wind = tuple(float(w) for w in wind)
    if len(wind) != dim:
        raise ValueError("wind must have dim components")
    h = 1.0 / (N + 1)
    P = [w * h * peclet / 2.0 for w in wind]
    offsets, coeffs = [], []
    # ascending column offset: -z, -y, -x, 0, +x, +y, +z
    for ax in reversed(range(dim)):
        d = [0] * dim
        d[ax] = -1
        offsets.append(tuple(d))
        coeffs.append(-1.0 - P[ax])
    offsets.append(tuple([0] * dim))
    coeffs.append(2.0 * dim)
    for ax in range(dim):
        d = [0] * dim
        d[ax] = 1
        offsets.append(tuple(d))
        coeffs.append(-1.0 + P[ax])
    return _stencil_csr((N,) * dim, offsets, coeffs)


def recirculating_flow(N: int, eps: float = 1.0 / 200.0):
    """The recirculating-wind problem on an N x N interior grid: (A, b).

    Rows in lexicographic order, x fastest; column order per row -y, -x, 0,
    +x, +y.  b holds the boundary data u = 1 on x = 1 (zero source).
    """
    N = int(N)
    h = 2.0 / (N + 1)
    t = -1.0 + (np.arange(N) + 1) * h
    X, Y = np.meshgrid(t, t, indexing="xy")  # X[j, i] = x_i, Y[j, i] = y_j
    px = (2.0 * Y * (1.0 - X * X) * h / (2.0 * eps)).ravel()
    py = (-2.0 * X * (1.0 - Y * Y) * h / (2.0 * eps)).ravel()
    n = N * N
    ii = np.tile(np.arange(N), N)
    jj = np.repeat(np.arange(N), N)
    idx = np.arange(n, dtype=np.int64)
    # (row validity, column, value) per stencil slot, in ascending column order
    slots = [
        (jj > 0, idx - N, -1.0 - py),
        (ii > 0, idx - 1, -1.0 - px),
        (np.ones(n, bool), idx, np.full(n, 4.0)),
        (ii < N - 1, idx + 1, -1.0 + px),
        (jj < N - 1, idx + N, -1.0 + py),
    ]
    valid = np.stack([s[0] for s in slots], axis=1)
    cols = np.stack([s[1] for s in slots], axis=1)
    vals = np.stack([s[2] for s in slots], axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(valid.sum(axis=1), out=row_ptr[1:])
    A = CSR(n, row_ptr.astype(np.int32), cols[valid].astype(np.int32),
            np.ascontiguousarray(vals[valid], dtype=np.float64))
    b = np.where(ii == N - 1, 1.0 - px, 0.0)
    return A, b


def laplacian5(N: int = 201) -> CSR:
    """Unscaled 5-point Laplacian (diagonal 4, neighbours -1) on N x N."""
    offsets = [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)]
    return _stencil_csr((N, N), offsets, [-1.0, -1.0, 4.0, -1.0, -1.0])


def stencil27_random(N: int, seed: int = 3, diag: float = 30.0,
                     spread: float = 0.3) -> CSR:
    """27-point stencil on N^3: diagonal ``diag``, off-diagonals -1+U(-spread, spread)."""
    offsets = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                offsets.append((dx, dy, dz))
    coeffs = [0.0 if o == (0, 0, 0) else -1.0 for o in offsets]
    A = _stencil_csr((N, N, N), offsets, coeffs)
    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.row_ptr))
    off = A.col_ind.astype(np.int64) != rows
    pert = np.random.default_rng(seed).uniform(-spread, spread, int(off.sum()))
    vals = A.vals.copy()
    vals[off] += pert
    vals[~off] = diag
    A.vals = vals
    return A


def _bidiag(diag: np.ndarray, sup: float) -> CSR:
    n = diag.size
    counts = np.full(n, 2, dtype=np.int64)
    counts[-1] = 1
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), dtype=np.int32)
    val = np.empty(int(row_ptr[-1]))
    col[row_ptr[:-1]] = np.arange(n)
    val[row_ptr[:-1]] = diag
    col[row_ptr[:-2] + 1] = np.arange(1, n)
    val[row_ptr[:-2] + 1] = sup
    return CSR(n, row_ptr.astype(np.int32), col, val)


def bidiag1() -> CSR:
    """BiDiag1 (Section IV): n=2000, diagonal 1..2000, superdiagonal 0.05."""
    return _bidiag(np.arange(1, 2001, dtype=np.float64), 0.05)


def bidiag2() -> CSR:
    """BiDiag2 (Section IV): n=5000, diagonal 0.1..0.9, 1..4991, superdiagonal 0.2."""
    d = np.concatenate([np.arange(1, 10) / 10.0, np.arange(1, 4992, dtype=np.float64)])
    return _bidiag(d, 0.2)


def random_csr(n: int, per_row: int, seed: int, diag_shift: float = 0.0,
               ragged: bool = True) -> CSR:
    """Random nonsymmetric CSR with sorted columns and an always-present diagonal.

    Row lengths vary between 1 and ``per_row`` (when ``ragged``), values
    ~ U(-1, 1), diagonal += ``diag_shift``.  Used for tiles with ragged rows.
    """
    rng = np.random.default_rng(seed)
    rp = [0]
    cols, vals = [], []
    for i in range(n):
        k = int(rng.integers(1, per_row + 1)) if ragged else per_row
        k = min(k, n)
        c = set(rng.choice(n, size=k, replace=False).tolist())
        c.add(i)
        c = sorted(c)
        v = rng.uniform(-1.0, 1.0, len(c))
        v[c.index(i)] += diag_shift
        cols.extend(c)
        vals.extend(v.tolist())
        rp.append(len(cols))
    return CSR(n, np.asarray(rp, dtype=np.int32), np.asarray(cols, dtype=np.int32),
               np.asarray(vals, dtype=np.float64))


# ----------------------------------------------------------------- configs
CONFIG_NAMES = {
    1: "cd2d_64_pe10",
    2: "cd3d_128_pe50",
    3: "stencil27_96_fp32ir",
    4: "cd2d_512_pe20_adjoint",
    5: "cd3d_256_pe100",
}


# ILU(0) + polynomial composition (Section VI, second example): the paper's
# eps = 1/200 and GMRES(50) at tol 1e-8, with its degree-12 polynomial (d = 13
# roots), on an N x N grid (the paper's mesh has 1025^2 vertices).
ILU_WORKLOAD = {"name": "recirc2d_257_eps200_ilu0", "N": 257, "eps": 1.0 / 200.0, "m": 50,
                "d": 13, "tol": 1e-8, "v0_seed": 106}
# Section VI, first example: the same flow with eps = 1/2, GMRES(50) at tol 1e-8
# without a preconditioner and with the paper's degrees 4 and 9 (d = 5 and 10
# roots), on the paper's size (1025^2 unknowns).
EX1_WORKLOAD = {"name": "recirc2d_1025_eps2", "N": 1025, "eps": 0.5, "m": 50,
                "degrees": [0, 5, 10], "tol": 1e-8, "v0_seed": 107}


def permutation(n: int, seed: int, block: Optional[int] = None) -> np.ndarray:
    """A seeded permutation of range(n): uniform over all of it (block None), or
    uniform within each run of `block` consecutive indices (locality kept)."""
    rng = np.random.default_rng(seed)
    if block is None:
        return rng.permutation(n)
    perm = np.arange(n)
    for s in range(0, n, block):
        perm[s:s + block] = s + rng.permutation(min(block, n - s))
    return perm


def permuted(A: CSR, perm: np.ndarray) -> CSR:
    """The symmetric permutation P A P^T: row and column perm[i] of A become row and
    column i (columns sorted within each row).  Same spectrum; no diagonal structure
    is left unless perm keeps it."""
    inv = np.empty_like(perm)
    inv[perm] = np.arange(A.n)
    lens = np.diff(A.row_ptr)[perm]
    rp = np.zeros(A.n + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    starts = A.row_ptr[perm].astype(np.int64)
    idx = np.repeat(starts - rp[:-1], lens) + np.arange(rp[-1])
    cols = inv[A.col_ind[idx]].astype(np.int32)
    vals = A.vals[idx]
    rows = np.repeat(np.arange(A.n), lens)
    order = np.lexsort((cols, rows))
    return CSR(A.n, rp.astype(np.int32), cols[order], vals[order])


def _rhs_from_solution(A: CSR, x: np.ndarray) -> np.ndarray:
    import scipy.sparse as sp
    M = sp.csr_matrix((A.vals, A.col_ind, A.row_ptr), shape=(A.n, A.n))
    return M @ x


def config(k: int, N: Optional[int] = None) -> Problem:
    """The five workloads, optionally on a smaller grid ``N`` (same recipe).

    1: 2D CD, 64^2, Pe 10, wind (1,1), x* ~ U(-1,1) seed 0, b = A x*,
       v0 ~ U(-1,1) seed 100, m=50, d=10, tol 1e-8.
    2: 3D CD, 128^3, Pe 50, wind (1,.5,.25), b ~ N(0,1) seed 1, v0 seed 101,
       m=50, d=25 (also 0/10/40), tol 1e-10.
    3: 27-point random stencil 96^3 (values seed 3), b ~ N(0,1) seed 2,
       v0 seed 102, m=40, d=25, tol 1e-10 (FP32 inside FP64 refinement).
    4: 2D CD, 512^2, Pe 20, wind (1,1), b ~ N(0,1) seed 4, target
       x_t ~ U(0,1) seed 5, forward v0 seed 104, adjoint v0 seed 204, d=15,
       tol 1e-12, 64 sampled entries (seed 6).
    5: 3D CD, 256^3, Pe 100, wind (1,.5,.25), b ~ N(0,1) seed 7, v0 seed 105,
       m=30, d=40, tol 1e-8.
    """
    if k == 1:
        N = N or 64
        A = convection_diffusion(N, 2, 10.0, (1.0, 1.0))
        xs = uniform(A.n, 0)
        return Problem(CONFIG_NAMES[1], A, _rhs_from_solution(A, xs), uniform(A.n, 100),
                       m=50, d=10, tol=1e-8, x_star=xs)
    if k == 2:
        N = N or 128
        A = convection_diffusion(N, 3, 50.0, (1.0, 0.5, 0.25))
        return Problem(CONFIG_NAMES[2], A, normal(A.n, 1), uniform(A.n, 101),
                       m=50, d=25, tol=1e-10, extra={"degrees": [0, 10, 25, 40]})
    if k == 3:
        N = N or 96
        A = stencil27_random(N, seed=3)
        return Problem(CONFIG_NAMES[3], A, normal(A.n, 2), uniform(A.n, 102),
                       m=40, d=25, tol=1e-10, extra={"inner_tol": 1e-5})
    if k == 4:
        N = N or 512
        A = convection_diffusion(N, 2, 20.0, (1.0, 1.0))
        return Problem(CONFIG_NAMES[4], A, normal(A.n, 4), uniform(A.n, 104),
                       m=50, d=15, tol=1e-12,
                       extra={"x_target": uniform(A.n, 5, 0.0, 1.0),
                              "v0_adjoint": uniform(A.n, 204),
                              "fd_entries": np.random.default_rng(6).choice(
                                  A.nnz, size=min(64, A.nnz), replace=False),
                              "fd_h": 1e-6})
    if k == 5:
        N = N or 256
        A = convection_diffusion(N, 3, 100.0, (1.0, 0.5, 0.25))
        return Problem(CONFIG_NAMES[5], A, normal(A.n, 7), uniform(A.n, 105),
                       m=30, d=40, tol=1e-8)
    raise ValueError(f"unknown config {k}")
