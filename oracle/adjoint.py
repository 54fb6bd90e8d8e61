"""Oracle: adjoint gradient of a linear solve (test infrastructure).

For x = A^{-1} b and a loss L(x), the adjoint lambda solves A^T lambda = dL/dx;
then dL/db = lambda and dL/dA_ij = -lambda_i x_j, restricted to the stored
pattern of A.  Here the solves are direct (dense LU for small n, SuperLU
otherwise), so the result does not depend on any iteration tolerance.

The finite-difference reference perturbs one stored entry, A + h e_i e_j^T,
and gets the perturbed solution exactly from the Sherman-Morrison formula
x(h) = x - h u x_j / (1 + h u_j) with u = A^{-1} e_i, so no iterative solve
is involved.  The central difference of L = 0.5 ||x - x_t||^2 is formed as
(L(h) - L(-h)) / 2h with L(h) - L(-h) expanded as
e.(dp - dm) + 0.5 (|dp|^2 - |dm|^2), e = x - x_t, dp/dm = x(+-h) - x,
which is algebraically the same number without the cancellation of two
large losses.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = ["DirectSolver", "loss", "adjoint_gradient", "fd_gradient_vals", "fd_gradient_b",
           "csr_rows"]


class DirectSolver:
    """Direct solves with A and A^T (dense LU for n <= 4096, SuperLU otherwise)."""

    def __init__(self, A):
        self.n = A.shape[0]
        if self.n <= 4096:
            import scipy.linalg
            Ad = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
            self._lu = scipy.linalg.lu_factor(Ad)
            self._dense = True
        else:
            self._lu = spla.splu(sp.csc_matrix(A))
            self._dense = False

    def solve(self, b, trans=False):
        if self._dense:
            import scipy.linalg
            return scipy.linalg.lu_solve(self._lu, b, trans=1 if trans else 0)
        return self._lu.solve(np.asarray(b, dtype=np.float64), trans="T" if trans else "N")


def loss(x, x_t):
    """L = 0.5 ||x - x_t||^2."""
    e = x - x_t
    return 0.5 * float(e @ e)


def csr_rows(row_ptr):
    """Row index of every stored entry."""
    row_ptr = np.asarray(row_ptr)
    return np.repeat(np.arange(row_ptr.size - 1), np.diff(row_ptr))


def adjoint_gradient(A_csr, b, x_t, solver=None):
    """(x, lambda, dL/db, dL/dvals) for L = 0.5 ||A^{-1} b - x_t||^2."""
    A = sp.csr_matrix(A_csr)
    S = solver or DirectSolver(A)
    x = S.solve(b)
    lam = S.solve(x - x_t, trans=True)
    rows = csr_rows(A.indptr)
    g_vals = -lam[rows] * x[A.indices]
    return x, lam, lam.copy(), g_vals


def fd_gradient_vals(A_csr, b, x_t, entries, h=1e-6, solver=None, x=None):
    """Central differences of L with respect to the stored values ``entries``."""
    A = sp.csr_matrix(A_csr)
    S = solver or DirectSolver(A)
    if x is None:
        x = S.solve(b)
    e = x - x_t
    rows = csr_rows(A.indptr)
    out = np.empty(len(entries))
    for t, k in enumerate(entries):
        i, j = int(rows[k]), int(A.indices[k])
        ei = np.zeros(A.shape[0])
        ei[i] = 1.0
        u = S.solve(ei)
        dp = -h * u * x[j] / (1.0 + h * u[j])
        dm = h * u * x[j] / (1.0 - h * u[j])
        dL = e @ (dp - dm) + 0.5 * (dp @ dp - dm @ dm)
        out[t] = dL / (2.0 * h)
    return out


def fd_gradient_b(A_csr, b, x_t, idx, h=1e-6, solver=None, x=None):
    """Central differences of L with respect to b[idx] (x(h) = x + h A^{-1} e_i exactly)."""
    A = sp.csr_matrix(A_csr)
    S = solver or DirectSolver(A)
    if x is None:
        x = S.solve(b)
    e = x - x_t
    out = np.empty(len(idx))
    for t, i in enumerate(idx):
        ei = np.zeros(A.shape[0])
        ei[int(i)] = 1.0
        u = S.solve(ei)
        # L(h) - L(-h) = 2 h e.u exactly (the quadratic terms cancel)
        out[t] = (2.0 * h * (e @ u)) / (2.0 * h)
    return out
