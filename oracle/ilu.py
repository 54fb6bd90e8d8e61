"""Oracle: ILU(0) on the left, the polynomial on the right (test infrastructure).

Section VI, second example: the polynomial preconditioner composed with an
incomplete LU factorisation M = L U with no fill (ILU(0)).  ILU(0) acts on
the left and the polynomial on the right, so GMRES(m) solves
M^-1 A p(M^-1 A) y = M^-1 b and x = p(M^-1 A) y; the polynomial is built for
the operator M^-1 A.

ILU(0) is the incomplete factorisation of Saad, "Iterative Methods for Sparse
Linear Systems", Section 10.3 (the IKJ form of Gaussian elimination with every
update outside the pattern of A dropped).  L is unit lower triangular and U
upper triangular, both on A's pattern, and (L U)_ij = a_ij for every stored
(i, j).  The factors are returned in one CSR matrix with A's pattern: the
strictly lower part holds L (its unit diagonal implied), the rest holds U.

Readings where the paper is silent: the rows keep A's order (no reordering);
A's columns must be sorted and unique in every row with a stored diagonal; a
zero pivot is an error; the stopping test is the preconditioned relative
residual ||M^-1 (b - A x)|| / ||M^-1 b||, with the unpreconditioned one
reported beside it.

Pins (tests/test_oracle_ilu.py): the product L U against A on the pattern;
exact LU from the textbook routine where the pattern has no fill; closed forms
for triangular A; level counts of grid orderings; the composed solve on a
matrix whose ILU(0) is exact.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .gmres import pp_gmres

__all__ = ["ilu0", "ilu0_split", "ilu0_solve", "dependency_levels", "pp_gmres_left_ilu0"]


def _checked_csr(A):
    A = sp.csr_matrix(A, dtype=np.float64)
    n = A.shape[0]
    rp, ci = A.indptr, A.indices
    diag = np.empty(n, dtype=np.int64)
    for i in range(n):
        cols = ci[rp[i]:rp[i + 1]]
        if np.any(np.diff(cols) <= 0):
            raise ValueError(f"row {i}: columns not sorted and unique")
        hit = np.nonzero(cols == i)[0]
        if hit.size != 1:
            raise ValueError(f"row {i}: no stored diagonal")
        diag[i] = rp[i] + hit[0]
    return A, diag


def ilu0(A):
    """ILU(0) factors of A on A's pattern, as one CSR matrix (see module doc).

    Row by row (i ascending): for every stored a_ik with k < i, in increasing k,
    divide by the pivot u_kk, then subtract l_ik times row k of U from the
    entries of row i whose column is stored in both rows.
    """
    A, diag = _checked_csr(A)
    n = A.shape[0]
    rp, ci = A.indptr, A.indices
    lu = A.data.copy()
    for i in range(n):
        where = {int(ci[p]): p for p in range(rp[i], rp[i + 1])}
        for p in range(rp[i], diag[i]):
            k = int(ci[p])
            pivot = lu[diag[k]]
            if pivot == 0.0:
                raise ZeroDivisionError(f"zero pivot in row {k}")
            lu[p] = lu[p] / pivot
            for q in range(diag[k] + 1, rp[k + 1]):
                t = where.get(int(ci[q]))
                if t is not None:
                    lu[t] = lu[t] - lu[p] * lu[q]
    if np.any(lu[diag] == 0.0):  # the last pivots are never divided by above
        raise ZeroDivisionError("zero pivot")
    return sp.csr_matrix((lu, ci.copy(), rp.copy()), shape=A.shape)


def ilu0_split(LU):
    """(L, U) as separate CSR matrices: L unit lower, U upper with the diagonal."""
    n = LU.shape[0]
    L = (sp.tril(LU, -1, format="csr") + sp.identity(n, format="csr")).tocsr()
    U = sp.triu(LU, 0, format="csr")
    L.sort_indices()
    U.sort_indices()
    return L, U


def ilu0_solve(LU, r, split=None):
    """M^-1 r = U^-1 (L^-1 r) by forward then backward substitution."""
    L, U = split if split is not None else ilu0_split(LU)
    r = np.asarray(r, dtype=np.float64)
    z = spla.spsolve_triangular(L, r, lower=True, unit_diagonal=True)
    return spla.spsolve_triangular(U, z, lower=False)


def dependency_levels(A, upper=False):
    """Level of every row in the triangular solve with A's pattern.

    Lower (forward) solve: row i waits for the rows k < i stored in row i;
    upper (backward) solve: for the rows k > i.  A row's level is one more than
    the highest level it waits for (0 when it waits for none), so the rows of
    one level are independent.  Returns an int array of n levels.
    """
    A = sp.csr_matrix(A)
    n = A.shape[0]
    rp, ci = A.indptr, A.indices
    lev = np.zeros(n, dtype=np.int64)
    order = range(n - 1, -1, -1) if upper else range(n)
    for i in order:
        deps = ci[rp[i]:rp[i + 1]]
        deps = deps[deps > i] if upper else deps[deps < i]
        if deps.size:
            lev[i] = 1 + int(lev[deps].max())
    return lev


def pp_gmres_left_ilu0(A, b, m, tol, v0=None, d=None, max_iters=100000, LU=None):
    """GMRES(m) on M^-1 A p(M^-1 A) y = M^-1 b, x = p(M^-1 A) y, M = ILU(0) of A.

    The polynomial (d roots, from v0) is built for the operator M^-1 A; the
    stopping test is ||M^-1 (b - A x)|| / ||M^-1 b|| < tol.  Returns
    (x, stats) with ``stats.relres_original`` = ||b - A x|| / ||b||.
    """
    A = sp.csr_matrix(A, dtype=np.float64)
    LU = ilu0(A) if LU is None else LU
    split = ilu0_split(LU)
    B = spla.LinearOperator(A.shape, matvec=lambda v: ilu0_solve(LU, A @ v, split),
                            dtype=np.float64)
    bt = ilu0_solve(LU, b, split)
    x, st = pp_gmres(B, bt, m, tol, v0=v0, d=d, max_iters=max_iters)
    st.relres_original = float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))
    return x, st
