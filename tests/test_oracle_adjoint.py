"""Pins of the oracle's adjoint gradient and its finite-difference reference.

The adjoint gradient and the Sherman-Morrison differences are checked
against brute-force central differences that re-solve the perturbed dense
system, so a wrong sign, a transposed solve or swapped indices fails here.
"""
import numpy as np
import scipy.sparse as sp

from oracle import adjoint
from paper_1907_00072_amd import workloads as W


def _tiny():
    A = W.random_csr(12, 4, seed=40, diag_shift=4.0)
    M = A.to_scipy()
    b = W.normal(12, 41)
    xt = W.uniform(12, 42, 0.0, 1.0)
    return A, M, b, xt


def _loss_dense(Ad, b, xt):
    x = np.linalg.solve(Ad, b)
    return 0.5 * np.sum((x - xt) ** 2)


def test_adjoint_gradient_vs_brute_force_differences():
    A, M, b, xt = _tiny()
    x, lam, gb, gv = adjoint.adjoint_gradient(M, b, xt)
    Ad = M.toarray()
    rows = adjoint.csr_rows(A.row_ptr)
    h = 1e-6
    for k in range(A.nnz):
        i, j = rows[k], A.col_ind[k]
        Ap = Ad.copy()
        Ap[i, j] += h
        Am = Ad.copy()
        Am[i, j] -= h
        fd = (_loss_dense(Ap, b, xt) - _loss_dense(Am, b, xt)) / (2 * h)
        assert abs(fd - gv[k]) <= 1e-6 * max(1.0, abs(gv[k]))
    for i in range(12):
        e = np.zeros(12)
        e[i] = h
        fd = (_loss_dense(Ad, b + e, xt) - _loss_dense(Ad, b - e, xt)) / (2 * h)
        assert abs(fd - gb[i]) <= 1e-6 * max(1.0, abs(gb[i]))


def test_sherman_morrison_differences_match_resolves():
    A, M, b, xt = _tiny()
    ents = np.arange(A.nnz)
    sm = adjoint.fd_gradient_vals(M, b, xt, ents, h=1e-4)
    Ad = M.toarray()
    rows = adjoint.csr_rows(A.row_ptr)
    h = 1e-4
    for t, k in enumerate(ents):
        Ap = Ad.copy()
        Ap[rows[k], A.col_ind[k]] += h
        Am = Ad.copy()
        Am[rows[k], A.col_ind[k]] -= h
        fd = (_loss_dense(Ap, b, xt) - _loss_dense(Am, b, xt)) / (2 * h)
        assert abs(fd - sm[t]) <= 1e-9 * max(1.0, abs(fd))
    gb = adjoint.fd_gradient_b(M, b, xt, np.arange(12))
    _, _, gref, _ = adjoint.adjoint_gradient(M, b, xt)
    assert np.allclose(gb, gref, rtol=1e-10, atol=1e-12)


def test_adjoint_on_reduced_config4_grid():
    P = W.config(4, N=48)
    M = P.A.to_scipy()
    xt = P.extra["x_target"]
    x, lam, gb, gv = adjoint.adjoint_gradient(M, P.b, xt)
    ents = np.random.default_rng(6).choice(P.A.nnz, size=16, replace=False)
    fd = adjoint.fd_gradient_vals(M, P.b, xt, ents, h=1e-6)
    assert np.max(np.abs(fd - gv[ents])) <= 1e-6 * np.max(np.abs(gv))
    # the gradient of a symmetric-pattern operator uses A^T, not A: check the solve
    assert np.linalg.norm(sp.csr_matrix(M).T @ lam - (x - xt)) <= 1e-10 * np.linalg.norm(x - xt)
