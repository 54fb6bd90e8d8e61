"""Pins of the oracle's ILU(0), its triangular solves, its dependency levels and
the composition of Section VI's second example (ILU(0) left, polynomial right).

Pinned against: the defining property of ILU(0) (L U equals A on A's
pattern), the textbook LU factorisation where the pattern admits no fill,
closed forms for triangular A, the level counts of natural grid orderings, and
a composed solve whose ILU(0) is exact (M^-1 A = I).
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

from oracle import ilu
from paper_1907_00072_amd import workloads as W


def _matrices():
    out = {
        "recirc_9": W.recirculating_flow(9)[0].to_scipy(),
        "cd3d_5": W.convection_diffusion(5, 3, 50.0, (1.0, 0.5, 0.25)).to_scipy(),
        "stencil27_4": W.stencil27_random(4, seed=3).to_scipy(),
        "random_60": W.random_csr(60, 6, seed=11, diag_shift=8.0).to_scipy(),
    }
    return out


@pytest.mark.parametrize("name", list(_matrices()))
def test_product_of_factors_equals_a_on_its_pattern(name):
    A = _matrices()[name]
    LU = ilu.ilu0(A)
    L, U = ilu.ilu0_split(LU)
    P = (L @ U).tocsr()
    pat = A.copy()
    pat.data[:] = 1.0
    diff = (P - A).multiply(pat)
    assert abs(diff).max() <= 1e-13 * abs(A).max(), name
    # the factors keep A's pattern: updates that fall outside it are dropped
    assert np.array_equal(LU.indices, A.indices) and np.array_equal(LU.indptr, A.indptr)


def test_no_fill_pattern_gives_the_exact_lu():
    # a tridiagonal matrix has no fill: ILU(0) is the LU factorisation itself;
    # column diagonal dominance makes partial pivoting a no-op
    n = 40
    rng = np.random.default_rng(5)
    lo, up = rng.uniform(-1, 1, n - 1), rng.uniform(-1, 1, n - 1)
    dg = 3.0 + rng.uniform(0, 1, n)
    A = sp.diags([lo, dg, up], [-1, 0, 1], format="csr")
    P, Lr, Ur = scipy.linalg.lu(A.toarray())
    assert np.array_equal(P, np.eye(n))
    L, U = ilu.ilu0_split(ilu.ilu0(A))
    assert np.allclose(L.toarray(), Lr, rtol=0, atol=1e-14)
    assert np.allclose(U.toarray(), Ur, rtol=0, atol=1e-14)


def test_dense_pattern_gives_the_exact_lu():
    n = 12
    rng = np.random.default_rng(6)
    M = rng.uniform(-1, 1, (n, n))
    M += np.diag(np.abs(M).sum(axis=0) + 1.0)  # column dominant: no row swaps
    P, Lr, Ur = scipy.linalg.lu(M)
    assert np.array_equal(P, np.eye(n))
    L, U = ilu.ilu0_split(ilu.ilu0(sp.csr_matrix(M)))
    assert np.allclose(L.toarray(), Lr, rtol=0, atol=1e-13)
    assert np.allclose(U.toarray(), Ur, rtol=0, atol=1e-13)


def test_triangular_matrices_in_closed_form():
    A = W.random_csr(50, 5, seed=3, diag_shift=4.0).to_scipy()
    low = sp.tril(A, 0, format="csr")
    L, U = ilu.ilu0_split(ilu.ilu0(low))
    d = low.diagonal()
    assert np.allclose(U.toarray(), np.diag(d), rtol=0, atol=0)
    assert np.allclose(L.toarray(), (low @ sp.diags(1.0 / d)).toarray(), rtol=1e-15, atol=0)
    upp = sp.triu(A, 0, format="csr")
    L, U = ilu.ilu0_split(ilu.ilu0(upp))
    assert np.array_equal(L.toarray(), np.eye(50))
    assert np.array_equal(U.toarray(), upp.toarray())


def test_triangular_solves_invert_the_product_of_factors():
    A = W.recirculating_flow(17)[0].to_scipy()
    LU = ilu.ilu0(A)
    L, U = ilu.ilu0_split(LU)
    r = W.normal(A.shape[0], 9)
    z = ilu.ilu0_solve(LU, r)
    assert np.linalg.norm(L @ (U @ z) - r) <= 1e-13 * np.linalg.norm(r)


@pytest.mark.parametrize("N", [1, 2, 7, 16])
def test_levels_of_grid_orderings(N):
    # natural order: the forward solve's levels are the anti-diagonals i + j (+ k)
    A2 = W.recirculating_flow(N)[0].to_scipy()
    for upper in (False, True):
        lev = ilu.dependency_levels(A2, upper=upper)
        assert lev.max() + 1 == 2 * N - 1
        i = np.tile(np.arange(N), N)
        j = np.repeat(np.arange(N), N)
        want = (i + j) if not upper else (2 * (N - 1) - i - j)
        assert np.array_equal(lev, want)
    A3 = W.convection_diffusion(N, 3, 10.0, (1.0, 1.0, 1.0)).to_scipy()
    assert ilu.dependency_levels(A3).max() + 1 == 3 * N - 2
    assert ilu.dependency_levels(A3, upper=True).max() + 1 == 3 * N - 2


@pytest.mark.parametrize("upper", [False, True])
def test_levels_are_longest_dependency_chains(upper):
    # the longest-path levels are the only ones with (1) every dependency on a
    # lower level and (2) a dependency exactly one level down for level > 0
    A = W.random_csr(300, 7, seed=21, diag_shift=5.0).to_scipy()
    lev = ilu.dependency_levels(A, upper=upper)
    for i in range(A.shape[0]):
        deps = A.indices[A.indptr[i]:A.indptr[i + 1]]
        deps = deps[deps > i] if upper else deps[deps < i]
        assert np.all(lev[deps] < lev[i])
        if lev[i] > 0:
            assert np.any(lev[deps] == lev[i] - 1)
        else:
            assert deps.size == 0
    assert lev.max() > 3


def test_bad_patterns_are_rejected():
    A = sp.csr_matrix(np.array([[1.0, 0.0], [1.0, 0.0]]))
    A.eliminate_zeros()
    with pytest.raises(ValueError):
        ilu.ilu0(A)  # row 1 has no stored diagonal
    B = sp.csr_matrix((np.ones(3), np.array([1, 0, 1]), np.array([0, 2, 3])), shape=(2, 2))
    with pytest.raises(ValueError):
        ilu.ilu0(B)  # row 0's columns are not sorted
    Z = sp.csr_matrix(np.array([[1.0, 1.0], [1.0, 1.0]]))
    with pytest.raises(ZeroDivisionError):
        ilu.ilu0(Z)  # u_11 = 1 - 1 * 1 = 0


def test_composed_solve_with_an_exact_factorisation():
    # tridiagonal: ILU(0) = LU, so M^-1 A = I and one Arnoldi step solves it
    n = 64
    A = sp.diags([-1.2 * np.ones(n - 1), 4.0 * np.ones(n), -0.7 * np.ones(n - 1)], [-1, 0, 1],
                 format="csr")
    b = W.normal(n, 2)
    x, st = ilu.pp_gmres_left_ilu0(A, b, 10, 1e-12, v0=W.uniform(n, 3), d=1)
    assert st.converged and st.iters == 1
    assert np.linalg.norm(x - np.linalg.solve(A.toarray(), b)) <= 1e-12 * np.linalg.norm(x)


def test_composition_cuts_iterations_on_the_recirculating_flow():
    # Section VI, second example: ILU(0) with the polynomial beats ILU(0) alone
    A, b = W.recirculating_flow(33)
    M = A.to_scipy()
    LU = ilu.ilu0(M)
    v0 = W.uniform(A.n, 106)
    x0, s0 = ilu.pp_gmres_left_ilu0(M, b, 50, 1e-8, max_iters=2000, LU=LU)
    x1, s1 = ilu.pp_gmres_left_ilu0(M, b, 50, 1e-8, v0=v0, d=13, max_iters=2000, LU=LU)
    assert s0.converged and s1.converged
    assert s1.iters * 3 < s0.iters, (s0.iters, s1.iters)
    xs = sp.linalg.spsolve(M.tocsc(), b)
    for x, st in ((x0, s0), (x1, s1)):
        assert np.linalg.norm(x - xs) <= 1e-5 * np.linalg.norm(xs)
        assert st.relres_original < 1e-6
