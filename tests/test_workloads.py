"""The seeded input generators: sizes, closed-form nnz counts and stencil values."""
import numpy as np
import pytest

from paper_1907_00072_amd import workloads as W


@pytest.mark.parametrize("N", [5, 17, 64])
def test_cd2d_nnz_and_values(N):
    A = W.convection_diffusion(N, 2, 10.0, (1.0, 1.0))
    assert A.n == N * N and A.nnz == 5 * A.n - 4 * N
    P = 1.0 / (N + 1) * 10.0 / 2
    D = A.to_dense()
    i = N + 1  # an interior node
    assert D[i, i] == 4.0
    assert np.isclose(D[i, i + 1], -1 + P) and np.isclose(D[i, i - 1], -1 - P)
    assert np.isclose(D[i, i + N], -1 + P) and np.isclose(D[i, i - N], -1 - P)
    assert D[N - 1, N] == 0.0           # no wrap-around across grid lines


@pytest.mark.parametrize("N", [4, 9])
def test_cd3d_nnz_and_sorted_columns(N):
    A = W.convection_diffusion(N, 3, 50.0, (1.0, 0.5, 0.25))
    assert A.nnz == 7 * A.n - 6 * N * N
    for i in range(A.n):
        c = A.col_ind[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c


def test_stencil27():
    A = W.stencil27_random(6, seed=3)
    assert A.nnz == (3 * 6 - 2) ** 3
    D = A.to_dense()
    assert np.all(np.diag(D) == 30.0)
    off = D[(D != 0) & ~np.eye(A.n, dtype=bool)]
    assert off.min() >= -1.3 and off.max() <= -0.7


def test_configs_sizes_small():
    P1 = W.config(1)
    assert P1.A.n == 4096 and P1.A.nnz == 20224 and (P1.m, P1.d, P1.tol) == (50, 10, 1e-8)
    assert np.allclose(P1.A.to_scipy() @ P1.x_star, P1.b)
    P2 = W.config(2, N=8)
    assert P2.A.n == 512 and P2.tol == 1e-10
    P4 = W.config(4, N=16)
    assert P4.extra["fd_entries"].size == 64 and P4.d == 15


def test_seeds_are_deterministic():
    assert np.array_equal(W.uniform(10, 100), W.uniform(10, 100))
    assert np.array_equal(W.normal(10, 1), np.random.default_rng(1).standard_normal(10))
    a = W.uniform(1000, 5, 0.0, 1.0)
    assert a.min() >= 0 and a.max() < 1


def test_symmetric_permutation_is_p_a_pt():
    A = W.config(5, N=10).A
    M = A.to_scipy().toarray()
    for blk in (None, 64):
        p = W.permutation(A.n, 5, blk)
        assert np.array_equal(np.sort(p), np.arange(A.n))
        if blk:
            assert np.all(p // blk == np.arange(A.n) // blk)   # stays inside its block
        B = W.permuted(A, p)
        assert np.array_equal(B.to_scipy().toarray(), M[np.ix_(p, p)])
        for i in range(B.n):
            assert np.all(np.diff(B.col_ind[B.row_ptr[i]:B.row_ptr[i + 1]]) > 0)
