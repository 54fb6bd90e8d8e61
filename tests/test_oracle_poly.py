"""Pins of the oracle's polynomial (construction, Leja order, application).

Every check compares the oracle with something other than itself: an
independent characterisation (harmonic Ritz values as a generalised
eigenproblem of an explicitly built Krylov basis), the paper's power-basis
normal equations (Section II, eqs. (1)-(2)), closed forms (diagonal and
triangular A, p(A) = A^{-1} at full degree), brute force (dense p(A) from
pi(A)), invariants (scaling, symmetry, conjugate closure), and the greedy
definition of the Leja order.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import poly
from paper_1907_00072_amd import workloads as W


def _rand_nonsym(n, seed, shift=3.0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n)) / np.sqrt(n) + shift * np.eye(n)


def _match(a, b):
    """Max distance after matching each a to its nearest b (greedy, both sorted)."""
    a = list(np.asarray(a, complex))
    b = list(np.asarray(b, complex))
    worst = 0.0
    for t in a:
        j = int(np.argmin([abs(t - u) for u in b]))
        worst = max(worst, abs(t - b[j]) / max(abs(t), 1e-300))
        b.pop(j)
    return worst


def _krylov_orth(A, v0, k):
    """Orthonormal basis of K_k(A, v0) from the explicit power basis (numpy QR)."""
    K = np.empty((v0.size, k))
    v = v0 / np.linalg.norm(v0)
    for j in range(k):
        K[:, j] = v
        v = A @ v
        v = v / np.linalg.norm(v)
    Q, _ = np.linalg.qr(K)
    return Q


def test_arnoldi_relation_and_orthonormality():
    A = _rand_nonsym(60, 1)
    v0 = W.uniform(60, 2)
    Q, H, s = poly.arnoldi(A, v0, 12)
    assert s == 12
    assert np.linalg.norm(Q.T @ Q - np.eye(13)) < 1e-13
    assert np.linalg.norm(A @ Q[:, :12] - Q @ H) < 1e-12 * np.linalg.norm(A)
    assert np.allclose(np.tril(H, -2), 0)
    assert np.allclose(Q[:, 0], v0 / np.linalg.norm(v0))


@pytest.mark.parametrize("seed,d", [(3, 4), (4, 6), (5, 8)])
def test_harmonic_ritz_equals_pencil_eigenvalues(seed, d):
    """theta from H + h^2 H^-T e e^T equals eig((AQ)^T AQ, (AQ)^T Q) (Petrov-Galerkin definition)."""
    n = 80
    A = _rand_nonsym(n, seed)
    v0 = W.uniform(n, seed + 10)
    _, Hbar, s = poly.arnoldi(A, v0, d)
    theta = poly.harmonic_ritz(Hbar)
    Q = _krylov_orth(A, v0, d)
    AQ = A @ Q
    ref = scipy.linalg.eigvals(AQ.T @ AQ, AQ.T @ Q)
    assert _match(theta, ref) < 1e-8


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_roots_equal_power_basis_normal_equations(d):
    """Paper eqs. (1)-(2) with deg = d-1: zeros of 1 - alpha p(alpha) are the harmonic Ritz values."""
    A = W.convection_diffusion(10, 2, 40.0, (1.0, 1.0)).to_scipy()
    v0 = W.uniform(A.shape[0], 7)
    y, info = poly.power_basis_poly(A, v0, d - 1)
    assert info == 0
    # pi(alpha) = 1 - sum_k y_k alpha^(k+1); numpy.roots wants highest degree first
    coeffs = np.concatenate([-y[::-1], [1.0]])
    ref = np.roots(coeffs)
    roots, s = poly.build_poly(A, v0, d)
    assert s == d
    assert _match(roots, ref) < 1e-7


def test_min_residual_property():
    """||v0 - A p(A) v0|| equals the least-squares minimum over all p of degree d-1."""
    n, d = 120, 7
    A = _rand_nonsym(n, 8, shift=2.0)
    v0 = W.uniform(n, 9)
    roots, s = poly.build_poly(A, v0, d)
    got = np.linalg.norm(v0 - A @ poly.apply_poly(A, roots, v0))
    # independent: minimise ||v0 - A K c|| over the orthonormalised Krylov basis K
    Q = _krylov_orth(A, v0, d)
    c, *_ = np.linalg.lstsq(A @ Q, v0, rcond=None)
    ref = np.linalg.norm(v0 - A @ Q @ c)
    assert abs(got - ref) <= 1e-10 * np.linalg.norm(v0)
    # and a perturbed polynomial is strictly worse
    worse = np.linalg.norm(v0 - A @ poly.apply_poly(A, roots * 1.01, v0))
    assert worse > got


def test_full_degree_is_the_inverse():
    """d = n: pi(A) = 0 (Cayley-Hamilton), so p(A) = A^{-1}."""
    n = 12
    A = _rand_nonsym(n, 12, shift=2.5)
    v0 = W.uniform(n, 13)
    roots, s = poly.build_poly(A, v0, n)
    assert s == n
    v = W.uniform(n, 14)
    ref = np.linalg.solve(A, v)
    assert np.linalg.norm(poly.apply_poly(A, roots, v) - ref) < 1e-9 * np.linalg.norm(ref)


def test_diagonal_matrix_closed_form():
    """Diagonal A: (p(A) v)_i = p(a_i) v_i with p(a) = (1 - prod(1 - a/theta)) / a."""
    a = np.linspace(0.5, 9.0, 50)
    A = np.diag(a)
    v0 = W.uniform(50, 15)
    roots, s = poly.build_poly(A, v0, 6)
    v = W.uniform(50, 16)
    pa = (1.0 - np.prod([1.0 - a / t for t in roots], axis=0).real) / a
    assert np.allclose(poly.apply_poly(A, roots, v), pa * v, rtol=1e-12, atol=1e-14)
    # full degree on a diagonal matrix: the roots are exactly its entries
    a5 = np.array([1.0, 2.0, 3.5, 5.0, 7.0])
    r5, _ = poly.build_poly(np.diag(a5), W.uniform(5, 17), 5)
    assert np.allclose(np.sort(r5.real), a5, rtol=1e-10)
    assert np.all(r5.imag == 0)


def test_bidiag_diagonal_of_p_is_p_of_diagonal():
    """Upper triangular A (BiDiag1, Section IV): (p(A))_ii = p(a_ii)."""
    Ac = W.bidiag1()
    A = Ac.to_scipy()
    v0 = W.uniform(Ac.n, 18)
    roots, s = poly.build_poly(A, v0, 8)
    for i in (0, 3, 500, 1999):
        e = np.zeros(Ac.n)
        e[i] = 1.0
        col = poly.apply_poly(A, roots, e)
        a = float(i + 1)
        pa = (1.0 - np.prod([1.0 - a / t for t in roots]).real) / a
        assert abs(col[i] - pa) <= 1e-10 * abs(pa)
        assert np.all(col[i + 1:] == 0)          # upper triangular stays upper


def test_symmetric_matrix_has_real_roots():
    A = W.laplacian5(30).to_scipy()
    roots, s = poly.build_poly(A, W.uniform(900, 19), 12)
    assert s == 12
    assert np.all(roots.imag == 0)
    assert np.all((roots.real > 0) & (roots.real < 8))


def test_scaling_invariance():
    """roots(cA) = c roots(A) and p_{cA}(cA) v = p_A(A) v / c."""
    A = _rand_nonsym(70, 20)
    v0 = W.uniform(70, 21)
    c = 3.7
    r1, _ = poly.build_poly(A, v0, 6)
    r2, _ = poly.build_poly(c * A, v0, 6)
    assert _match(r2, c * r1) < 1e-11
    v = W.uniform(70, 22)
    assert np.allclose(poly.apply_poly(c * A, r2, v), poly.apply_poly(A, r1, v) / c, rtol=1e-11)


@pytest.mark.parametrize("seed,n,d", [(23, 20, 5), (24, 40, 9), (25, 64, 12)])
def test_dense_brute_force(seed, n, d):
    """Every column of p(A) equals A^{-1} (I - prod_i (I - A/theta_i)) formed densely."""
    A = _rand_nonsym(n, seed, shift=1.5)
    roots, s = poly.build_poly(A, W.uniform(n, seed + 1), d)
    P = np.eye(n, dtype=complex)
    for t in roots:
        P = P @ (np.eye(n) - A / t)
    ref = np.linalg.solve(A, np.eye(n) - P).real
    got = np.column_stack([poly.apply_poly(A, roots, e) for e in np.eye(n)])
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


def test_complex_roots_are_conjugate_pairs_and_result_is_real():
    A = _rand_nonsym(90, 26, shift=1.0)
    roots, s = poly.build_poly(A, W.uniform(90, 27), 10)
    assert np.any(roots.imag != 0), "expected complex roots for this matrix"
    i = 0
    while i < roots.size:
        if roots[i].imag != 0:
            assert roots[i].imag > 0 and roots[i + 1] == np.conj(roots[i])
            i += 2
        else:
            i += 1
    v = W.uniform(90, 28)
    ctype_y = v.astype(complex)
    prod = ctype_y.copy()
    y = np.zeros_like(prod)
    for k, t in enumerate(roots):
        y += prod / t
        prod = prod - (A @ prod) / t
    assert np.linalg.norm(y.imag) <= 1e-13 * np.linalg.norm(y.real)


def _leja_property(order):
    """Check the greedy definition of the modified Leja order on an ordered list."""
    order = list(order)
    first = order[0]
    assert all(abs(first) >= abs(t) - 1e-15 for t in order)
    taken = []
    i = 0
    while i < len(order):
        t = order[i]
        if taken:
            rest = [u for u in order[i:] if u.imag >= 0]
            def score(u):
                dist = np.abs(u - np.asarray(taken))
                return -np.inf if np.any(dist == 0) else np.sum(np.log(dist))
            best = max(score(u) for u in rest)
            assert score(t) >= best - 1e-12 * max(1.0, abs(best)) or (best == -np.inf)
        assert t.imag >= 0
        taken.append(t)
        if t.imag > 0:
            assert order[i + 1] == np.conj(t)
            taken.append(order[i + 1])
            i += 2
        else:
            i += 1


def test_leja_order_greedy_definition():
    rng = np.random.default_rng(29)
    for trial in range(20):
        nr = int(rng.integers(0, 6))
        nc = int(rng.integers(0, 4))
        re = list(rng.uniform(-5, 5, nr))
        cx = list(rng.uniform(-5, 5, nc) + 1j * rng.uniform(0.1, 3, nc))
        pts = np.array(re + cx + [np.conj(c) for c in cx], dtype=complex)
        if pts.size == 0:
            continue
        rng.shuffle(pts)
        out = poly.leja_order(pts)
        assert sorted(out, key=lambda t: (t.real, t.imag)) == sorted(pts, key=lambda t: (t.real, t.imag))
        _leja_property(out)


def test_leja_repeats_go_last_and_rejects_unpaired():
    out = poly.leja_order(np.array([2.0, 1.0, 2.0, -3.0, 1.0]))
    assert list(out[:3].real) == [-3.0, 2.0, 1.0]
    assert sorted(out[3:].real) == [1.0, 2.0]
    with pytest.raises(ValueError):
        poly.leja_order(np.array([1.0 + 1j, 2.0]))


def test_happy_breakdown_reduces_degree():
    """v0 in a 3-dimensional invariant subspace: only 3 roots, and p(A) v0 = A^{-1} v0."""
    a = np.array([1.0, 2.0, 4.0] * 10)
    A = np.diag(a)
    v0 = W.uniform(30, 30)
    roots, s = poly.build_poly(A, v0, 6)
    assert s == 3 and roots.size == 3
    assert np.allclose(np.sort(roots.real), [1.0, 2.0, 4.0], rtol=1e-10)
    assert np.allclose(poly.apply_poly(A, roots, v0), v0 / a, rtol=1e-10)


def test_power_basis_warning_onset(golden_dir):
    """Section IV: POTRF starts warning around degree 10-12 on the test matrices; none at low degree."""
    g = json.load(open(os.path.join(golden_dir, "sec4_bidiag.json")))
    for f, spec in ((W.bidiag1, g["bidiag1"]), (W.bidiag2, g["bidiag2"])):
        Ac = f()
        assert Ac.n == spec["n"]
        A = Ac.to_scipy()
        for seed in range(3):
            b = A @ np.random.default_rng(seed).random(Ac.n)
            first = None
            for deg in range(3, 19):
                y, info = poly.power_basis_poly(A, b, deg)
                if deg <= 9:
                    assert info == 0 and np.all(np.isfinite(y))
                if info > 0 and first is None:
                    first = deg
                    break
            assert first is not None and 10 <= first <= 15


def test_bidiag_definitions(golden_dir):
    b1, b2 = W.bidiag1(), W.bidiag2()
    d1 = b1.vals[b1.row_ptr[:-1]]
    d2 = b2.vals[b2.row_ptr[:-1]]
    assert np.array_equal(d1, np.arange(1, 2001))
    assert np.allclose(d2[:9], np.arange(1, 10) / 10) and np.array_equal(d2[9:], np.arange(1, 4992))
    assert np.all(b1.vals[b1.row_ptr[:-2] + 1] == 0.05)
    assert np.all(b2.vals[b2.row_ptr[:-2] + 1] == 0.2)


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_power_series_apply_equals_root_form(d):
    """The paper's coefficients applied as sum y_k A^k v equal the Leja product form (d <= 5)."""
    A = W.convection_diffusion(10, 2, 40.0, (1.0, 1.0)).to_scipy()
    v0 = W.uniform(A.shape[0], 7)
    y, info = poly.power_basis_poly(A, v0, d - 1)
    assert info == 0 and y.size == d
    roots, _ = poly.build_poly(A, v0, d)
    v = W.uniform(A.shape[0], 8)
    ref = poly.apply_poly(A, roots, v)
    assert np.linalg.norm(poly.apply_power(A, y, v) - ref) <= 1e-8 * np.linalg.norm(ref)


def test_auto_degree_is_last_degree_without_warning():
    """Section IV: the highest degree whose Gram matrix factors (onset of warnings at 10-12)."""
    import scipy.linalg
    for f in (W.bidiag1, W.bidiag2):
        Ac = f()
        A = Ac.to_scipy()
        b = A @ np.random.default_rng(1).random(Ac.n)
        deg, y, info = poly.auto_degree(A, b, 18)
        assert info > 0 and 8 <= deg <= 13 and y.size == deg + 1
        G, rhs = poly._power_gram(A, b, deg + 1)
        assert scipy.linalg.lapack.dpotrf(G[: deg + 2, : deg + 2], lower=0)[1] > 0
        assert scipy.linalg.lapack.dpotrf(G[: deg + 1, : deg + 1], lower=0)[1] == 0
        # the selected polynomial preconditions: GMRES(50) converges with it
        from oracle import gmres
        _, st = gmres.pp_gmres(A, b, 50, 1e-8, coeffs=y, max_iters=3000)
        assert st.converged


def test_warned_degree_keeps_lower_coefficients():
    """Reading of a POTRF warning: coefficients of the leading factorable block, zeros above
    (the plateau of Table I)."""
    Ac = W.bidiag2()
    A = Ac.to_scipy()
    b = A @ np.random.default_rng(1).random(Ac.n)
    y, info = poly.power_basis_poly(A, b, 16)
    assert info > 0
    k = info - 1
    assert np.all(y[k:] == 0) and np.all(np.isfinite(y[:k])) and np.any(y[:k] != 0)


def test_power_form_gmres_matches_root_form():
    from oracle import gmres
    P = W.config(1)
    A = P.A.to_scipy()
    y, info = poly.power_basis_poly(A, P.v0, 5)
    assert info == 0
    _, s_pow = gmres.pp_gmres(A, P.b, P.m, P.tol, coeffs=y, max_iters=2000)
    _, s_root = gmres.pp_gmres(A, P.b, P.m, P.tol, v0=P.v0, d=6, max_iters=2000)
    assert s_pow.converged and s_root.converged
    assert abs(s_pow.iters - s_root.iters) <= max(1, round(0.02 * s_root.iters))
