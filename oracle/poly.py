"""Oracle: the GMRES minimum-residual polynomial p(A) (test infrastructure).

Notation.  d = number of roots = degree of phi(alpha) = alpha*p(alpha);
p itself has degree d-1.  The paper's degree deg is d-1: it builds a power basis
with deg+1 columns (Section II) and needs deg+1 matrix-vector products to do
so (Section III).  The residual polynomial is pi(alpha) = 1 - alpha*p(alpha),
pi(0) = 1, and its zeros are the harmonic Ritz values theta_1..theta_d of A
with respect to the Krylov space K_d(A, v0).

Two constructions are provided:

* ``build_poly`` -- d Arnoldi steps on v0 give the (d+1) x d Hessenberg
  matrix Hbar; the harmonic Ritz values are the eigenvalues of
  H_d + h_{d+1,d}^2 H_d^{-T} e_d e_d^T; they are put in modified Leja order.
  The paper refers to such "more stable" constructions (end of Section II and
  Section VIII) without giving them; this is the root (product) form.
* ``power_basis_poly`` -- the paper's own construction (Section II, eqs. (1)
  and (2)): V = [v0, A v0, ..., A^deg v0], solve (AV)^T (AV) y = (AV)^T v0
  by Cholesky, p(A) = sum_k y_k A^(k-1).  In exact arithmetic it is the same
  polynomial (both minimise ||v0 - A p(A) v0|| over p of degree d-1); it is
  ill-conditioned beyond small degrees, as the paper reports (Section IV).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

__all__ = ["matvec", "arnoldi", "harmonic_ritz", "leja_order", "build_poly",
           "apply_poly", "power_basis_poly", "apply_power", "auto_degree", "BREAKDOWN_RTOL"]

# Happy breakdown of Arnoldi: the orthogonalised vector is at most this
# fraction of ||A q_j|| (the Krylov space is numerically invariant).
BREAKDOWN_RTOL = 1e-12


def matvec(A, x):
    """A @ x for a real sparse or dense A; complex x is split into two real products."""
    if np.iscomplexobj(x):
        return matvec(A, x.real) + 1j * matvec(A, x.imag)
    return A @ x


def arnoldi(A, v0, k):
    """k steps of Arnoldi on v0 with two unconditional classical Gram-Schmidt passes.

    Returns (Q, Hbar, s): Q is n x (s+1) with orthonormal columns, Hbar is the
    (s+1) x s upper Hessenberg matrix with A Q[:, :s] = Q Hbar, and s <= k is
    the number of steps taken (s < k only on a happy breakdown, when the
    Krylov space became invariant; then Hbar[s, s-1] is ~0).
    Arithmetic in v0's dtype; Hbar is float64.
    """
    v0 = np.asarray(v0)
    n = v0.size
    Q = np.zeros((n, k + 1), dtype=v0.dtype, order="F")
    H = np.zeros((k + 1, k))
    beta = np.linalg.norm(v0)
    if not beta > 0:
        raise ValueError("start vector is zero or not finite")
    Q[:, 0] = v0 / beta
    for j in range(k):
        w = matvec(A, Q[:, j])
        w0 = np.linalg.norm(w)
        Qj = Q[:, : j + 1]
        h1 = Qj.T @ w
        w = w - Qj @ h1
        h2 = Qj.T @ w
        w = w - Qj @ h2
        H[: j + 1, j] = np.asarray(h1, dtype=np.float64) + np.asarray(h2, dtype=np.float64)
        hn = float(np.linalg.norm(w))
        H[j + 1, j] = hn
        if hn <= BREAKDOWN_RTOL * w0:
            return Q[:, : j + 2], H[: j + 2, : j + 1], j + 1
        Q[:, j + 1] = w / hn
    return Q, H, k


def harmonic_ritz(Hbar):
    """Harmonic Ritz values from the (s+1) x s Arnoldi Hessenberg matrix.

    theta = eig(H_s + h^2 f e_s^T) with f = H_s^{-T} e_s and h = Hbar[s, s-1].
    Raises numpy.linalg.LinAlgError if H_s is singular.
    """
    Hbar = np.asarray(Hbar, dtype=np.float64)
    s = Hbar.shape[1]
    Hs = Hbar[:s, :s]
    h = Hbar[s, s - 1]
    e = np.zeros(s)
    e[-1] = 1.0
    f = np.linalg.solve(Hs.T, e)
    M = Hs.copy()
    M[:, -1] += h * h * f
    return np.linalg.eigvals(M)


def leja_order(theta):
    """Modified Leja order of a set of roots closed under conjugation.

    1. Start with the root of largest modulus (ties: larger real part, then
       positive imaginary part).
    2. Repeatedly take the remaining root that maximises the product of its
       distances to the roots already taken (sum of logs, so no overflow); a
       root equal to one already taken scores -inf, so repeats go last.
    3. Only roots with Im >= 0 are candidates; taking a complex root appends
       its conjugate right after it.
    4. Remaining ties go to the earlier root in (Re, Im) lexicographic order.
    Roots are "real" iff their imaginary part is exactly zero.
    """
    theta = np.asarray(theta, dtype=np.complex128)
    pos = [t for t in theta if t.imag > 0]
    neg = [t for t in theta if t.imag < 0]
    if len(pos) != len(neg):
        raise ValueError("roots are not closed under conjugation")
    cand = sorted([t for t in theta if t.imag >= 0], key=lambda t: (t.real, t.imag))
    if not cand:
        return theta[:0]
    # start: largest modulus, then larger Re, then Im > 0
    best = 0
    for i, t in enumerate(cand):
        b = cand[best]
        if (abs(t), t.real, t.imag > 0) > (abs(b), b.real, b.imag > 0):
            best = i
    order = []

    def take(i):
        t = cand.pop(i)
        order.append(t)
        if t.imag > 0:
            order.append(np.conj(t))

    take(best)
    while cand:
        scores = []
        for t in cand:
            dist = np.abs(t - np.asarray(order))
            scores.append(-np.inf if np.any(dist == 0) else float(np.sum(np.log(dist))))
        best = 0
        for i, sc in enumerate(scores):
            if sc > scores[best]:
                best = i
        take(best)
    return np.asarray(order, dtype=np.complex128)


def build_poly(A, v0, d):
    """Roots of the degree-d GMRES residual polynomial for (A, v0), in Leja order.

    Returns (roots, s): s <= d is the number of roots (s < d on a happy
    breakdown of Arnoldi, where the polynomial is then exact on the
    invariant subspace).
    """
    if d < 1:
        raise ValueError("d must be >= 1")
    _, Hbar, s = arnoldi(A, v0, d)
    theta = harmonic_ritz(Hbar)
    if not np.all(np.isfinite(theta)) or np.any(theta == 0):
        raise np.linalg.LinAlgError("zero or non-finite harmonic Ritz value")
    return leja_order(theta), s


def apply_poly(A, roots, v):
    """y = p(A) v evaluated one root at a time in complex arithmetic.

    With pi_k = prod_{i<=k} (1 - alpha/theta_i):
    p_k(alpha) = p_{k-1}(alpha) + pi_{k-1}(alpha)/theta_k, so
    y += prod/theta_k and then prod <- prod - A prod / theta_k.
    The result is real up to rounding for a conjugation-closed root set;
    its real part is returned (in v's real dtype).
    """
    v = np.asarray(v)
    ctype = np.result_type(v.dtype, np.complex64)
    roots = np.asarray(roots, dtype=ctype)
    prod = v.astype(ctype)
    y = np.zeros_like(prod)
    for k, th in enumerate(roots):
        y += prod / th
        if k + 1 < roots.size:
            prod = prod - matvec(A, prod) / th
    return y.real.astype(v.dtype)


def _power_gram(A, v0, deg):
    """W = [A v0, ..., A^(deg+1) v0]; returns (W^T W, W^T v0)."""
    v0 = np.asarray(v0, dtype=np.float64)
    cols = []
    v = v0
    for _ in range(deg + 1):
        v = matvec(A, v)
        cols.append(v)
    W = np.column_stack(cols)
    return W.T @ W, W.T @ v0


def _cholesky_solve(G, rhs):
    """Solve G y = rhs by LAPACK POTRF/POTRS; on POTRF failure at column k (info = k)
    solve with the leading (k-1) x (k-1) block and set the other coefficients to 0."""
    c, info = scipy.linalg.lapack.dpotrf(G, lower=0)
    if info < 0:
        raise ValueError("dpotrf argument error")
    k = G.shape[0] if info == 0 else info - 1
    y = np.zeros(G.shape[0])
    if k > 0:
        ck, info_k = scipy.linalg.lapack.dpotrf(G[:k, :k], lower=0)
        y[:k], _ = scipy.linalg.lapack.dpotrs(ck, rhs[:k], lower=0)
    return y, int(info)


def power_basis_poly(A, v0, deg):
    """The paper's construction (Section II, eqs. (1)-(2)).

    Builds V = [v0, A v0, ..., A^deg v0] and W = A V, and solves the normal
    equations (W^T W) y = W^T v0 with LAPACK POTRF/POTRS.  Returns (y, info):
    y[k] multiplies A^k in p(A) (degree deg), and info is POTRF's status.
    When POTRF reports that the Gram matrix is not numerically positive definite
    at column k (info = k > 0), the coefficients are still returned, as in the
    paper (Section IV): those of the leading (k-1) x (k-1) block, with zeros above
    -- the plateau of Table I, where the coefficients past the warning degree are
    negligible (below 1e-200).
    """
    G, rhs = _power_gram(A, v0, deg)
    return _cholesky_solve(G, rhs)


def auto_degree(A, v0, deg_max):
    """Section IV's heuristic: the highest degree whose Gram matrix factors without a
    POTRF warning.  The Gram matrices of degrees 0..deg_max are the leading blocks of
    the deg_max one; they are factored in increasing order and the scan stops at the
    first warning.  Returns (deg, y, info) with info the POTRF status of the first
    degree that warned (0 if none up to deg_max)."""
    G, rhs = _power_gram(A, v0, deg_max)
    last_ok, info_fail = 0, 0
    for k in range(1, deg_max + 2):
        c, info = scipy.linalg.lapack.dpotrf(G[:k, :k], lower=0)
        if info != 0:
            info_fail = int(info)
            break
        last_ok = k
    if last_ok == 0:
        raise np.linalg.LinAlgError("A v0 = 0: no polynomial")
    c, _ = scipy.linalg.lapack.dpotrf(G[:last_ok, :last_ok], lower=0)
    y, _ = scipy.linalg.lapack.dpotrs(c, rhs[:last_ok], lower=0)
    return last_ok - 1, y, info_fail


def apply_power(A, coeffs, v):
    """y = sum_k coeffs[k] A^k v, the powers formed one after the other (eq. (2))."""
    v = np.asarray(v)
    y = coeffs[0] * v
    pk = v
    for ck in coeffs[1:]:
        pk = matvec(A, pk)
        y = y + ck * pk
    return y
