"""Oracle: right-polynomial-preconditioned restarted GMRES(m) (test infrastructure).

The method of Section III: GMRES(m) whose Arnoldi step orthogonalises with
two unconditional passes of classical Gram-Schmidt (two block inner products
and one norm, counted as three "dots"), and the minimum-residual polynomial
used as a right preconditioner: solve A p(A) y = b, x = p(A) y.  The stopping
test is the relative residual ||b - A x|| / ||b|| < tol.

Readings taken where the paper is silent:
* the implicit least-squares residual |g_{j+1}| / ||b|| < tol ends a cycle
  early; convergence is decided by the true residual recomputed after the
  cycle's solution update (a cycle that stops on the implicit estimate but
  fails the true test restarts);
* iterations are counted as Arnoldi steps (Section V counts the iterations
  of GMRES(50) this way);
* attainable accuracy: once the true relative residual is below 100 * tol,
  three consecutive cycles that each end on the implicit estimate (it reached
  tol) but fail to reduce the true residual by 10% end the solve unconverged:
  the Krylov recurrence believes it has converged and the true residual no
  longer follows (its rounding floor).  A cycle that runs all m steps without
  its estimate reaching tol is slow convergence, not a floor, and never
  counts (Section VI's first example: GMRES(50) does converge, slowly);
* counters: per Arnoldi step d products with A (d-1 for p, one for A) and 3
  dots; per cycle end d-1 products for the update p(A) u, one for the new
  residual and one norm; the initial residual costs one product and one
  norm; building the polynomial costs d products and 3d+1 dots.

The least-squares problem min ||beta e1 - Hbar y|| is solved afresh at every
step by a complete QR factorisation of the small Hessenberg matrix (the
residual norm is |beta * Q[0, -1]|), which is slower than Givens rotations
but self-evidently correct.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .poly import BREAKDOWN_RTOL, apply_poly, apply_power, build_poly, matvec
from .rng import uniform_pm1

STAGNATION_BAND = 100.0    # the stagnation test applies below this multiple of tol
STAGNATION_FACTOR = 0.9    # a cycle must reduce the true residual at least this much
STAGNATION_CYCLES = 3      # consecutive failing cycles that end the solve

__all__ = ["GmresStats", "gmres_cycle", "pp_gmres", "pp_gmres_ir", "lsq_residual",
           "jacobi_left", "pp_gmres_left_jacobi"]


@dataclass
class GmresStats:
    converged: bool = False
    iters: int = 0          # Arnoldi steps
    restarts: int = 0       # cycles started after the first
    cycles: int = 0
    spmvs: int = 0
    dots: int = 0
    relres_true: float = float("nan")
    relres_implicit: float = float("nan")
    history: list = field(default_factory=list)       # implicit, per step
    true_history: list = field(default_factory=list)  # per cycle end
    roots: object = None
    nroots: int = 0


def lsq_residual(Hbar, beta):
    """Solve min_y ||beta e1 - Hbar y|| by complete QR; return (y, residual norm)."""
    k1, k = Hbar.shape
    Q, R = np.linalg.qr(Hbar, mode="complete")
    g = beta * Q[0, :]
    y = np.linalg.solve(R[:k, :k], g[:k])
    return y, abs(g[k])


def _precondition(A, roots, coeffs, v):
    if coeffs is not None:
        return apply_power(A, coeffs, v)
    return apply_poly(A, roots, v)


def gmres_cycle(A, r0, roots, m, tol_abs, max_steps, st: GmresStats, coeffs=None):
    """One GMRES cycle from residual r0 on the operator A p(A).

    Stops after m steps, after ``max_steps`` steps, on a happy breakdown, or
    when the implicit residual norm drops below ``tol_abs``.  Returns the
    solution update dx = p(A) V y (dtype of r0) and the implicit residual.
    Appends the implicit residual norm after every step to ``st.history``
    (divided by st._bnorm).
    """
    n = r0.size
    dt = r0.dtype
    d = (len(coeffs) if coeffs is not None else 0) or (0 if roots is None else len(roots))
    beta = float(np.linalg.norm(r0))
    V = np.zeros((n, m + 1), dtype=dt, order="F")
    V[:, 0] = r0 / beta
    H = np.zeros((m + 1, m))
    k = 0
    y = np.zeros(0)
    res = beta
    for j in range(min(m, max_steps)):
        z = _precondition(A, roots, coeffs, V[:, j]) if d else V[:, j]
        w = matvec(A, z)
        st.spmvs += max(d, 1)
        w0 = np.linalg.norm(w)
        Vj = V[:, : j + 1]
        h1 = Vj.T @ w
        w = w - Vj @ h1
        h2 = Vj.T @ w
        w = w - Vj @ h2
        st.dots += 3
        H[: j + 1, j] = np.asarray(h1, np.float64) + np.asarray(h2, np.float64)
        hn = float(np.linalg.norm(w))
        H[j + 1, j] = hn
        k = j + 1
        st.iters += 1
        y, res = lsq_residual(H[: k + 1, :k], beta)
        st.history.append(res / st._bnorm)
        if hn <= BREAKDOWN_RTOL * w0 or res < tol_abs:
            break
        V[:, j + 1] = w / hn
    u = V[:, :k] @ y.astype(dt)
    dx = _precondition(A, roots, coeffs, u) if d else u
    if d:
        st.spmvs += d - 1
    return dx, res


def pp_gmres(A, b, m, tol, roots=None, x0=None, max_iters=100000, v0=None, d=None,
             coeffs=None, v0_seed=0):
    """Restarted GMRES(m) with p(A) as right preconditioner.

    Either pass Leja-ordered ``roots`` (None or empty: no preconditioning), or
    a start vector ``v0`` and the number of roots ``d`` to build them, or the
    power-basis coefficients ``coeffs`` (p(A) = sum_k coeffs[k] A^k; degree
    len(coeffs)-1, so d = len(coeffs) products per step).  With ``d`` and no
    ``v0`` the polynomial is built from the seeded U(-1, 1) vector of
    ``rng.uniform_pm1(n, v0_seed)`` (Section V's random start vector).
    Works in b's dtype.  Returns (x, GmresStats).
    """
    st = GmresStats()
    b = np.asarray(b)
    dt = b.dtype
    if roots is None and d and v0 is None:
        v0 = uniform_pm1(b.size, v0_seed)
    if roots is None and d:
        roots, s = build_poly(A, np.asarray(v0, dtype=dt), d)
        st.spmvs += s
        st.dots += 3 * s + 1
    if roots is not None and len(roots) == 0:
        roots = None
    st.roots = roots
    st.nroots = len(coeffs) if coeffs is not None else (0 if roots is None else len(roots))
    st._bnorm = float(np.linalg.norm(b))
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=dt).copy()
    r = b - matvec(A, x)
    st.spmvs += 1
    st.dots += 1
    beta = float(np.linalg.norm(r))
    st.relres_true = beta / st._bnorm
    st.true_history.append(st.relres_true)
    stagnant = 0
    while st.relres_true >= tol and st.iters < max_iters and stagnant < STAGNATION_CYCLES:
        prev = st.relres_true
        st.cycles += 1
        dx, res = gmres_cycle(A, r, roots, m, tol * st._bnorm, max_iters - st.iters, st,
                              coeffs=coeffs)
        st.relres_implicit = res / st._bnorm
        x = x + dx
        r = b - matvec(A, x)
        st.spmvs += 1
        st.dots += 1
        st.relres_true = float(np.linalg.norm(r)) / st._bnorm
        st.true_history.append(st.relres_true)
        if not np.isfinite(st.relres_true):
            break
        if (res < tol * st._bnorm and st.relres_true < STAGNATION_BAND * tol
                and st.relres_true > STAGNATION_FACTOR * prev):
            stagnant += 1
        else:
            stagnant = 0
    st.restarts = max(st.cycles - 1, 0)
    st.converged = bool(st.relres_true < tol)
    return x, st


def pp_gmres_ir(A, b, m, d, tol, v0, inner_tol=None, max_outer=200, x0=None, v0_seed=0):
    """FP32 inner PP-GMRES inside an FP64 iterative-refinement loop.

    Outer loop (float64): r = b - A x; stop when ||r||/||b|| < tol; otherwise
    solve A p32(A32) y = r/||r|| with ONE float32 GMRES cycle of at most m
    steps that stops early at implicit relative residual < tau, and update
    x += ||r|| * p32(A32) V y (update accumulated in float64).  tau is
    inner_tol when given; inner_tol = None takes tau = max(1e-5, 0.5 tol /
    (||r||/||b||)): 1e-5, loosened on a step that needs less, so the last inner
    cycle stops near the reduction still missing (with a factor-2 margin).
    The float32 polynomial is built once, from a float32 Arnoldi on
    float32(v0); its roots come from the float64 eigen-solve of that Hessenberg.
    v0 = None draws the seeded vector ``rng.uniform_pm1(n, v0_seed)``.
    Returns (x, GmresStats) with ``st.outer`` = number of refinement steps.
    """
    import scipy.sparse as sp
    b = np.asarray(b, dtype=np.float64)
    if v0 is None and d:
        v0 = uniform_pm1(b.size, v0_seed)
    A32 = (sp.csr_matrix(A, dtype=np.float32) if sp.issparse(A)
           else np.asarray(A, dtype=np.float32))
    st = GmresStats()
    st._bnorm = float(np.linalg.norm(b))
    roots = None
    if d:
        roots, s = build_poly(A32, np.asarray(v0, dtype=np.float32), d)
        st.spmvs += s
        st.dots += 3 * s + 1
    st.roots = roots
    st.nroots = 0 if roots is None else len(roots)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    st.outer = 0
    inner = GmresStats()
    inner._bnorm = 1.0
    for _ in range(max_outer):
        r = b - matvec(A, x)
        st.spmvs += 1
        st.dots += 1
        rn = float(np.linalg.norm(r))
        st.relres_true = rn / st._bnorm
        st.true_history.append(st.relres_true)
        if st.relres_true < tol or not np.isfinite(rn):
            break
        r32 = (r / rn).astype(np.float32)
        tau = inner_tol if inner_tol is not None else max(1e-5, 0.5 * tol / st.relres_true)
        dx, res = gmres_cycle(A32, r32, roots, m, tau * float(np.linalg.norm(r32)), m, inner)
        x = x + rn * dx.astype(np.float64)
        st.outer += 1
    st.iters = inner.iters
    st.spmvs += inner.spmvs
    st.dots += inner.dots
    st.history = inner.history
    st.cycles = st.outer
    st.converged = bool(st.relres_true < tol)
    return x, st


def jacobi_left(A, b):
    """The left-preconditioned system D^{-1} A x = D^{-1} b with D = diag(A)."""
    import scipy.sparse as sp
    d = np.asarray(A.diagonal(), dtype=np.float64)
    if np.any(d == 0) or not np.all(np.isfinite(d)):
        raise np.linalg.LinAlgError("zero or non-finite diagonal")
    Dinv = sp.diags(1.0 / d)
    return sp.csr_matrix(Dinv @ A), np.asarray(b, dtype=np.float64) / d


def pp_gmres_left_jacobi(A, b, m, tol, v0=None, d=None, max_iters=100000):
    """Polynomial preconditioning composed with a left Jacobi preconditioner.

    Section II: with a preconditioned system M A x = M b the polynomial is built
    for the operator M A.  Here M = D^{-1}: GMRES(m) runs on D^{-1} A p(D^{-1} A) y
    = D^{-1} b, x = p(D^{-1} A) y, and stops on the preconditioned relative residual
    ||D^{-1}(b - A x)|| / ||D^{-1} b|| < tol.  Returns (x, stats) with
    ``stats.relres_original`` = ||b - A x|| / ||b||.
    """
    As, bs = jacobi_left(A, b)
    x, st = pp_gmres(As, bs, m, tol, v0=v0, d=d, max_iters=max_iters)
    st.relres_original = float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))
    return x, st
