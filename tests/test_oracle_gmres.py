"""Pins of the oracle's PP-GMRES(m) and its FP32 iterative-refinement loop.

Pinned against: the numbers printed for the Laplacian example of Section V
(tests/golden/sec5_laplacian.json), dense direct solves, finite termination
of full GMRES, monotone residuals, and the counting convention of Section III
(three dots per iteration).
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import gmres, poly
from paper_1907_00072_amd import workloads as W


@pytest.fixture(scope="module")
def sec5(golden_dir):
    return json.load(open(os.path.join(golden_dir, "sec5_laplacian.json")))


@pytest.fixture(scope="module")
def lap():
    A = W.laplacian5(201)
    return A.to_scipy(), np.ones(A.n)


def _alpha_p(roots, alpha):
    return 1.0 - np.prod([1.0 - alpha / t for t in roots], axis=0).real


def test_sec5_bad_polynomial_from_b(sec5, lap):
    A, b = lap
    assert A.shape[0] == 40401
    roots, s = poly.build_poly(A, b, sec5["roots"])
    al = np.linspace(0.0, 8.0, 40001)
    lo = _alpha_p(roots, al).min()
    ref = sec5["v0_equals_b"]["min_alpha_p_alpha_on_0_8"]
    assert ref - 50 <= lo <= ref + 50, lo


@pytest.mark.slow
def test_sec5_stall_after_2550_iterations(sec5, lap):
    A, b = lap
    roots, s = poly.build_poly(A, b, sec5["roots"])
    x, st = gmres.pp_gmres(A, b, sec5["m"], sec5["tol"], roots=roots, max_iters=2550)
    assert st.iters == 2550 and not st.converged
    ref = sec5["v0_equals_b"]["relres_after_2550_iterations"]
    assert abs(st.relres_true - ref) <= 0.005, st.relres_true


def test_sec5_random_start_vector(sec5, lap):
    A, b = lap
    v0 = W.uniform(A.shape[0], 0)
    x, st = gmres.pp_gmres(A, b, sec5["m"], sec5["tol"], v0=v0, d=sec5["roots"], max_iters=400)
    ref = sec5["random_v0_uniform_m1_1"]["iterations_to_tol"]
    assert st.converged and abs(st.iters - ref) <= 4, st.iters
    lo, hi = sec5["random_v0_uniform_m1_1"]["alpha_p_alpha_range_on_bulk"]
    vals = _alpha_p(st.roots, np.linspace(0.5, 8.0, 20001))
    assert vals.min() >= lo and vals.max() <= hi


def test_full_gmres_terminates_and_matches_dense_solve():
    n = 40
    rng = np.random.default_rng(31)
    A = rng.standard_normal((n, n)) / np.sqrt(n) + 2 * np.eye(n)
    b = rng.standard_normal(n)
    x, st = gmres.pp_gmres(A, b, m=n, tol=1e-13)
    assert st.cycles == 1 and st.iters <= n
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_polynomial_gmres_matches_dense_solve():
    n = 60
    rng = np.random.default_rng(32)
    A = rng.standard_normal((n, n)) / np.sqrt(n) + 2 * np.eye(n)
    b = rng.standard_normal(n)
    x, st = gmres.pp_gmres(A, b, m=10, tol=1e-12, v0=W.uniform(n, 33), d=5, max_iters=200)
    ref = np.linalg.solve(A, b)
    assert st.converged
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("d", [0, 10])
def test_config1_solution_and_monotone_residuals(d):
    P = W.config(1)
    A = P.A.to_scipy()
    x, st = gmres.pp_gmres(A, P.b, P.m, P.tol, v0=P.v0, d=d, max_iters=1000)
    assert st.converged
    assert np.linalg.norm(P.b - A @ x) / np.linalg.norm(P.b) < P.tol
    ref = spla.spsolve(A.tocsc(), P.b)
    # forward error <= cond * tol; cond(A) of this operator is ~1e3
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-4
    h = np.asarray(st.history)
    # the implicit residual never increases inside a cycle; the true one never across cycles
    starts = np.cumsum([0] + [P.m] * (st.cycles - 1))
    for c0 in starts:
        seg = h[c0:c0 + P.m]
        assert np.all(np.diff(seg) <= 1e-12 * seg[:-1])
    th = np.asarray(st.true_history)
    assert np.all(np.diff(th) <= 1e-10 * th[:-1])


def test_polynomial_reduces_iterations_and_dots():
    P = W.config(1)
    A = P.A.to_scipy()
    _, s0 = gmres.pp_gmres(A, P.b, P.m, P.tol, max_iters=1000)
    _, s1 = gmres.pp_gmres(A, P.b, P.m, P.tol, v0=P.v0, d=P.d, max_iters=1000)
    assert s1.iters * 5 < s0.iters
    assert s1.dots * 5 < s0.dots


def test_counting_convention():
    """Section III: three dots per Arnoldi step; d products with A per preconditioned step."""
    P = W.config(1)
    A = P.A.to_scipy()
    for d in (0, 10):
        _, st = gmres.pp_gmres(A, P.b, P.m, P.tol, v0=P.v0, d=d, max_iters=1000)
        s = st.nroots
        build_spmv = s
        build_dots = 3 * s + 1 if d else 0
        per_step = max(s, 1)
        cyc = st.cycles
        assert st.spmvs == build_spmv + 1 + st.iters * per_step + cyc * (max(s - 1, 0) + 1)
        assert st.dots == build_dots + 1 + 3 * st.iters + cyc


def test_single_cycle_implicit_equals_true_residual():
    n = 200
    rng = np.random.default_rng(34)
    A = rng.standard_normal((n, n)) / np.sqrt(n) + 3 * np.eye(n)
    b = rng.standard_normal(n)
    x, st = gmres.pp_gmres(A, b, m=15, tol=1e-30, max_iters=15)
    assert st.cycles == 1 and st.iters == 15
    assert abs(st.relres_implicit - st.relres_true) <= 1e-9 * st.relres_true


def test_iterative_refinement_fp32_inner():
    P = W.config(1)
    A = P.A.to_scipy()
    x, st = gmres.pp_gmres_ir(A, P.b, P.m, P.d, 1e-10, P.v0, max_outer=20)
    assert st.converged and st.relres_true < 1e-10
    assert st.outer >= 2            # one FP32 cycle cannot reach 1e-10 alone
    ref = spla.spsolve(A.tocsc(), P.b)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-6
    # the float32 polynomial is close to (but not the same as) the float64 one
    r64, _ = poly.build_poly(A, P.v0, P.d)
    assert np.max(np.abs(np.sort(st.roots.real) - np.sort(r64.real)) / np.abs(np.sort(r64.real))) < 1e-3


def test_iterative_refinement_automatic_inner_stop():
    """inner_tol = None: each inner cycle stops once its implicit residual drops
    below tau_k = max(1e-5, 0.5 tol / relres_k) (relative to ||r_k||).  Checked
    against runs with that tau fixed: the first refinement step (relres_0 = 1)
    is the fixed 1e-5 run's first step, and a second step near tol stops at the
    looser tau, so the automatic run takes fewer inner steps and still converges."""
    P = W.config(1)
    A = P.A.to_scipy()
    tol = 1e-8
    xa, sa = gmres.pp_gmres_ir(A, P.b, P.m, P.d, tol, P.v0, max_outer=20)
    xf, sf = gmres.pp_gmres_ir(A, P.b, P.m, P.d, tol, P.v0, inner_tol=1e-5, max_outer=20)
    assert sa.converged and sf.converged and sa.outer >= 2
    # both start with the same step: same polynomial, same first inner cycle
    assert sa.true_history[:2] == sf.true_history[:2]
    # the automatic second inner cycle stops at its own tau, never below it
    tau1 = max(1e-5, 0.5 * tol / sa.true_history[1])
    assert tau1 > 1e-5
    _, s1 = gmres.pp_gmres_ir(A, P.b, P.m, P.d, tol, P.v0, inner_tol=1e-5, max_outer=1)
    k1 = s1.iters                        # inner steps of the first refinement step
    second = sa.history[k1:]
    assert second[-1] < tau1 and (len(second) == 1 or second[-2] >= tau1)
    assert sa.iters < sf.iters


@pytest.mark.parametrize("cfg,N", [(1, None), (4, 128)])
def test_iterative_refinement_inner_arithmetic_is_fp32(cfg, N):
    """The refinement's inner cycle and its polynomial run in FP32, not FP64.

    Pinned by attainable accuracy: a GMRES cycle computed in a precision with
    unit roundoff u cannot leave a true residual much below u (times modest
    growth), however small its implicit estimate gets.  With inner_tol = 1e-14
    one refinement step therefore stops near FP32's u = 6e-8, while the same
    cycle (same roots, same m) in FP64 goes below 1e-12: a float64 inner cycle
    would fail the lower bound.  The FP32-built roots differ from the FP64-built
    ones by FP32 rounding, far above FP64's: a float64 Arnoldi would fail it.
    """
    P = W.config(cfg, N=N) if N else W.config(cfg)
    A = P.A.to_scipy()
    x, st = gmres.pp_gmres_ir(A, P.b, P.m, P.d, 1e-30, P.v0, inner_tol=1e-14, max_outer=1)
    assert st.outer == 1 and st.history[-1] < 1e-12      # the implicit estimate went low
    rr = np.linalg.norm(P.b - A @ x) / np.linalg.norm(P.b)
    assert 1e-8 < rr < 1e-4, rr
    _, s64 = gmres.pp_gmres(A, P.b, P.m, 1e-14, roots=st.roots, max_iters=P.m)
    assert s64.relres_true < 1e-12, s64.relres_true
    r64, _ = poly.build_poly(A, P.v0, P.d)
    a, b = np.sort_complex(st.roots), np.sort_complex(r64)
    diff = np.max(np.abs(a - b) / np.abs(b))
    assert 1e-9 < diff < 1e-3, diff


def test_left_jacobi_composition():
    """Section II composition: the polynomial built for D^-1 A; solution equals A^-1 b."""
    import scipy.sparse as sp
    Ah = W.random_csr(300, 8, seed=50, diag_shift=0.0)
    A = Ah.to_scipy()
    dg = np.random.default_rng(51).uniform(2.0, 400.0, 300)      # widely varying diagonal
    A = sp.csr_matrix(A + sp.diags(dg - A.diagonal()))
    b = W.normal(300, 52)
    As, bs = gmres.jacobi_left(A, b)
    assert np.allclose(As.diagonal(), 1.0)
    x, st = gmres.pp_gmres_left_jacobi(A, b, 20, 1e-12, v0=W.uniform(300, 53), d=6, max_iters=500)
    ref = np.linalg.solve(A.toarray(), b)
    assert st.converged and np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
    # the row scaling makes this problem far easier than the unscaled one
    _, st0 = gmres.pp_gmres(A, b, 20, 1e-12, v0=W.uniform(300, 53), d=6, max_iters=500)
    assert st.iters < st0.iters


def test_stagnation_at_attainable_accuracy_ends_the_solve():
    """A tolerance below the FP64 floor ends on the stagnation test, not the iteration cap."""
    P = W.config(1, N=32)
    A = P.A.to_scipy()
    x, st = gmres.pp_gmres(A, P.b, 20, 1e-16, v0=P.v0, d=6, max_iters=5000)
    assert not st.converged and st.iters < 1000
    assert st.relres_true < 1e-14
    th = np.asarray(st.true_history)
    assert np.all(th[-3:] > 0.9 * th[-4:-1])


def test_slow_convergence_near_tol_is_not_taken_for_stagnation():
    """GMRES(5) on the eps = 1/2 recirculating flow (Section VI's first example, which
    converges without a preconditioner) gains less than 10% per cycle for dozens of
    cycles just above tol.  Those cycles run all m steps without their estimate
    reaching tol, so the attainable-accuracy rule must not end the solve."""
    A, b = W.recirculating_flow(33, 0.5)
    x, st = gmres.pp_gmres(A.to_scipy(), b, 5, 1e-8, max_iters=60000)
    assert st.converged
    th = np.asarray(st.true_history)
    slow = (th[1:] > 0.9 * th[:-1]) & (th[1:] < 1e-6)
    run = best = 0
    for v in slow:
        run = run + 1 if v else 0
        best = max(best, run)
    assert best >= 3, best
