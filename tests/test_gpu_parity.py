"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances.  FP64 p(A)v: each chain step adds O(u) relative rounding to the
running product and accumulator, so after d-1 steps the relative error is
bounded by about c*d*u*growth, with growth = max_k ||prod_k|| * sum|c_k| /
||y|| of order 10-100 on these problems: 1e-12 leaves a wide margin while
still catching any wrong index, coefficient or tile boundary (those give O(1)
errors).  FP32: the same bound with u = 6e-8 gives the 1e-4 used.  Solves
follow the parity rule of the method's readings: iteration counts within 2%
and, when the counts agree, ||x_gpu - x_oracle|| / ||x_oracle|| <= 1e-8.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import adjoint as oadj
from oracle import gmres as ogmres
from oracle import poly as opoly
from paper_1907_00072_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_00072_amd import binding
    binding.lib()  # raises if the library was not built
    return binding


def _up(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda:0", dtype=dtype)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _matrix(name):
    if name == "cd2d_32":
        return W.config(1, N=32).A
    if name == "cd3d_16_pe50":
        return W.config(2, N=16).A
    if name == "rand_777":
        return W.random_csr(777, 12, seed=5, diag_shift=4.0)
    if name == "rand_longrows_600":
        return W.random_csr(600, 400, seed=6, diag_shift=30.0)
    if name == "rand_5":
        return W.random_csr(5, 3, seed=7, diag_shift=3.0)
    if name == "one":
        return W.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.5]))
    raise KeyError(name)


APPLY_CASES = [("cd2d_32", 10), ("cd3d_16_pe50", 12), ("rand_777", 9), ("rand_longrows_600", 7),
               ("rand_5", 5), ("one", 1)]


LAYOUTS = ["csr", "sell"]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("name,d", APPLY_CASES)
def test_apply_matches_oracle_fp64(B, name, d, layout):
    Ah = _matrix(name)
    As = Ah.to_scipy()
    roots, s = opoly.build_poly(As, W.uniform(Ah.n, 11), d)
    A = B.CSRMatrix.from_host(Ah, layout=layout)
    p = B.pp_poly_from_roots(Ah.n, roots)
    for seed in (1, 2):
        v = W.uniform(Ah.n, seed)
        y = B.pp_apply(A, p, _up(v)).cpu().numpy()
        assert _rel(y, opoly.apply_poly(As, roots, v)) <= 1e-12, name


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("name,d", APPLY_CASES)
def test_apply_matches_oracle_fp32(B, name, d, layout):
    Ah = _matrix(name)
    As = Ah.to_scipy()
    roots, s = opoly.build_poly(As, W.uniform(Ah.n, 11), d)
    A = B.CSRMatrix.from_host(Ah, dtype=torch.float32, layout=layout)
    p = B.pp_poly_from_roots(Ah.n, roots, dtype="f32")
    v = W.uniform(Ah.n, 3)
    y = B.pp_apply(A, p, _up(v, torch.float32)).cpu().numpy().astype(np.float64)
    assert _rel(y, opoly.apply_poly(As, roots, v)) <= 1e-4, name


# every chain-kernel variant: real step, folded last real after a real step,
# folded last real after a pair, a pair as the last step, a single real root
ROOT_SETS = {
    "single_real": [4.0],
    "two_real_fold": [4.0, 2.5],
    "real_then_last_pair": [5.0, 2.0 + 1.0j, 2.0 - 1.0j],
    "pair_then_last_real": [2.0 + 1.0j, 2.0 - 1.0j, 5.0],
    "two_pairs": [2.0 + 1.0j, 2.0 - 1.0j, 3.0 + 0.5j, 3.0 - 0.5j],
    "mixed": [6.0, 1.5 + 2.0j, 1.5 - 2.0j, 3.0, 4.0 + 0.3j, 4.0 - 0.3j, 2.0],
}


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("key", list(ROOT_SETS))
def test_apply_chain_variants(B, key, layout):
    Ah = W.random_csr(1000, 8, seed=12, diag_shift=4.0)
    As = Ah.to_scipy()
    roots = np.array(ROOT_SETS[key], dtype=complex)
    A = B.CSRMatrix.from_host(Ah, layout=layout)
    p = B.pp_poly_from_roots(Ah.n, roots)
    v = W.uniform(Ah.n, 13)
    y = B.pp_apply(A, p, _up(v)).cpu().numpy()
    assert _rel(y, opoly.apply_poly(As, roots, v)) <= 1e-12, key


@pytest.mark.parametrize("layout", LAYOUTS)
def test_apply_with_empty_rows(B, layout):
    n = 700
    rng = np.random.default_rng(14)
    counts = rng.integers(0, 4, n)
    counts[::7] = 0
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum(counts)
    ci = np.concatenate([np.sort(rng.choice(n, c, replace=False)) for c in counts]).astype(np.int32)
    va = rng.uniform(-1, 1, ci.size)
    Ah = W.CSR(n, rp, ci, va)
    roots = np.array([3.0, 1.0 + 1.0j, 1.0 - 1.0j, -2.0])
    p = B.pp_poly_from_roots(n, roots)
    v = W.uniform(n, 15)
    y = B.pp_apply(B.CSRMatrix.from_host(Ah, layout=layout), p, _up(v)).cpu().numpy()
    assert _rel(y, opoly.apply_poly(Ah.to_scipy(), roots, v)) <= 1e-12


def _match_sets(a, b):
    a = sorted(np.asarray(a, complex), key=lambda t: (t.real, t.imag))
    b = sorted(np.asarray(b, complex), key=lambda t: (t.real, t.imag))
    return max(abs(x - y) / abs(y) for x, y in zip(a, b))


@pytest.mark.parametrize("name,d", [("cd2d_32", 10), ("cd3d_16_pe50", 12), ("rand_777", 8)])
def test_build_poly_matches_oracle(B, name, d):
    Ah = _matrix(name)
    v0 = W.uniform(Ah.n, 21)
    ref, s = opoly.build_poly(Ah.to_scipy(), v0, d)
    p = B.pp_build_poly(B.CSRMatrix.from_host(Ah), _up(v0), d)
    got = p.roots()
    assert got.size == ref.size == d
    assert _match_sets(got, ref) <= 1e-8


def test_build_poly_degree_reduced(B):
    a = np.array([1.0, 2.0, 4.0] * 100)
    n = a.size
    Ah = W.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), a)
    with pytest.warns(B.PPWarning):
        p = B.pp_build_poly(B.CSRMatrix.from_host(Ah), _up(W.uniform(n, 1)), 6)
    r = np.sort(p.roots().real)
    assert r.size == 3 and np.allclose(r, [1.0, 2.0, 4.0], rtol=1e-10)


def _solve_both(B, Ah, b, v0, m, d, tol, max_iters=5000, op_form="pi", layout="auto"):
    A = B.CSRMatrix.from_host(Ah, layout=layout)
    x, st = B.pp_gmres_solve(A, _up(b), m=m, d=d, tol=tol, v0=_up(v0), max_iters=max_iters,
                             op_form=op_form)
    xo, so = ogmres.pp_gmres(Ah.to_scipy(), b, m, tol, v0=v0, d=d, max_iters=max_iters)
    return x.cpu().numpy(), st, xo, so


def _assert_parity(st, so, xg, xo, tol):
    assert st.relres_true < tol and so.converged
    assert abs(st.iters - so.iters) <= max(1, round(0.02 * so.iters)), (st.iters, so.iters)
    if st.iters == so.iters:
        assert _rel(xg, xo) <= 1e-8
        assert st.spmvs == so.spmvs and st.dots == so.dots


@pytest.mark.parametrize("d,op_form", [(10, "pi"), (10, "p"), (0, "pi"), (4, "pi"), (1, "pi"),
                                       (1, "p")])
def test_solve_config1_full(B, d, op_form):
    P = W.config(1)
    xg, st, xo, so = _solve_both(B, P.A, P.b, P.v0, P.m, d, P.tol, op_form=op_form)
    _assert_parity(st, so, xg, xo, P.tol)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_solve_cd3d_ragged_tiles(B, layout):
    P = W.config(2, N=23)   # n = 12167: 48 full tiles and a ragged one (190 slices, last partial)
    xg, st, xo, so = _solve_both(B, P.A, P.b, P.v0, P.m, 10, P.tol, layout=layout)
    _assert_parity(st, so, xg, xo, P.tol)
    assert st.layout_used == layout


@pytest.mark.parametrize("op_form,layout", [("pi", "auto"), ("p", "auto"), ("pi", "sell")])
def test_solve_complex_roots(B, op_form, layout):
    Ah = W.random_csr(777, 12, seed=5, diag_shift=4.0)
    b = W.normal(777, 3)
    v0 = W.uniform(777, 4)
    roots, _ = opoly.build_poly(Ah.to_scipy(), v0, 6)
    assert np.any(roots.imag != 0)
    xg, st, xo, so = _solve_both(B, Ah, b, v0, 20, 6, 1e-10, op_form=op_form, layout=layout)
    _assert_parity(st, so, xg, xo, 1e-10)


@pytest.mark.parametrize("op_form", ["pi", "p"])
def test_solve_all_complex_roots_cd3d(B, op_form):
    P = W.config(2, N=24)   # mesh Peclet ~1: all but one of the 25 roots are complex
    roots, _ = opoly.build_poly(P.A.to_scipy(), P.v0, 25)
    assert np.sum(roots.imag != 0) == 24
    xg, st, xo, so = _solve_both(B, P.A, P.b, P.v0, P.m, 25, P.tol, op_form=op_form)
    _assert_parity(st, so, xg, xo, P.tol)


def test_solve_is_bitwise_deterministic(B):
    P = W.config(1, N=40)
    A = B.CSRMatrix.from_host(P.A)
    xs = []
    for _ in range(2):
        x, st = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=P.d, tol=P.tol, v0=_up(P.v0))
        xs.append(x.cpu().numpy())
    assert np.array_equal(xs[0], xs[1])


def test_solve_reuses_given_polynomial(B):
    P = W.config(1, N=40)
    A = B.CSRMatrix.from_host(P.A)
    p = B.pp_build_poly(A, _up(P.v0), P.d)
    x1, s1 = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=P.d, tol=P.tol, v0=_up(P.v0))
    x2, s2 = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=0, tol=P.tol, poly=p)
    assert s1.iters == s2.iters and np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    assert s2.nroots == P.d


def test_iterative_refinement_fp32(B):
    P = W.config(1)
    A = B.CSRMatrix.from_host(P.A)
    x, st = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=P.d, tol=1e-10, v0=_up(P.v0),
                             precision="f32_ir")
    xo, so = ogmres.pp_gmres_ir(P.A.to_scipy(), P.b, P.m, P.d, 1e-10, P.v0, max_outer=50)
    x64, s64 = ogmres.pp_gmres(P.A.to_scipy(), P.b, P.m, 1e-12, v0=P.v0, d=P.d, max_iters=5000)
    xg = x.cpu().numpy()
    assert st.relres_true < 1e-10 and so.converged
    assert abs(st.outer - so.outer) <= 1
    if st.outer == so.outer:  # the automatic inner stop: inner step totals within 2%
        assert abs(st.iters - so.iters) <= max(1, round(0.02 * so.iters)), (st.iters, so.iters)
    # forward error against the FP64 oracle solution: both are within cond * tol of it
    assert _rel(xg, x64) <= 1e-7 and _rel(xo, x64) <= 1e-7


def test_warnings_and_errors(B):
    P = W.config(1, N=32)
    A = B.CSRMatrix.from_host(P.A)
    with pytest.warns(B.PPWarning):
        x, st = B.pp_gmres_solve(A, _up(P.b), m=10, d=0, tol=1e-12, max_iters=15)
    assert st.status == B.PP_WARN_NOT_CONVERGED and st.iters == 15
    with pytest.raises(B.PPError):
        B.pp_gmres_solve(A, _up(P.b), m=0, d=4, tol=1e-8)
    bad = P.b.copy()
    bad[5] = np.nan
    with pytest.raises(B.PPError):
        B.pp_gmres_solve(A, _up(bad), m=10, d=4, tol=1e-8, v0=_up(P.v0))


@pytest.mark.parametrize("name", ["cd2d_32", "rand_777", "rand_longrows_600"])
def test_transpose_and_grad(B, name):
    Ah = _matrix(name)
    A = B.CSRMatrix.from_host(Ah)
    At = B.pp_csr_transpose(A)
    ref = sp.csr_matrix(Ah.to_scipy().T)
    ref.sort_indices()
    assert np.array_equal(At.row_ptr.cpu().numpy(), ref.indptr)
    assert np.array_equal(At.col_ind.cpu().numpy(), ref.indices)
    assert np.array_equal(At.vals.cpu().numpy(), ref.data)
    lam = W.normal(Ah.n, 1)
    x = W.normal(Ah.n, 2)
    g = B.pp_csr_grad(A, _up(lam), _up(x)).cpu().numpy()
    rows = oadj.csr_rows(Ah.row_ptr)
    assert np.array_equal(g, -lam[rows] * x[Ah.col_ind])


def test_transpose_with_duplicates_is_deterministic(B):
    # duplicate (i, j) entries: the transpose keeps them in A's order, on every call
    rng = np.random.default_rng(41)
    n = 300
    rows = np.sort(rng.integers(0, n, 4000))
    cols = rng.integers(0, n, 4000)
    cols[1::9] = cols[::9][: cols[1::9].size]  # plenty of repeats inside rows
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    vals = rng.standard_normal(rows.size)
    Ah = W.CSR(n, rp, cols.astype(np.int32), vals)
    A = B.CSRMatrix.from_host(Ah)
    # the reference: entries ordered by column, ties by their position in A
    k = np.argsort(cols, kind="stable")
    ref_rp = np.zeros(n + 1, np.int64)
    np.add.at(ref_rp, cols + 1, 1)
    ref_rp = np.cumsum(ref_rp)
    for _ in range(3):
        At = B.pp_csr_transpose(A)
        assert np.array_equal(At.row_ptr.cpu().numpy(), ref_rp)
        assert np.array_equal(At.col_ind.cpu().numpy(), rows[k])
        assert np.array_equal(At.vals.cpu().numpy(), vals[k])


def test_malformed_csr_is_rejected_before_any_product(B):
    P = W.config(1, N=16)
    n = P.A.n
    b, v0 = _up(P.b), _up(P.v0)
    bad_col = P.A.col_ind.copy()
    bad_col[17] = n            # one column past the end
    neg_col = P.A.col_ind.copy()
    neg_col[3] = -1
    bad_rp = P.A.row_ptr.copy()
    bad_rp[40] = bad_rp[42]    # row_ptr decreasing at row 41
    short_rp = P.A.row_ptr.copy()
    short_rp[-1] -= 1          # row_ptr[n] != nnz
    for rp, ci in ((P.A.row_ptr, bad_col), (P.A.row_ptr, neg_col), (bad_rp, P.A.col_ind),
                   (short_rp, P.A.col_ind)):
        A = B.CSRMatrix.from_host(W.CSR(n, rp, ci, P.A.vals), validate=False)
        calls = (lambda: B.pp_gmres_solve(A, b, m=10, d=4, tol=1e-8, v0=v0),
                 lambda: B.pp_build_poly(A, v0, 4),
                 lambda: B.pp_apply(A, B.pp_poly_from_roots(n, [2.0, 3.0]), v0),
                 lambda: B.pp_csr_transpose(A),
                 lambda: B.pp_csr_grad(A, v0, b),
                 lambda: B.pp_build_poly_power(A, v0, 3))
        for call in calls:
            with pytest.raises(B.PPError) as e:
                call()
            assert e.value.code == B.PP_ERR_ARG


def test_adjoint_gradient_reduced_config4(B):
    from paper_1907_00072_amd.autograd import SolveConfig, pp_solve
    P = W.config(4, N=48)
    Ah = P.A
    xt = P.extra["x_target"]
    pattern = B.CSRMatrix.from_host(Ah)
    vals = _up(Ah.vals).requires_grad_(True)
    b = _up(P.b).requires_grad_(True)
    cfg = SolveConfig(m=P.m, d=P.d, tol=P.tol, v0=_up(P.v0), adj_v0=_up(P.extra["v0_adjoint"]))
    x = pp_solve(pattern, vals, b, cfg)
    loss = 0.5 * ((x - _up(xt)) ** 2).sum()
    loss.backward()
    gv = vals.grad.cpu().numpy()
    gb = b.grad.cpu().numpy()
    M = Ah.to_scipy()
    _, lam, gb_ref, gv_ref = oadj.adjoint_gradient(M, P.b, xt)
    assert np.max(np.abs(gv - gv_ref)) <= 1e-6 * np.max(np.abs(gv_ref))
    assert np.max(np.abs(gb - gb_ref)) <= 1e-6 * np.max(np.abs(gb_ref))
    ents = np.random.default_rng(6).choice(Ah.nnz, 16, replace=False)
    fd = oadj.fd_gradient_vals(M, P.b, xt, ents, h=1e-6)
    assert np.max(np.abs(gv[ents] - fd)) <= 1e-6 * np.max(np.abs(gv_ref))
    assert [ph for ph, _ in cfg.stats] == ["forward", "adjoint"]


# ---- the paper's power-basis construction (Section II eqs. (1)-(2), Section IV)
# Coefficient agreement is limited by the conditioning of the Gram matrix
# (cond 5e2, 2e5, 4e7, 2e12 at degrees 1, 2, 3, 5 on the 64^2 problem): rounding
# in the Gram entries moves the coefficients by about u * cond.
@pytest.mark.parametrize("deg,coef_tol", [(1, 1e-10), (2, 1e-9), (3, 1e-8), (5, 1e-6)])
def test_power_basis_build_and_apply(B, deg, coef_tol):
    P = W.config(1)
    As = P.A.to_scipy()
    A = B.CSRMatrix.from_host(P.A)
    p, info = B.pp_build_poly_power(A, _up(P.v0), deg)
    c = B.pp_poly_coeffs(p)
    ref, info_ref = opoly.power_basis_poly(As, P.v0, deg)
    assert info == info_ref == 0 and c.size == deg + 1
    assert np.max(np.abs(c - ref) / np.abs(ref)) <= coef_tol
    v = W.uniform(P.A.n, 31)
    y = B.pp_apply(A, p, _up(v)).cpu().numpy()
    assert _rel(y, opoly.apply_power(As, c, v)) <= 1e-10   # Horner vs explicit powers
    obj = np.linalg.norm(P.v0 - As @ opoly.apply_power(As, c, P.v0))
    obj_ref = np.linalg.norm(P.v0 - As @ opoly.apply_power(As, ref, P.v0))
    assert abs(obj - obj_ref) <= 1e-10 * obj_ref


def test_power_basis_auto_degree_bidiag(B):
    Ac = W.bidiag2()
    As = Ac.to_scipy()
    b = As @ np.random.default_rng(1).random(Ac.n)
    p, info = B.pp_build_poly_power(B.CSRMatrix.from_host(Ac), _up(b), 18, auto_degree=True)
    deg_ref, y_ref, info_ref = opoly.auto_degree(As, b, 18)
    c = B.pp_poly_coeffs(p)
    # the onset sits where the Gram matrix loses definiteness in the last digits, so
    # the two Gram matrices (different summation orders) may disagree by one degree
    assert abs((c.size - 1) - deg_ref) <= 1 and abs(info - info_ref) <= 1
    with pytest.warns(B.PPWarning):
        p2, info2 = B.pp_build_poly_power(B.CSRMatrix.from_host(Ac), _up(b), 16)
    c2 = B.pp_poly_coeffs(p2)
    assert info2 > 0 and np.all(c2[info2 - 1:] == 0)


def test_power_basis_solve_parity(B):
    P = W.config(1)
    As = P.A.to_scipy()
    A = B.CSRMatrix.from_host(P.A)
    p, info = B.pp_build_poly_power(A, _up(P.v0), 5)
    c = B.pp_poly_coeffs(p)
    x, st = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=0, tol=P.tol, poly=p)
    xo, so = ogmres.pp_gmres(As, P.b, P.m, P.tol, coeffs=c, max_iters=3000)
    assert st.nroots == 6
    xg = x.cpu().numpy()
    assert st.relres_true < P.tol and so.converged
    assert abs(st.iters - so.iters) <= max(1, round(0.02 * so.iters))
    if st.iters == so.iters:
        assert _rel(xg, xo) <= 1e-8
    p0, _ = B.pp_build_poly_power(A, _up(P.v0), 0)
    v = W.uniform(P.A.n, 32)
    c0 = B.pp_poly_coeffs(p0)
    assert np.allclose(B.pp_apply(A, p0, _up(v)).cpu().numpy(), c0[0] * v, rtol=1e-15)


# ---- composition with a left Jacobi preconditioner (Section II: polynomial of M A)
def _varied_diagonal_matrix(n, seed):
    Ah = W.random_csr(n, 8, seed=seed, diag_shift=0.0)
    A = Ah.to_scipy()
    dg = np.random.default_rng(seed + 1).uniform(2.0, 400.0, n)
    A = sp.csr_matrix(A + sp.diags(dg - A.diagonal()))
    A.sort_indices()
    return A


def test_left_jacobi_composition_parity(B):
    A = _varied_diagonal_matrix(777, 60)
    b = W.normal(777, 61)
    v0 = W.uniform(777, 62)
    Ad = B.CSRMatrix.from_host(A)
    x, st = B.pp_gmres_solve(Ad, _up(b), m=20, d=6, tol=1e-10, v0=_up(v0), left_jacobi=True)
    xo, so = ogmres.pp_gmres_left_jacobi(A, b, 20, 1e-10, v0=v0, d=6, max_iters=2000)
    xg = x.cpu().numpy()
    assert st.relres_true < 1e-10 and so.converged
    assert abs(st.iters - so.iters) <= max(1, round(0.02 * so.iters))
    if st.iters == so.iters:
        assert _rel(xg, xo) <= 1e-8
    assert abs(st.relres_original - so.relres_original) <= 1e-3 * so.relres_original + 1e-15
    # without the row scaling the same problem needs more iterations
    _, s0 = B.pp_gmres_solve(Ad, _up(b), m=20, d=6, tol=1e-10, v0=_up(v0), max_iters=2000)
    assert st.iters < s0.iters


def test_left_jacobi_rejects_zero_diagonal(B):
    A = _varied_diagonal_matrix(300, 63).tolil()
    A[5, 5] = 0.0
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    with pytest.raises(B.PPError) as e:
        B.pp_gmres_solve(B.CSRMatrix.from_host(A), _up(W.normal(300, 1)), m=10, d=3, tol=1e-8,
                         v0=_up(W.uniform(300, 2)), left_jacobi=True)
    assert e.value.code == B.PP_ERR_SINGULAR


# ---- basis wider than one fused CGS2 sweep (64 columns): the chunked paths
def test_gmres_with_more_than_64_basis_columns(B):
    P = W.config(1)
    xg, st, xo, so = _solve_both(B, P.A, P.b, P.v0, 100, 0, P.tol)
    assert st.iters > 64          # the Arnoldi basis outgrew one sweep
    _assert_parity(st, so, xg, xo, P.tol)


def test_build_with_more_than_64_roots(B):
    Ah = W.convection_diffusion(20, 2, 10.0, (1.0, 1.0))   # n = 400
    v0 = W.uniform(Ah.n, 70)
    ref, s = opoly.build_poly(Ah.to_scipy(), v0, 72)
    got = B.pp_build_poly(B.CSRMatrix.from_host(Ah), _up(v0), 72).roots()
    assert got.size == ref.size == 72
    assert _match_sets(got, ref) <= 1e-6


# ---- streams and workspace
def test_solve_on_a_side_stream_and_after_workspace_release(B):
    P = W.config(1, N=40)
    A = B.CSRMatrix.from_host(P.A)
    x0, s0 = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=P.d, tol=P.tol, v0=_up(P.v0))
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        b = _up(P.b)
        v0 = _up(P.v0)
        x1, s1 = B.pp_gmres_solve(A, b, m=P.m, d=P.d, tol=P.tol, v0=v0, stream=side)
    side.synchronize()
    B.pp_release_workspace()
    x2, s2 = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=P.d, tol=P.tol, v0=_up(P.v0))
    assert s0.iters == s1.iters == s2.iters
    assert np.array_equal(x0.cpu().numpy(), x1.cpu().numpy())
    assert np.array_equal(x0.cpu().numpy(), x2.cpu().numpy())


def test_history_and_timing_fields(B):
    P = W.config(1, N=40)
    A = B.CSRMatrix.from_host(P.A)
    x, st = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=P.d, tol=P.tol, v0=_up(P.v0), history=500,
                             timing=True)
    h = st.history
    assert h.size == st.iters and h[-1] < P.tol and np.all(np.diff(h) <= 1e-12 * h[:-1])
    assert st.t_chain > 0 and st.t_orth > 0 and st.bytes_chain > 0 and st.launches_chain > 0
    assert st.t_total >= st.t_poly > 0


# ---- sliced-ELL layout: selection and agreement with CSR
def test_auto_layout_choice(B):
    P = W.config(1, N=40)       # 5-point stencil: padding only at the grid boundary
    x, st = B.pp_gmres_solve(B.CSRMatrix.from_host(P.A), _up(P.b), m=P.m, d=P.d, tol=P.tol,
                             v0=_up(P.v0))
    assert st.layout_used == "sell"
    ns = -(-P.A.n // 64)
    assert P.A.nnz <= st.nnz_stored <= 64 * ns * 5
    # one long row per slice: sliced ELL would store ~16x nnz, so AUTO keeps CSR
    n = 1024
    counts = np.ones(n, np.int64)
    counts[::64] = 60
    rng = np.random.default_rng(31)
    rows = []
    for i, c in enumerate(counts):
        others = rng.choice(n - 1, c - 1, replace=False)
        rows.append(np.sort(np.concatenate([[i], others + (others >= i)])))
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum([r.size for r in rows])
    ci = np.concatenate(rows).astype(np.int32)
    va = rng.uniform(-1, 1, ci.size) + 8.0 * (ci == np.repeat(np.arange(n), np.diff(rp)))
    Ah = W.CSR(n, rp, ci, va)
    b = W.normal(n, 32)
    xa, sa = B.pp_gmres_solve(B.CSRMatrix.from_host(Ah), _up(b), m=20, d=4, tol=1e-10,
                              v0=_up(W.uniform(n, 33)))
    assert sa.layout_used == "csr" and sa.nnz_stored == Ah.nnz
    xs, ss = B.pp_gmres_solve(B.CSRMatrix.from_host(Ah, layout="sell"), _up(b), m=20, d=4,
                              tol=1e-10, v0=_up(W.uniform(n, 33)))
    assert ss.layout_used == "sell" and ss.nnz_stored == 64 * (n // 64) * 60
    assert sa.iters == ss.iters and _rel(xs.cpu().numpy(), xa.cpu().numpy()) <= 1e-10


@pytest.mark.parametrize("precision", ["f64", "f32_ir"])
def test_layouts_agree_on_solve(B, precision):
    P = W.config(3, N=20)       # 27-point stencil, n = 8000 (125 slices)
    A = B.CSRMatrix.from_host(P.A)
    out = {}
    for layout in LAYOUTS:
        x, st = B.pp_gmres_solve(A.with_layout(layout), _up(P.b), m=P.m, d=P.d, tol=P.tol,
                                 v0=_up(P.v0), precision=precision)
        assert st.layout_used == layout and st.relres_true < P.tol
        out[layout] = (x.cpu().numpy(), st)
    (xc, sc), (xs, ss) = out["csr"], out["sell"]
    # the layouts differ only in summation rounding; the FP32 inner cycles may
    # stop a step apart on their 1e-5 implicit test
    assert abs(sc.iters - ss.iters) <= (1 if precision == "f64" else 2 * max(sc.outer, 1))
    assert _rel(xs, xc) <= (1e-8 if precision == "f64" else 1e-6)


def test_refinement_with_given_fp32_values_on_sell(B):
    P = W.config(1)
    A = B.CSRMatrix.from_host(P.A, layout="sell")
    v32 = _up(P.A.vals, torch.float32)
    x1, s1 = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=P.d, tol=1e-10, v0=_up(P.v0),
                              precision="f32_ir", vals_f32=v32)
    x2, s2 = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=P.d, tol=1e-10, v0=_up(P.v0),
                              precision="f32_ir")
    assert s1.layout_used == s2.layout_used == "sell"
    # the given FP32 values equal the internal cast: identical runs
    assert s1.iters == s2.iters and np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())


def _mixed_structure_matrix():
    """2D 5-point stencil whose rows 512..767 are replaced by random rows: slices 8..11
    of the sliced copy need explicit columns, the others are stored by diagonal."""
    S = W.config(1, N=32).A
    R = W.random_csr(1024, 9, seed=41, diag_shift=6.0)
    rows = []
    for i in range(1024):
        src = R if 512 <= i < 768 else S
        a, b = src.row_ptr[i], src.row_ptr[i + 1]
        rows.append((src.col_ind[a:b], src.vals[a:b]))
    rp = np.zeros(1025, np.int32)
    rp[1:] = np.cumsum([r[0].size for r in rows])
    return W.CSR(1024, rp, np.concatenate([r[0] for r in rows]).astype(np.int32),
                 np.concatenate([r[1] for r in rows]))


@pytest.mark.parametrize("layout", LAYOUTS)
def test_apply_mixed_diagonal_and_explicit_slices(B, layout):
    Ah = _mixed_structure_matrix()
    roots = np.array([6.0, 3.0 + 1.0j, 3.0 - 1.0j, 2.0, 8.0])
    p = B.pp_poly_from_roots(Ah.n, roots)
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-4)):
        v = W.uniform(Ah.n, 42)
        A = B.CSRMatrix.from_host(Ah, dtype=dt, layout=layout)
        pp = p if dt == torch.float64 else B.pp_poly_from_roots(Ah.n, roots, dtype="f32")
        y = B.pp_apply(A, pp, _up(v, dt)).cpu().numpy().astype(np.float64)
        assert _rel(y, opoly.apply_poly(Ah.to_scipy(), roots, v)) <= tol


@pytest.mark.parametrize("layout", LAYOUTS)
def test_apply_unsorted_rows_and_duplicate_columns(B, layout):
    base = W.config(1, N=24).A            # n = 576: 9 slices
    rp, ci, va = base.row_ptr.copy(), base.col_ind.copy(), base.vals.copy()
    for i in range(0, base.n, 5):         # reverse every fifth row's column order
        a, b = rp[i], rp[i + 1]
        ci[a:b] = ci[a:b][::-1].copy()
        va[a:b] = va[a:b][::-1].copy()
    # split the diagonal entry of every seventh row into two duplicate entries
    rows_ci, rows_va = [], []
    for i in range(base.n):
        c, v = list(ci[rp[i]:rp[i + 1]]), list(va[rp[i]:rp[i + 1]])
        if i % 7 == 0:
            k = c.index(i)
            c.insert(k, i)
            v[k] = 0.25 * v[k]
            v.insert(k, 3.0 * v[k])
        rows_ci.append(c)
        rows_va.append(v)
    rp2 = np.zeros(base.n + 1, np.int32)
    rp2[1:] = np.cumsum([len(c) for c in rows_ci])
    Ah = W.CSR(base.n, rp2, np.concatenate(rows_ci).astype(np.int32), np.concatenate(rows_va))
    As = Ah.to_scipy()                    # scipy sums duplicates in its products
    assert np.allclose(As.toarray(), base.to_scipy().toarray())
    roots = np.array([5.0, 2.0 + 0.5j, 2.0 - 0.5j, 7.0])
    p = B.pp_poly_from_roots(Ah.n, roots)
    v = W.uniform(Ah.n, 43)
    y = B.pp_apply(B.CSRMatrix.from_host(Ah, layout=layout), p, _up(v)).cpu().numpy()
    assert _rel(y, opoly.apply_poly(As, roots, v)) <= 1e-12


def test_sliced_copy_stores_stencils_by_diagonal(B):
    # the bytes per chain launch drop to values + offsets when every slice is diagonal:
    # 8 * stored + small; an explicit-column copy would add 4 bytes per stored entry
    P = W.config(2, N=24)
    x, st = B.pp_gmres_solve(B.CSRMatrix.from_host(P.A), _up(P.b), m=P.m, d=10, tol=P.tol,
                             v0=_up(P.v0), timing=True)
    assert st.layout_used == "sell" and st.relres_true < P.tol
    n, stored = P.A.n, st.nnz_stored
    ns = -(-n // 64)
    per_launch = st.bytes_chain / st.launches_chain
    # values + one offset per 64 stored slots + slice offsets and flags + at most 4 vectors
    assert per_launch <= 8.0 * stored + stored / 16.0 + 8.0 * ns + 4.0 + 32.0 * n
    # explicit columns would cost at least 12 bytes per stored slot plus 2 vectors
    assert 12.0 * stored + 16.0 * n > 8.0 * stored + stored / 16.0 + 8.0 * ns + 4.0 + 32.0 * n


def test_auto_layout_keeps_csr_for_a_short_apply(B):
    # two roots on a small stencil: the conversion would cost more than it saves, AUTO keeps
    # CSR; the result is the same polynomial either way
    Ah = W.config(1, N=48).A
    roots = np.array([4.0, 6.0])
    p = B.pp_poly_from_roots(Ah.n, roots)
    v = W.uniform(Ah.n, 51)
    ys = {lay: B.pp_apply(B.CSRMatrix.from_host(Ah, layout=lay), p, _up(v)).cpu().numpy()
          for lay in ("auto", "csr", "sell")}
    ref = opoly.apply_poly(Ah.to_scipy(), roots, v)
    for lay, y in ys.items():
        assert _rel(y, ref) <= 1e-13, lay
    assert np.array_equal(ys["auto"], ys["csr"])


# ---- Section VI's first example (recirculating flow, eps = 1/2) at a reduced grid
@pytest.mark.parametrize("d", [5, 10])
def test_recirculating_flow_example1_matches_oracle(B, d):
    Ah, b = W.recirculating_flow(65, 0.5)
    v0 = W.uniform(Ah.n, 107)
    A = B.CSRMatrix.from_host(Ah)
    x, st = B.pp_gmres_solve(A, _up(b), m=50, d=d, tol=1e-8, v0=_up(v0), max_iters=5000)
    xo, so = ogmres.pp_gmres(Ah.to_scipy(), b, 50, 1e-8, v0=v0, d=d, max_iters=5000)
    assert so.converged and st.relres_true < 1e-8
    assert abs(st.iters - so.iters) <= max(1, round(0.02 * so.iters)), (st.iters, so.iters)
    if st.iters == so.iters:
        assert _rel(x.cpu().numpy(), xo) <= 1e-8


def test_slow_convergence_is_not_stopped_as_stagnation(B):
    # many cycles each gain < 10% just above tol, but none ends on the estimate
    Ah, b = W.recirculating_flow(33, 0.5)
    A = B.CSRMatrix.from_host(Ah)
    x, st = B.pp_gmres_solve(A, _up(b), m=5, d=0, tol=1e-8, max_iters=60000)
    xo, so = ogmres.pp_gmres(Ah.to_scipy(), b, 5, 1e-8, max_iters=60000)
    assert so.converged and st.status == B.PP_OK and st.relres_true < 1e-8
    assert abs(st.iters - so.iters) <= max(1, round(0.02 * so.iters)), (st.iters, so.iters)


# ---- slab-skewed chain schedule (matrix-powers style, Section VII): same bits
@pytest.mark.parametrize("group,slab", [(2, 2048), (5, 4096), (40, 1024), (3, 1 << 21)])
@pytest.mark.parametrize("precision", ["f64", "f32_ir"])
def test_blocked_chain_gives_identical_results(B, group, slab, precision):
    P = W.config(2, N=32)  # bandwidth 1024 rows, complex root pairs
    A = B.CSRMatrix.from_host(P.A)
    kw = dict(m=20, d=10, tol=1e-10, v0=_up(P.v0), precision=precision)
    x0, s0 = B.pp_gmres_solve(A, _up(P.b), **kw)
    x1, s1 = B.pp_gmres_solve(A, _up(P.b), chain_group=group, chain_slab_rows=slab, **kw)
    x2, s2 = B.pp_gmres_solve(A, _up(P.b), chain_group=1, **kw)
    assert s0.relres_true < 1e-10
    assert s1.iters == s0.iters and torch.equal(x0, x1)
    assert s2.iters == s0.iters and torch.equal(x0, x2)
    # automatic: this matrix fits the cache, so full-range cached launches
    assert (s0.chain_slab_rows, s0.chain_cached) == (0, True)
    assert (s1.chain_slab_rows, s1.chain_cached) == (slab, True)
    assert (s2.chain_slab_rows, s2.chain_cached) == (0, False)


@pytest.mark.parametrize("precision", ["f64", "f32_ir"])
def test_blocked_chain_on_the_csr_layout(B, precision):
    # CSR products tile by 256 rows in both precisions
    P = W.config(2, N=24)
    A = B.CSRMatrix.from_host(P.A, layout="csr")
    kw = dict(m=20, d=8, tol=1e-10, v0=_up(P.v0), precision=precision)
    x0, s0 = B.pp_gmres_solve(A, _up(P.b), **kw)
    x1, s1 = B.pp_gmres_solve(A, _up(P.b), chain_group=3, chain_slab_rows=1500, **kw)
    assert s0.layout_used == s1.layout_used == "csr"
    assert s1.iters == s0.iters and torch.equal(x0, x1)


@pytest.mark.parametrize("group,slab", [(2, 2048), (40, 1024)])
def test_blocked_horner_and_product_form_chains(B, group, slab):
    # the power basis' Horner chain and the product-form operator (A (p(A) v)) in
    # the slab-skewed order: the same bits as full-range launches
    P = W.config(2, N=32)
    A = B.CSRMatrix.from_host(P.A)
    p, _ = B.pp_build_poly_power(A, _up(P.v0), 8)
    runs = [dict(poly=p), dict(d=10, op_form="p")]
    for extra in runs:
        kw = dict(m=20, d=extra.pop("d", 8), tol=1e-10, v0=_up(P.v0), **extra)
        x0, s0 = B.pp_gmres_solve(A, _up(P.b), chain_group=1, **kw)
        x1, s1 = B.pp_gmres_solve(A, _up(P.b), chain_group=group, chain_slab_rows=slab, **kw)
        x2, s2 = B.pp_gmres_solve(A, _up(P.b), **kw)
        assert s0.relres_true < 1e-10, extra
        assert s1.iters == s0.iters and torch.equal(x0, x1), extra
        assert s2.iters == s0.iters and torch.equal(x0, x2), extra


def test_automatic_schedule_past_the_cache_budget(B):
    # a 160^3 stencil (4.1M rows) is past the cache budget: in natural order
    # (bandwidth 25,600 rows) the automatic choice is the slab-skewed order; under
    # a random symmetric permutation (bandwidth ~ n) it falls back to full-range
    # non-temporal launches.  Both give the bits of chain_group 1.
    import warnings
    P = W.config(2, N=160)
    S = P.A.to_scipy()
    perm = np.random.default_rng(3).permutation(S.shape[0])
    Sp = S[perm][:, perm].tocsr()
    Sp.sort_indices()
    for Ah, b, v0, blocked in ((S, P.b, P.v0, True), (Sp, P.b[perm], P.v0[perm], False)):
        A = B.CSRMatrix.from_host(Ah)
        kw = dict(m=10, d=6, tol=1e-12, v0=_up(v0), max_iters=20)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", B.PPWarning)  # stopped at max_iters
            x0, s0 = B.pp_gmres_solve(A, _up(b), **kw)
            x1, s1 = B.pp_gmres_solve(A, _up(b), chain_group=1, **kw)
        assert s0.iters >= 10 and s1.iters == s0.iters and torch.equal(x0, x1)
        if blocked:
            assert s0.chain_cached and 0 < s0.chain_slab_rows < S.shape[0]
        else:
            assert (s0.chain_slab_rows, s0.chain_cached) == (0, False)


def test_chain_schedule_options_are_checked(B):
    P = W.config(1, N=16)
    A = B.CSRMatrix.from_host(P.A)
    for kw in (dict(chain_group=-1), dict(chain_slab_rows=-5)):
        with pytest.raises(B.PPError) as e:
            B.pp_gmres_solve(A, _up(P.b), m=10, d=4, tol=1e-8, v0=_up(P.v0), **kw)
        assert e.value.code == B.PP_ERR_ARG


@pytest.mark.parametrize("precision", ["f64", "f32_ir"])
def test_blocked_chain_with_a_ragged_tail(B, precision):
    # n = 27000: a partial last slice (64 rows), FP64 tile (256) and FP32 tile (512),
    # and slabs that are not whole tiles (rounded down)
    P = W.config(2, N=30)
    A = B.CSRMatrix.from_host(P.A)
    kw = dict(m=20, d=9, tol=1e-10, v0=_up(P.v0), precision=precision)
    x0, s0 = B.pp_gmres_solve(A, _up(P.b), chain_group=1, **kw)
    assert s0.relres_true < 1e-10
    for group, slab in ((2, 1000), (40, 777), (5, 27000)):
        x1, s1 = B.pp_gmres_solve(A, _up(P.b), chain_group=group, chain_slab_rows=slab, **kw)
        assert s1.iters == s0.iters and torch.equal(x0, x1), (group, slab)


def test_blocked_chain_with_wide_bandwidth(B):
    # bandwidth about n: each launch trails the previous by more than a slab
    Ah = W.random_csr(3000, 6, seed=12, diag_shift=8.0)
    A = B.CSRMatrix.from_host(Ah)
    kw = dict(m=15, d=6, tol=1e-10, v0=_up(W.uniform(3000, 13)))
    x0, s0 = B.pp_gmres_solve(A, _up(W.normal(3000, 14)), **kw)
    x1, s1 = B.pp_gmres_solve(A, _up(W.normal(3000, 14)), chain_group=4, chain_slab_rows=512,
                              **kw)
    assert s1.iters == s0.iters and torch.equal(x0, x1)


def test_pp_log_traces_cycles_and_steps(B):
    # PP_LOG is read once per process: run a tiny solve in a child process
    import subprocess
    import sys
    code = ("import numpy as np, torch\n"
            "from paper_1907_00072_amd import binding as B, workloads as W\n"
            "P = W.config(1, N=16)\n"
            "A = B.CSRMatrix.from_host(P.A)\n"
            "x, st = B.pp_gmres_solve(A, torch.from_numpy(P.b).cuda(), m=10, d=4, tol=1e-8,\n"
            "                         v0=torch.from_numpy(P.v0).cuda())\n"
            "print('iters', st.iters, 'cycles', st.cycles)\n")
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=root,
                       env=dict(os.environ, PP_LOG="2"), timeout=120)
    assert r.returncode == 0, r.stderr[-1000:]
    iters = int(r.stdout.split()[1])
    cycles = int(r.stdout.split()[3])
    assert r.stderr.count("[pp] cycle") == cycles
    assert "[pp] chain: full-range, cached (FP64)" in r.stderr  # the matrix fits the cache
    assert r.stderr.count("implicit relres") >= iters


def test_failure_paths(B):
    P = W.config(1, N=16)
    n = P.A.n
    A = B.CSRMatrix.from_host(P.A)
    b, v0 = _up(P.b), _up(P.v0)
    for kw in (dict(tol=0.0), dict(tol=-1e-8), dict(d=n + 1), dict(d=257), dict(m=0)):
        args = dict(m=10, d=4, tol=1e-8, v0=v0)
        args.update(kw)
        with pytest.raises(B.PPError) as e:
            B.pp_gmres_solve(A, b, **args)
        assert e.value.code == B.PP_ERR_ARG, kw
    # a polynomial built for another size
    with pytest.raises(B.PPError) as e:
        B.pp_gmres_solve(A, b, m=10, tol=1e-8, poly=B.pp_poly_from_roots(n + 1, [2.0, 3.0]))
    assert e.value.code == B.PP_ERR_ARG
    # zero start vector: no Krylov space to build the polynomial from
    with pytest.raises(B.PPError) as e:
        B.pp_build_poly(A, torch.zeros_like(v0), 4)
    assert e.value.code == B.PP_ERR_SINGULAR
    # b = 0: x = 0 at once
    x, st = B.pp_gmres_solve(A, torch.zeros_like(b), m=10, d=4, tol=1e-8, v0=v0)
    assert st.status == B.PP_OK and st.iters == 0 and not torch.any(x)
    # NaN in A's values: never reported as a success
    vals = P.A.vals.copy()
    vals[7] = np.nan
    An = B.CSRMatrix.from_host(W.CSR(n, P.A.row_ptr, P.A.col_ind, vals))
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        try:
            _, st = B.pp_gmres_solve(An, b, m=10, d=4, tol=1e-8, v0=v0)
            assert st.status == B.PP_WARN_NONFINITE
        except B.PPError as err:
            assert err.code in (B.PP_ERR_SINGULAR, B.PP_ERR_ARG)


def test_arnoldi_breakdown_reduces_the_degree(B):
    # v0 an eigenvector of a diagonal matrix: the Krylov space is one-dimensional
    n = 50
    dg = np.linspace(1.0, 5.0, n)
    Ah = W.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), dg)
    A = B.CSRMatrix.from_host(Ah)
    e3 = np.zeros(n)
    e3[3] = 1.0
    with pytest.warns(B.PPWarning):
        p = B.pp_build_poly(A, _up(e3), 6)
    roots = p.roots()
    assert roots.size == 1 and abs(roots[0] - dg[3]) <= 1e-13 * dg[3]


@pytest.mark.parametrize("d", [0, 3])
def test_lucky_breakdown_ends_the_solve(B, d):
    # b an eigenvector of a diagonal A: the first Arnoldi step already spans the
    # solution (h_21 = 0).  The step issued ahead of it normalises a zero vector; its
    # results are never read, and the solve ends after one step with x = b / a_33.
    n = 50
    dg = np.linspace(1.0, 5.0, n)
    Ah = W.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), dg)
    A = B.CSRMatrix.from_host(Ah)
    b = np.zeros(n)
    b[3] = 2.0
    x, st = B.pp_gmres_solve(A, _up(b), m=10, d=d, tol=1e-12, v0=_up(W.uniform(n, 5)))
    assert st.iters == 1 and st.relres_true < 1e-14
    ref = np.zeros(n)
    ref[3] = 2.0 / dg[3]
    assert np.allclose(x.cpu().numpy(), ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("layout", ["csr", "sell"])
def test_smallest_systems(B, layout):
    """Degenerate sizes: one row, and two rows whose two roots are a conjugate pair.
    With d = n roots the residual polynomial vanishes on A, so p(A) = A^-1 (the
    special case of the method that reduces to a direct solve): p(A) v is checked
    against numpy.linalg.solve, and the solve ends after one Arnoldi step."""
    # n = 1: one root, theta = a
    A1 = W.CSR(1, np.array([0, 1], dtype=np.int32), np.array([0], dtype=np.int32),
               np.array([3.0]))
    Ad = B.CSRMatrix.from_host(A1, layout=layout)
    p = B.pp_build_poly(Ad, _up(np.array([0.7])), 1)
    r = B.pp_poly_roots(p)
    assert np.allclose(r.real, [3.0], rtol=1e-15) and not np.any(r.imag)
    y = B.pp_apply(Ad, p, _up(np.array([6.0]))).cpu().numpy()
    assert abs(y[0] - 2.0) <= 1e-15
    x, st = B.pp_gmres_solve(Ad, _up(np.array([6.0])), m=1, d=1, tol=1e-12,
                             v0=_up(np.array([0.7])))
    assert st.iters == 1 and abs(x.cpu().numpy()[0] - 2.0) <= 1e-15
    # n = 2: A = [[2, -1], [1, 2]], eigenvalues 2 +- i: one pair step
    Ad2 = np.array([[2.0, -1.0], [1.0, 2.0]])
    As = sp.csr_matrix(Ad2)
    A2 = W.CSR(2, As.indptr.astype(np.int32), As.indices.astype(np.int32), As.data)
    Ad = B.CSRMatrix.from_host(A2, layout=layout)
    p = B.pp_build_poly(Ad, _up(np.array([1.0, 0.3])), 2)
    r = B.pp_poly_roots(p)
    assert np.allclose(np.sort(r.real), [2.0, 2.0], rtol=1e-14)
    assert np.allclose(np.sort(r.imag), [-1.0, 1.0], rtol=1e-14)
    v = np.array([0.4, -1.3])
    y = B.pp_apply(Ad, p, _up(v)).cpu().numpy()
    ref = np.linalg.solve(Ad2, v)
    assert np.max(np.abs(y - ref)) <= 1e-14 * np.max(np.abs(ref))
    x, st = B.pp_gmres_solve(Ad, _up(v), m=2, d=2, tol=1e-12, v0=_up(np.array([1.0, 0.3])))
    assert st.iters == 1 and st.relres_true < 1e-14
    assert np.max(np.abs(x.cpu().numpy() - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_checkpoint_and_resume_is_exact(B):
    # a solve interrupted at a cycle boundary and resumed from (x, roots) ends with
    # the same bits as the uninterrupted solve.  The layout is fixed: with "auto" a
    # separate pp_build_poly (only d products) may keep CSR where the solve takes
    # the sliced copy, and the two sum the products in different orders.
    import warnings
    P = W.config(1, N=32)
    A = B.CSRMatrix.from_host(P.A, layout="sell")
    b, v0 = _up(P.b), _up(P.v0)
    m, d = 10, 4
    x_full, s_full = B.pp_gmres_solve(A, b, m=m, d=d, tol=1e-10, v0=v0)
    assert s_full.relres_true < 1e-10 and s_full.cycles >= 3
    p = B.pp_build_poly(A, v0, d)
    roots = p.roots()
    k = 2 * m  # two complete cycles
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        x_part, s_part = B.pp_gmres_solve(A, b, m=m, tol=1e-10, poly=p, max_iters=k)
    assert s_part.status == B.PP_WARN_NOT_CONVERGED and s_part.iters == k
    saved_x = x_part.cpu().numpy().copy()
    resumed = B.pp_poly_from_roots(P.A.n, roots)
    x_res, s_res = B.pp_gmres_solve(A, b, _up(saved_x), m=m, tol=1e-10, poly=resumed)
    assert s_res.relres_true < 1e-10
    assert s_part.iters + s_res.iters == s_full.iters
    assert torch.equal(x_res, x_full)


@pytest.mark.parametrize("cfg,N,precision", [(1, None, "f64"), (4, 128, "f64"), (4, 400, "f64"),
                                             (1, None, "f32_ir"), (2, 16, "f64")])
def test_folded_reductions_are_bitwise_the_separate_launches(B, cfg, N, precision, monkeypatch):
    """Each CGS2 sweep whose partials are few (at most 256) also does the
    reduction's second stage in its last workgroup; PP_FOLD=0 keeps the separate
    launches.  Same bits, step for step: 64^2 and 128^2 fold every sweep, 400^2
    folds the dot sweeps and leaves some update sweeps (313 partials) to the
    separate launches, and the 16^3 case with m = 80 also runs steps past 64
    basis columns (chunked sweeps, never folded)."""
    import warnings
    P = W.config(cfg, N=N) if N else W.config(cfg)
    A = B.CSRMatrix.from_host(P.A)
    kw = dict(m=P.m, d=P.d, tol=P.tol, v0=_up(P.v0), history=2000)
    if precision == "f32_ir":
        kw.update(precision="f32_ir", inner_tol=1e-5)
    if cfg == 2:
        kw.update(m=80, d=6, tol=1e-12, max_iters=200)
    runs = []
    for fold in ("1", "0"):
        monkeypatch.setenv("PP_FOLD", fold)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", B.PPWarning)
            x, st = B.pp_gmres_solve(A, _up(P.b), **kw)
        runs.append((x, st))
    (x1, s1), (x0, s0) = runs
    assert s1.iters == s0.iters and s1.cycles == s0.cycles and s1.iters > 0
    assert torch.equal(x1, x0)
    assert np.array_equal(s1.history, s0.history)


@pytest.mark.parametrize("cfg,N,precision,m", [(1, None, "f64", None), (4, 96, "f64", None),
                                               (4, 96, "f64", 7), (3, 12, "f32_ir", None),
                                               (1, None, "f64_plain", 13)])
def test_lookahead_is_bitwise_the_serial_steps(B, cfg, N, precision, m, monkeypatch):
    """Short Arnoldi steps are issued one ahead of the host (the device part of step
    j + 1 before step j's column is read); PP_LOOKAHEAD=0 runs them one at a time.
    Same kernels in the same order: the same bits, iteration counts, residual
    history and counters (a step issued past a cycle's stop is taken back out of
    them).  Restart cycles of 7 and 13 steps stop both at the cycle's end and in its
    middle."""
    import warnings
    P = W.config(cfg, N=N) if N else W.config(cfg)
    A = B.CSRMatrix.from_host(P.A)
    kw = dict(m=m or P.m, d=P.d, tol=P.tol, v0=_up(P.v0), history=4000, max_iters=4000)
    if precision == "f32_ir":
        kw.update(precision="f32_ir", inner_tol=1e-5)
    if precision == "f64_plain":
        kw.update(d=0)
    runs = []
    for la in ("1", "0"):
        monkeypatch.setenv("PP_LOOKAHEAD", la)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", B.PPWarning)
            x, st = B.pp_gmres_solve(A, _up(P.b), **kw)
        runs.append((x, st))
    (x1, s1), (x0, s0) = runs
    assert s1.iters == s0.iters and s1.cycles == s0.cycles and s1.iters > 0
    assert torch.equal(x1, x0)
    assert np.array_equal(s1.history, s0.history)
    assert (s1.spmvs, s1.dots) == (s0.spmvs, s0.dots)
    assert s1.bytes_chain == s0.bytes_chain and s1.bytes_orth == s0.bytes_orth


@pytest.mark.parametrize("block,layout", [(None, "auto"), (None, "sell"), (None, "csr"),
                                          (4096, "auto")])
def test_permuted_stencil_solve_matches_oracle(B, block, layout):
    """A matrix without diagonal structure: the 40^3 convection-diffusion problem
    (Peclet 100) under a seeded symmetric permutation P A P^T, uniform over all rows
    or within blocks of 4096.  Its slices hold explicit columns (no shared
    diagonals), its bandwidth is about n.  The solve follows the parity rule
    against the oracle on the same permuted system, and un-permuted it solves the
    original system."""
    P = W.config(5, N=40)
    perm = W.permutation(P.A.n, 17, block)
    Ap = W.permuted(P.A, perm)
    bp, v0p = P.b[perm], P.v0[perm]
    xg, st, xo, so = _solve_both(B, Ap, bp, v0p, 30, 12, 1e-8, layout=layout)
    _assert_parity(st, so, xg, xo, 1e-8)
    x = np.empty_like(xg)
    x[perm] = xg
    assert np.linalg.norm(P.b - P.A.to_scipy() @ x) <= 1e-8 * np.linalg.norm(P.b)
    if layout != "auto":
        assert st.layout_used == layout
    # automatic schedule: the bandwidth rules out the slab-skewed order
    assert st.chain_slab_rows == 0


def _dense_p(A, roots):
    """p(A) formed densely from its roots: A^{-1} (I - prod_i (I - A/theta_i))."""
    n = A.shape[0]
    Pi = np.eye(n, dtype=complex)
    for t in roots:
        Pi = Pi @ (np.eye(n) - A / t)
    return np.linalg.solve(A, np.eye(n) - Pi).real


@pytest.mark.parametrize("name,d,layout", [("cd2d_8", 10, "auto"), ("cd2d_8", 10, "csr"),
                                           ("dense_40", 9, "auto"), ("dense_40", 9, "sell"),
                                           ("rand_64", 12, "csr"), ("rand_64", 12, "sell")])
def test_apply_every_column_against_dense_p(B, name, d, layout):
    """Brute force (n <= 64): every column of p(A), i.e. pp_apply on each unit
    vector, against p(A) formed densely from the same roots; both real roots and
    conjugate pairs occur in these root sets."""
    if name == "cd2d_8":
        Ah = W.config(1, N=8).A
    elif name == "dense_40":
        rng = np.random.default_rng(41)
        M = rng.standard_normal((40, 40)) / np.sqrt(40) + 1.5 * np.eye(40)
        S = sp.csr_matrix(M)
        Ah = W.CSR(40, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.copy())
    else:
        Ah = W.random_csr(64, 9, seed=43, diag_shift=3.0)
    M = Ah.to_dense()
    roots, _ = opoly.build_poly(Ah.to_scipy(), W.uniform(Ah.n, 44), d)
    ref = _dense_p(M, roots)
    A = B.CSRMatrix.from_host(Ah, layout=layout)
    poly = B.pp_poly_from_roots(Ah.n, roots)
    got = np.column_stack([B.pp_apply(A, poly, _up(e)).cpu().numpy() for e in np.eye(Ah.n)])
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # FP32: the same columns to FP32 rounding
    A32 = B.CSRMatrix.from_host(Ah, layout=layout, dtype=torch.float32)
    p32 = B.pp_poly_from_roots(Ah.n, roots, dtype="f32")
    got32 = np.column_stack([B.pp_apply(A32, p32, _up(e, torch.float32)).cpu().numpy()
                             for e in np.eye(Ah.n)])
    assert np.max(np.abs(got32 - ref)) <= 1e-4 * np.max(np.abs(ref))
