"""GPU parity of ILU(0) and of its composition with the polynomial (Section VI,
second example: ILU(0) on the left, the polynomial of M^-1 A on the right),
through the C ABI, against the CPU oracle.

Tolerances.  The factors: each entry is at most a few dozen multiply-subtracts
and one division from A's values, done in the same order on both sides; the
device may fuse a multiply-subtract into one rounding, so entries agree to a
few ulps of the largest one (1e-12 relative leaves a wide margin and still
catches any wrong index or merge, which give O(1) errors).  The sweeps: the
same argument over at most 2 * (entries per row) operations per row and the
growth of the triangular solves on these diagonally dominant rows: 1e-12 in
norm.  Solves follow the parity rule used for every solve here: iteration
counts within 2%, and ||x_gpu - x_oracle|| / ||x_oracle|| <= 1e-8 when the
counts agree.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import ilu as oilu
from paper_1907_00072_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_00072_amd import binding
    binding.lib()
    return binding


def _up(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda:0", dtype=dtype)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _tridiag(n):
    rng = np.random.default_rng(41)
    return sp.diags([rng.uniform(-1, 1, n - 1), 3.0 + rng.uniform(0, 1, n),
                     rng.uniform(-1, 1, n - 1)], [-1, 0, 1], format="csr")


def _matrix(name):
    if name == "recirc_33":
        return W.recirculating_flow(33)[0].to_scipy()
    if name == "recirc_1":
        return W.recirculating_flow(1)[0].to_scipy()
    if name == "cd3d_40":  # middle levels wider than one run: launches of their own
        return W.convection_diffusion(40, 3, 50.0, (1.0, 0.5, 0.25)).to_scipy()
    if name == "stencil27_12":
        return W.stencil27_random(12, seed=3).to_scipy()
    if name == "rand_900":
        return W.random_csr(900, 10, seed=31, diag_shift=6.0).to_scipy()
    if name == "tridiag_500":
        return _tridiag(500)
    if name == "tridiag_5000":  # 5000 one-row levels: a chain longer than one run holds
        return _tridiag(5000)
    if name == "ninept_48":  # four entries a row in each triangle: the widest LDS-ring rows
        return _nine_point(48)
    raise KeyError(name)


def _nine_point(N):
    # 2D nine-point stencil with seeded perturbations, diagonally dominant
    rng = np.random.default_rng(43)
    T = sp.diags([-1.0, 0.0, -1.0], [-1, 0, 1], shape=(N, N))
    I = sp.identity(N)
    A = (sp.kron(I, T) + sp.kron(T, I) + sp.kron(T, T)).tocsr()
    A.data = A.data * (1.0 + 0.3 * rng.uniform(-1, 1, A.nnz))
    A = A + sp.diags(9.0 + rng.uniform(0, 1, N * N))
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A


NAMES = ["recirc_33", "recirc_1", "cd3d_40", "stencil27_12", "rand_900", "tridiag_500",
         "ninept_48", "tridiag_5000"]
_cache = {}


def _case(B, name):
    if name not in _cache:
        A = _matrix(name)
        A.sort_indices()
        _cache[name] = (A, oilu.ilu0(A))
    A, LU = _cache[name]
    Ad = B.CSRMatrix.from_host(A)
    return A, LU, Ad, B.pp_ilu0_factor(Ad)


@pytest.mark.parametrize("name", NAMES)
def test_factors_match_oracle(B, name):
    A, LU, Ad, M = _case(B, name)
    lu = B.pp_ilu0_values(M).cpu().numpy()
    ref = LU.data
    assert np.max(np.abs(lu - ref)) <= 1e-12 * np.max(np.abs(ref)), name


@pytest.mark.parametrize("name", NAMES)
def test_levels_match_oracle(B, name):
    A, LU, Ad, M = _case(B, name)
    f, b, launches = M.levels()
    assert f == oilu.dependency_levels(A).max() + 1
    assert b == oilu.dependency_levels(A, upper=True).max() + 1
    if name == "recirc_33":
        # every level fits one run per sweep; each sweep adds the level-order gather
        # of its right-hand side and the scatter of the run's solutions to rows
        assert f == b == 2 * 33 - 1 and launches == 6
    if name == "cd3d_40":
        assert f == b == 3 * 40 - 2 and launches > 2  # wide levels get their own launch
    if name == "tridiag_5000":
        # each sweep: two runs (4096 + 904 levels); the second waits for the first's last
        # row, taken out of its right-hand side first: gather, 2 x (run, scatter), update
        assert f == b == 5000 and launches == 12
    if name == "ninept_48":
        # level of (x, y) is x + 2 y in both directions: one ring run per sweep
        assert f == b == 3 * 48 - 2 and launches == 6


@pytest.mark.parametrize("name", NAMES)
def test_apply_matches_oracle(B, name):
    A, LU, Ad, M = _case(B, name)
    n = A.shape[0]
    for seed in (1, 2):
        r = W.normal(n, seed)
        z = B.pp_ilu0_apply(M, _up(r)).cpu().numpy()
        assert _rel(z, oilu.ilu0_solve(LU, r)) <= 1e-12, name
    # in place gives the same bits
    rd = _up(W.normal(n, 3))
    z1 = B.pp_ilu0_apply(M, rd).clone()
    B.pp_ilu0_apply(M, rd, rd)
    assert torch.equal(z1, rd)


def test_exact_factorisation_inverts_a(B):
    # no fill in a tridiagonal pattern: M = A, so M^-1 (A x) = x
    A, LU, Ad, M = _case(B, "tridiag_500")
    x = W.uniform(500, 4)
    z = B.pp_ilu0_apply(M, _up(A @ x)).cpu().numpy()
    assert _rel(z, x) <= 1e-13


def test_bad_patterns_are_rejected(B):
    # missing diagonal
    A = sp.csr_matrix(np.array([[2.0, 1.0, 0.0], [1.0, 0.0, 1.0], [0.0, 1.0, 2.0]]))
    A.eliminate_zeros()
    with pytest.raises(B.PPError) as e:
        B.pp_ilu0_factor(B.CSRMatrix.from_host(A))
    assert e.value.code == B.PP_ERR_ARG
    # unsorted columns in row 0
    rp = torch.tensor([0, 2, 4], dtype=torch.int32, device="cuda:0")
    ci = torch.tensor([1, 0, 0, 1], dtype=torch.int32, device="cuda:0")
    va = torch.tensor([1.0, 3.0, 1.0, 3.0], dtype=torch.float64, device="cuda:0")
    with pytest.raises(B.PPError) as e:
        B.pp_ilu0_factor(B.CSRMatrix(rp, ci, va))
    assert e.value.code == B.PP_ERR_ARG
    # FP32 values
    with pytest.raises(B.PPError) as e:
        B.pp_ilu0_factor(B.CSRMatrix.from_host(_tridiag(10), dtype=torch.float32))
    assert e.value.code == B.PP_ERR_ARG
    # zero pivot: u_11 = 1 - 1 * 1
    Z = sp.csr_matrix(np.array([[1.0, 1.0], [1.0, 1.0]]))
    with pytest.raises(B.PPError) as e:
        B.pp_ilu0_factor(B.CSRMatrix.from_host(Z))
    assert e.value.code == B.PP_ERR_SINGULAR


@pytest.mark.parametrize("d", [0, 13])
def test_composed_solve_matches_oracle(B, d):
    A, b = W.recirculating_flow(33)
    As = A.to_scipy()
    v0 = W.uniform(A.n, 106)
    Ad = B.CSRMatrix.from_host(A)
    M = B.pp_ilu0_factor(Ad)
    x, st = B.pp_gmres_solve(Ad, _up(b), m=50, d=d, tol=1e-8, v0=_up(v0), max_iters=2000,
                             left_ilu=M)
    xo, so = oilu.pp_gmres_left_ilu0(As, b, 50, 1e-8, v0=v0 if d else None, d=d or None,
                                     max_iters=2000, LU=_case(B, "recirc_33")[1])
    xg = x.cpu().numpy()
    assert so.converged and st.relres_true < 1e-8
    assert abs(st.iters - so.iters) <= max(1, round(0.02 * so.iters)), (st.iters, so.iters)
    if st.iters == so.iters:
        assert _rel(xg, xo) <= 1e-8
    assert abs(st.relres_original - so.relres_original) <= 1e-3 * so.relres_original + 1e-15
    assert st.nroots == d


def test_composed_solve_product_form_and_determinism(B):
    A, b = W.recirculating_flow(33)
    v0 = _up(W.uniform(A.n, 106))
    Ad = B.CSRMatrix.from_host(A)
    M = B.pp_ilu0_factor(Ad)
    x1, s1 = B.pp_gmres_solve(Ad, _up(b), m=50, d=8, tol=1e-8, v0=v0, left_ilu=M)
    x2, s2 = B.pp_gmres_solve(Ad, _up(b), m=50, d=8, tol=1e-8, v0=v0, left_ilu=M)
    assert s1.iters == s2.iters and torch.equal(x1, x2)
    x3, s3 = B.pp_gmres_solve(Ad, _up(b), m=50, d=8, tol=1e-8, v0=v0, left_ilu=M, op_form="p")
    assert s3.relres_true < 1e-8 and abs(s3.iters - s1.iters) <= 1
    assert _rel(x3.cpu().numpy(), x1.cpu().numpy()) <= 1e-5


def test_composed_solve_lookahead_is_bitwise(B, monkeypatch):
    # the one-step lookahead of short Arnoldi steps (PP_LOOKAHEAD=0: one at a time)
    A, b = W.recirculating_flow(33)
    Ad = B.CSRMatrix.from_host(A)
    M = B.pp_ilu0_factor(Ad)
    v0 = _up(W.uniform(A.n, 106))
    runs = []
    for la in ("1", "0"):
        monkeypatch.setenv("PP_LOOKAHEAD", la)
        runs.append(B.pp_gmres_solve(Ad, _up(b), m=4, d=8, tol=1e-10, v0=v0, left_ilu=M,
                                     history=500))
    (x1, s1), (x0, s0) = runs
    assert s1.iters == s0.iters and s1.cycles == s0.cycles and s1.cycles > 1
    assert torch.equal(x1, x0) and np.array_equal(s1.history, s0.history)
    assert (s1.spmvs, s1.dots) == (s0.spmvs, s0.dots)


def test_chain_schedule_is_ignored_with_ilu(B):
    # M^-1 couples all rows, so the slab-skewed chain schedule does not apply
    A, b = W.recirculating_flow(33)
    Ad = B.CSRMatrix.from_host(A)
    M = B.pp_ilu0_factor(Ad)
    v0 = _up(W.uniform(A.n, 106))
    x0, s0 = B.pp_gmres_solve(Ad, _up(b), m=50, d=8, tol=1e-8, v0=v0, left_ilu=M)
    x1, s1 = B.pp_gmres_solve(Ad, _up(b), m=50, d=8, tol=1e-8, v0=v0, left_ilu=M,
                              chain_group=4, chain_slab_rows=256)
    assert s1.iters == s0.iters and torch.equal(x0, x1)


def test_composed_solve_rejects_other_modes(B):
    A, b = W.recirculating_flow(9)
    Ad = B.CSRMatrix.from_host(A)
    M = B.pp_ilu0_factor(Ad)
    for kw in ({"precision": "f32_ir"}, {"left_jacobi": True}):
        with pytest.raises(B.PPError) as e:
            B.pp_gmres_solve(Ad, _up(b), m=10, d=3, tol=1e-8, left_ilu=M, **kw)
        assert e.value.code == B.PP_ERR_ARG
    M2 = B.pp_ilu0_factor(B.CSRMatrix.from_host(W.recirculating_flow(8)[0]))
    with pytest.raises(B.PPError) as e:
        B.pp_gmres_solve(Ad, _up(b), m=10, d=3, tol=1e-8, left_ilu=M2)
    assert e.value.code == B.PP_ERR_ARG


def test_concurrent_applies_on_one_factor(B):
    # two host threads, two streams, one pp_ilu: its work vector is taken in turn
    import threading
    A, LU, Ad, M = _case(B, "recirc_33")
    n = A.shape[0]
    rs = [_up(W.normal(n, 21)), _up(W.normal(n, 22))]
    refs = [B.pp_ilu0_apply(M, r).clone() for r in rs]
    outs = [[], []]

    def work(k):
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            for _ in range(20):
                z = torch.empty_like(rs[k])
                B.pp_ilu0_apply(M, rs[k], z, stream=st)
                outs[k].append(z)
    ts = [threading.Thread(target=work, args=(k,)) for k in (0, 1)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    torch.cuda.synchronize()
    for k in (0, 1):
        assert len(outs[k]) == 20 and all(torch.equal(z, refs[k]) for z in outs[k])
