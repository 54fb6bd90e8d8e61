"""GPU parity at the full workload sizes, in the launch configuration bench.py uses.

* 128^3 convection-diffusion (n = 2.1M) and the 96^3 27-point stencil (n = 885k):
  iteration counts, counters, roots and 64 sampled solution entries against
  oracle runs stored in tests/golden/fullsize_refs.json (written by
  tests/golden/make_fullsize_refs.py, which calls only the oracle).
* 256^3 (n = 16.8M, the benchmark): p(A)v on the automatic slab-skewed schedule
  against the oracle's complex-arithmetic evaluation on the whole vector, and at
  sampled rows against the oracle on the sub-grid box of radius d-1 around each
  row (entries of p(A)v at a row depend only on v within graph distance d-1); the
  true residual of the solve recomputed by SciPy, and the stored oracle solve.
* 160^3 (n = 4.1M, past the cache budget, so the slab-skewed schedule runs): the
  whole solution after a fixed number of steps against the oracle run to the
  same count in the test (R10 (ii)).
* 128^3 FP32 refinement: outer count and inner step total against the stored
  oracle run.
* 512^2 adjoint (n = 262k): dL/dvals and dL/db against the oracle's direct
  adjoint on every stored entry and Sherman-Morrison central differences on the
  64 sampled entries; the backward solve alone (PP-GMRES on A^T, d = 15, tol
  1e-12) against the stored oracle run on the same right-hand side: step count,
  stop reason (the stagnation test at FP64's attainable accuracy) and final
  residual, each against the rounding floor of the residual itself.
* 257^2 recirculating flow with ILU(0) on the left and d = 13 on the right
  (Section VI's second example, n = 66k): every factor entry and M^-1 r against
  the oracle, and the solve against the stored oracle solve.
"""
import json
import os
import warnings

import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import gmres as ogmres
from oracle import ilu as oilu
from oracle import poly as opoly
from paper_1907_00072_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REFS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_refs.json")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_00072_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def refs():
    return json.load(open(REFS))


def _up(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda:0", dtype=dtype)


def _match_sets(a, b):
    a = sorted(np.asarray(a, complex), key=lambda t: (t.real, t.imag))
    b = sorted(np.asarray(b, complex), key=lambda t: (t.real, t.imag))
    return max(abs(x - y) / abs(y) for x, y in zip(a, b))


def _check_against_ref(ref, st, x, tol):
    xg = x.cpu().numpy()
    assert st.relres_true < tol and ref["converged"]
    assert abs(st.iters - ref["iters"]) <= max(1, round(0.02 * ref["iters"])), (st.iters,
                                                                                 ref["iters"])
    if st.iters == ref["iters"]:
        idx = np.asarray(ref["sample_idx"])
        err = np.max(np.abs(xg[idx] - np.asarray(ref["x_sample"])))
        assert err <= 1e-8 * ref["x_absmax"], err
        assert abs(np.linalg.norm(xg) - ref["x_norm"]) <= 1e-8 * ref["x_norm"]
    return xg


@pytest.fixture(scope="module")
def cd3d_128(B):
    P = W.config(2)
    return P, B.CSRMatrix.from_host(P.A)


@pytest.mark.parametrize("d", [25, 10, 40, 0])
def test_cd3d_128_solve(B, refs, cd3d_128, d):
    P, A = cd3d_128
    ref = refs[f"cd3d_128_pe50_d{d}"]
    x, st = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=d, tol=P.tol, v0=_up(P.v0))
    _check_against_ref(ref, st, x, P.tol)
    if st.iters == ref["iters"]:
        assert st.spmvs == ref["spmvs"] and st.dots == ref["dots"]
    if d:
        p = B.pp_build_poly(A, _up(P.v0), d)
        ref_roots = np.asarray(ref["roots_re"]) + 1j * np.asarray(ref["roots_im"])
        assert _match_sets(p.roots(), ref_roots) <= 1e-8


def test_cd3d_128_product_form_matches(B, refs, cd3d_128):
    P, A = cd3d_128
    ref = refs["cd3d_128_pe50_d25"]
    x, st = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=25, tol=P.tol, v0=_up(P.v0), op_form="p")
    _check_against_ref(ref, st, x, P.tol)


def test_stencil27_96_fp64_and_refinement(B, refs):
    P = W.config(3)
    A = B.CSRMatrix.from_host(P.A)
    x64, s64 = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=P.d, tol=P.tol, v0=_up(P.v0))
    _check_against_ref(refs["stencil27_96_f64_d25"], s64, x64, P.tol)
    ref = refs["stencil27_96_ir_d25"]
    x, st = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=P.d, tol=P.tol, v0=_up(P.v0),
                             precision="f32_ir", inner_tol=P.extra["inner_tol"])
    assert st.relres_true < P.tol and ref["converged"]
    assert abs(st.outer - ref["outer"]) <= 1
    # both refinement solves are within cond * tol of the FP64 solution
    xg, xf = x.cpu().numpy(), x64.cpu().numpy()
    assert np.linalg.norm(xg - xf) <= 1e-8 * np.linalg.norm(xf)


def _box_rows(N, center, r):
    """Row indices of the sub-grid box of radius r around grid point `center` (x fastest)."""
    cz, cy, cx = center
    zs = np.arange(max(cz - r, 0), min(cz + r, N - 1) + 1)
    ys = np.arange(max(cy - r, 0), min(cy + r, N - 1) + 1)
    xs = np.arange(max(cx - r, 0), min(cx + r, N - 1) + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return (Z * N * N + Y * N + X).ravel()


def test_cd3d_256_sampled_chain_rows_and_solve(B, refs):
    P = W.config(5)
    N = 256
    A = B.CSRMatrix.from_host(P.A)
    As = P.A.to_scipy()
    d = P.d
    p = B.pp_build_poly(A, _up(P.v0), d)
    roots = p.roots()
    v = W.uniform(P.A.n, 9)
    y = B.pp_apply(A, p, _up(v)).cpu().numpy()
    rng = np.random.default_rng(12)
    centers = [(0, 0, 0), (N - 1, 17, 200)] + [tuple(rng.integers(0, N, 3)) for _ in range(2)]
    yinf = np.max(np.abs(y))
    # the whole vector, by the oracle's complex evaluation one root at a time
    yo = opoly.apply_poly(As, roots, v)
    err = np.max(np.abs(y - yo))
    assert err <= 1e-12 * np.max(np.abs(yo)), err
    del yo
    for c in centers:
        rows = _box_rows(N, c, d - 1)
        sub = As[rows][:, rows]
        yb = opoly.apply_poly(sub, roots, v[rows])
        i_loc = int(np.searchsorted(rows, c[0] * N * N + c[1] * N + c[2]))
        i_glob = rows[i_loc]
        assert abs(y[i_glob] - yb[i_loc]) <= 1e-12 * yinf, (c, y[i_glob], yb[i_loc])
    x, st = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=d, tol=P.tol, v0=_up(P.v0))
    xg = x.cpu().numpy()
    relres = np.linalg.norm(P.b - As @ xg) / np.linalg.norm(P.b)
    assert relres < P.tol and abs(relres - st.relres_true) <= 1e-3 * relres
    ref = refs.get("cd3d_256_pe100_d40")
    assert ref is not None, "run tests/golden/make_fullsize_refs.py --only cd3d_256_pe100_d40"
    _check_against_ref(ref, st, x, P.tol)
    # the automatic chain schedule at this size: slab-skewed over cache-sized slabs
    # with cached loads; the same bits as full-range non-temporal launches
    assert st.chain_cached and 0 < st.chain_slab_rows < P.A.n
    x1, st1 = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=d, tol=P.tol, v0=_up(P.v0), chain_group=1)
    assert st1.chain_slab_rows == 0 and not st1.chain_cached
    assert st1.iters == st.iters and torch.equal(x1, x)
    kw = dict(m=P.m, d=d, tol=P.tol, v0=_up(P.v0), precision="f32_ir", inner_tol=1e-5)
    x2, st2 = B.pp_gmres_solve(A, _up(P.b), **kw)
    x3, st3 = B.pp_gmres_solve(A, _up(P.b), chain_group=1, **kw)
    assert st2.chain_cached and st2.chain_slab_rows > st.chain_slab_rows  # 37 B a row
    assert st3.iters == st2.iters and torch.equal(x2, x3) and st2.relres_true < P.tol


def test_cd3d_128_fp32_refinement_counts(B, refs, cd3d_128):
    """FP32 inner PP-GMRES inside FP64 refinement: outer steps within one, inner
    Arnoldi steps within one per refinement step (or 2%), of the oracle's run."""
    P, A = cd3d_128
    ref = refs["cd3d_128_pe50_ir_d25"]
    x, st = B.pp_gmres_solve(A, _up(P.b), m=P.m, d=25, tol=P.tol, v0=_up(P.v0),
                             precision="f32_ir", inner_tol=ref["inner_tol"])
    assert st.relres_true < P.tol and ref["converged"]
    assert abs(st.outer - ref["outer"]) <= 1, (st.outer, ref["outer"])
    slack = max(ref["outer"], round(0.02 * ref["iters"]))
    assert abs(st.iters - ref["iters"]) <= slack, (st.iters, ref["iters"])
    xg = x.cpu().numpy()
    idx = np.asarray(ref["sample_idx"])
    # both solutions are within cond * tol of A^-1 b: compared at the sampled entries
    assert np.max(np.abs(xg[idx] - np.asarray(ref["x_sample"]))) <= 1e-8 * ref["x_absmax"]


def test_cd3d_160_slab_schedule_whole_solution(B):
    """R10 (ii) where the slab-skewed schedule runs: 20 steps of PP-GMRES(10), d = 6,
    on the 160^3 problem (Peclet 100), the oracle run to the same step count here,
    and the whole solutions compared."""
    P = W.config(5, N=160)
    A = B.CSRMatrix.from_host(P.A)
    m, d, cap = 10, 6, 20
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", B.PPWarning)     # stops at the step cap
        x, st = B.pp_gmres_solve(A, _up(P.b), m=m, d=d, tol=P.tol, v0=_up(P.v0),
                                 max_iters=cap)
    assert st.status == B.PP_WARN_NOT_CONVERGED and st.iters == cap
    assert st.chain_cached and 0 < st.chain_slab_rows < P.A.n
    xo, so = ogmres.pp_gmres(P.A.to_scipy(), P.b, m, P.tol, v0=P.v0, d=d, max_iters=st.iters)
    assert so.iters == st.iters and so.cycles == st.cycles
    assert st.spmvs == so.spmvs and st.dots == so.dots
    xg = x.cpu().numpy()
    rel = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    assert rel <= 1e-8, rel
    assert abs(st.relres_true - so.relres_true) <= 1e-6 * so.relres_true


def _residual_floor(M, x, b):
    """u * || |A| |x| + |b| || / ||b||: the rounding level of the computed residual
    b - A x itself, below which no solver's true residual can be certified."""
    import scipy.sparse as sp
    Aabs = sp.csr_matrix((np.abs(M.data), M.indices, M.indptr), shape=M.shape)
    return np.finfo(np.float64).eps * np.linalg.norm(Aabs @ np.abs(x) + np.abs(b)) / np.linalg.norm(b)


def test_adjoint_512_backward_solve(B, refs):
    """The backward solve of the 512^2 adjoint, on the right-hand side dL/dx = x - x_t
    at the direct solution (the stored oracle run's): PP-GMRES(50) on A^T with its
    own polynomial (d = 15, v0 seed 204), tol 1e-12.  Both the oracle and the
    library end on the stagnation test (three restart cycles in a row that reach
    tol in the Krylov estimate but do not cut the true residual by 10%) at FP64's
    attainable accuracy; the step counts agree within 2% and both final residuals
    lie below twice the rounding level of the computed residual b - A^T lam."""
    ref = refs["cd2d_512_pe20_adjoint_d15"]
    P = W.config(4)
    M = P.A.to_scipy()
    xd = oadj.DirectSolver(M).solve(P.b)
    rhs = xd - P.extra["x_target"]
    Mt = M.T.tocsr()
    At = B.CSRMatrix.from_host(W.CSR(Mt.shape[0], Mt.indptr.astype(np.int32),
                                     Mt.indices.astype(np.int32), Mt.data.copy()))
    with warnings.catch_warnings(record=True) as caught:
        warnings.simplefilter("always", B.PPWarning)
        lam, st = B.pp_gmres_solve(At, _up(rhs), m=P.m, d=ref["d"], tol=P.tol,
                                   v0=_up(P.extra["v0_adjoint"]))
    assert ref["stop"] == "stagnation" and not ref["converged"]
    assert st.status == B.PP_WARN_NOT_CONVERGED
    assert [w for w in caught if issubclass(w.category, B.PPWarning)]
    assert st.iters < 100000                          # not the step cap: the stagnation test
    assert abs(st.iters - ref["iters"]) <= max(1, round(0.02 * ref["iters"])), (st.iters,
                                                                                ref["iters"])
    lg = lam.cpu().numpy()
    floor = _residual_floor(Mt, lg, rhs)
    relres = np.linalg.norm(rhs - Mt @ lg) / np.linalg.norm(rhs)
    assert abs(relres - st.relres_true) <= 0.05 * relres
    # both stop at the rounding level of the residual itself (the oracle at 0.20 of
    # it, SuperLU's direct solution at 0.36): below it the two differ by rounding only
    assert ref["relres_true"] <= 2 * floor and st.relres_true <= 2 * floor, (
        ref["relres_true"], st.relres_true, floor)
    # the solution itself against the direct adjoint (the oracle's is 4.7e-13 away)
    lam_d = oadj.DirectSolver(M).solve(rhs, trans=True)
    assert np.linalg.norm(lg - lam_d) <= 1e-10 * np.linalg.norm(lam_d)


def test_adjoint_512(B, refs):
    from paper_1907_00072_amd.autograd import SolveConfig, pp_solve
    P = W.config(4)
    Ah = P.A
    xt = P.extra["x_target"]
    pattern = B.CSRMatrix.from_host(Ah)
    vals = _up(Ah.vals).requires_grad_(True)
    b = _up(P.b).requires_grad_(True)
    cfg = SolveConfig(m=P.m, d=P.d, tol=P.tol, v0=_up(P.v0), adj_v0=_up(P.extra["v0_adjoint"]))
    x = pp_solve(pattern, vals, b, cfg)
    loss = 0.5 * ((x - _up(xt)) ** 2).sum()
    with warnings.catch_warnings(record=True) as caught:
        # tol 1e-12 is below FP64's attainable accuracy for the adjoint system: the
        # backward solve ends on the stagnation test (PP_WARN_NOT_CONVERGED), as the
        # oracle's does on the same system
        warnings.simplefilter("always", B.PPWarning)
        loss.backward()
    assert all("not converged" in str(w.message) for w in caught
               if issubclass(w.category, B.PPWarning))
    gv = vals.grad.cpu().numpy()
    gb = b.grad.cpu().numpy()
    fwd, adj = cfg.stats[0][1], cfg.stats[1][1]
    ref = refs["cd2d_512_pe20_adjoint_d15"]
    assert fwd.relres_true < P.tol
    assert adj.status in (B.PP_OK, B.PP_WARN_NOT_CONVERGED) and adj.iters < 100000
    assert abs(adj.iters - ref["iters"]) <= max(1, round(0.02 * ref["iters"])), (adj.iters,
                                                                                 ref["iters"])
    M = Ah.to_scipy()
    xg = x.detach().cpu().numpy()
    gx = xg - xt
    Mt = M.T.tocsr()
    assert adj.relres_true <= 2 * _residual_floor(Mt, gb, gx)
    S = oadj.DirectSolver(M)
    xo, lam, gb_ref, gv_ref = oadj.adjoint_gradient(M, P.b, xt, solver=S)
    assert np.max(np.abs(gv - gv_ref)) <= 1e-6 * np.max(np.abs(gv_ref))
    assert np.max(np.abs(gb - gb_ref)) <= 1e-6 * np.max(np.abs(gb_ref))
    ents = P.extra["fd_entries"]
    fd = oadj.fd_gradient_vals(M, P.b, xt, ents, h=P.extra["fd_h"], solver=S, x=xo)
    assert np.max(np.abs(gv[ents] - fd)) <= 1e-6 * np.max(np.abs(gv_ref))


def test_recirc_257_ilu0_left_poly_right(B, refs):
    wl = W.ILU_WORKLOAD
    Ah, b = W.recirculating_flow(wl["N"], wl["eps"])
    As = Ah.to_scipy()
    A = B.CSRMatrix.from_host(Ah)
    M = B.pp_ilu0_factor(A)
    LU = oilu.ilu0(As)
    lu = B.pp_ilu0_values(M).cpu().numpy()
    assert np.max(np.abs(lu - LU.data)) <= 1e-12 * np.max(np.abs(LU.data))
    assert M.levels()[:2] == (2 * wl["N"] - 1, 2 * wl["N"] - 1)
    r = W.normal(Ah.n, 12)
    z = B.pp_ilu0_apply(M, _up(r)).cpu().numpy()
    zo = oilu.ilu0_solve(LU, r)
    assert np.linalg.norm(z - zo) <= 1e-12 * np.linalg.norm(zo)
    ref = refs["recirc2d_257_eps200_ilu0_d13"]
    x, st = B.pp_gmres_solve(A, _up(b), m=wl["m"], d=wl["d"], tol=wl["tol"],
                             v0=_up(W.uniform(Ah.n, wl["v0_seed"])), left_ilu=M)
    _check_against_ref(ref, st, x, wl["tol"])
    assert abs(st.relres_original - ref["relres_original"]) <= 1e-3 * ref["relres_original"]
