"""GPU: pp_apply_noalloc, the allocation-free variant of pp_apply.

It runs the chain on A's CSR arrays with its temporaries in the library's fixed
per-GPU scratch array.  Checked through the C ABI against pp_apply on two calls
in a row, the second smaller than the first (the first at the largest n the
array admits, 2^21 rows in FP64): bit for bit against pp_apply on the CSR layout
(the same kernels), within 1e-12 of max |y| against pp_apply's default sliced
layout and the oracle's complex-arithmetic evaluation; then an FP32 call, and an
n above the limit, which is rejected before any kernel runs.
"""
import numpy as np
import pytest

from oracle import poly as opoly
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


def _call(B, A, poly, v, y):
    """pp_apply_noalloc through the C ABI; returns its status code."""
    L = B.lib()
    return L.pp_apply_noalloc(B.ctypes.byref(A.c()), poly.handle, B._ptr(v), B._ptr(y),
                              B._stream(None))


def _roots(P, d):
    """Leja-ordered roots of the oracle's polynomial for a (small) problem."""
    roots, _ = opoly.build_poly(P.A.to_scipy(), P.v0, d)
    return roots


def _mixed_roots():
    """Four conjugate pairs (a 24^3 convection-diffusion polynomial) and four real
    roots (a 40^2 one), in modified Leja order: both kinds of chain step."""
    pairs = _roots(W.config(2, N=24), 12)[:8]
    reals = _roots(W.config(1, N=40), 8)[:4]
    return opoly.leja_order(np.concatenate([pairs, reals]))


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_matches_pp_apply_two_calls(B, order):
    cases = [W.config(2), W.config(1)]             # n = 2^21 (the limit), then n = 4096
    assert cases[0].A.n == 1 << 21 and cases[1].A.n < cases[0].A.n
    small_roots = _mixed_roots()
    assert np.sum(small_roots.imag != 0) == 8 and np.sum(small_roots.imag == 0) == 4
    for P in cases:
        A = B.CSRMatrix.from_host(P.A)
        poly = B.pp_poly_from_roots(P.A.n, small_roots)
        v = _up(W.uniform(P.A.n, 31))
        y = torch.full_like(v, float("nan"))       # stale contents must not matter
        assert _call(B, A, poly, v, y) == B.PP_OK, B.lib().pp_last_error()
        y_csr = B.pp_apply(A.with_layout("csr"), poly, v)
        assert torch.equal(y, y_csr)
        y_auto = B.pp_apply(A, poly, v)
        ymax = float(y_auto.abs().max())
        assert float((y - y_auto).abs().max()) <= 1e-12 * ymax
        if P.A.n <= 4096:
            yo = opoly.apply_poly(P.A.to_scipy(), small_roots, v.cpu().numpy())
            assert np.max(np.abs(y.cpu().numpy() - yo)) <= 1e-12 * np.max(np.abs(yo))
        del A, v, y, y_csr, y_auto


def test_noalloc_fp32_and_size_limit(B):
    P = W.config(1, N=40)
    roots = _roots(P, 8)
    A32 = B.CSRMatrix.from_host(P.A, dtype=torch.float32)
    poly = B.pp_poly_from_roots(P.A.n, roots, dtype="f32")
    v = _up(W.uniform(P.A.n, 32), torch.float32)
    y = torch.empty_like(v)
    assert _call(B, A32, poly, v, y) == B.PP_OK
    assert torch.equal(y, B.pp_apply(A32.with_layout("csr"), poly, v))
    # one row past the FP64 limit: a diagonal matrix, rejected with the reason stated
    n = (1 << 21) + 1
    ident = W.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                  np.full(n, 2.0))
    Abig = B.CSRMatrix.from_host(ident)
    pbig = B.pp_poly_from_roots(n, [2.0])
    vb = torch.ones(n, dtype=torch.float64, device="cuda:0")
    yb = torch.zeros_like(vb)
    assert _call(B, Abig, pbig, vb, yb) == B.PP_ERR_ARG
    assert b"scratch" in B.lib().pp_last_error()
    assert float(yb.abs().max()) == 0.0            # nothing ran
    # the same call fits pp_apply, which allocates its own workspace
    assert float((B.pp_apply(Abig, pbig, vb) - 0.5).abs().max()) == 0.0
