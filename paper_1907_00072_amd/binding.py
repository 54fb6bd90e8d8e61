"""ctypes binding of libpp (include/pp.h): argument marshalling only.

Every numerical step runs in the HIP library; this module turns torch CUDA
tensors into device pointers and the current torch stream into the hipStream_t
the C ABI takes.  If the shared library has not been built the import of the
functions below raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import warnings
from dataclasses import dataclass
from typing import Optional

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libpp.so")

PP_OK = 0
PP_ERR_ARG, PP_ERR_HIP, PP_ERR_NOMEM, PP_ERR_EIG, PP_ERR_SINGULAR = -1, -2, -3, -4, -5
PP_WARN_DEGREE_REDUCED, PP_WARN_NOT_CONVERGED, PP_WARN_NONFINITE, PP_WARN_CHOLESKY = 1, 2, 3, 4
PP_F64, PP_F32 = 0, 1
PP_PREC_F64, PP_PREC_F32_IR = 0, 1
PP_OP_RESIDUAL_POLY, PP_OP_PRODUCT = 0, 1
PP_LAYOUT_AUTO, PP_LAYOUT_CSR, PP_LAYOUT_SELL = 0, 1, 2
LAYOUTS = {"auto": PP_LAYOUT_AUTO, "csr": PP_LAYOUT_CSR, "sell": PP_LAYOUT_SELL}

EXPORTS = ("pp_build_poly", "pp_apply", "pp_gmres_solve", "pp_poly_roots", "pp_poly_from_roots",
           "pp_poly_free", "pp_roots_from_hessenberg", "pp_csr_transpose", "pp_csr_grad",
           "pp_release_workspace", "pp_status_string", "pp_version", "pp_build_poly_power",
           "pp_poly_coeffs", "pp_ilu0_factor", "pp_ilu0_apply", "pp_ilu0_values",
           "pp_ilu0_levels", "pp_ilu0_free", "pp_uniform_vector", "pp_last_error",
           "pp_apply_noalloc")


class pp_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_ind", ctypes.c_void_p), ("vals", ctypes.c_void_p), ("dtype", ctypes.c_int32),
                ("layout", ctypes.c_int32)]


class pp_opts(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("v0", ctypes.c_void_p), ("poly", ctypes.c_void_p), ("vals_f32", ctypes.c_void_p),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("op_form", ctypes.c_int32),
                ("left_jacobi", ctypes.c_int32), ("left_ilu", ctypes.c_void_p),
                ("chain_group", ctypes.c_int32), ("chain_slab_rows", ctypes.c_int32),
                ("v0_seed", ctypes.c_uint64)]


class pp_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("outer", ctypes.c_int32), ("nroots", ctypes.c_int32),
                ("history_len", ctypes.c_int32), ("spmvs", ctypes.c_int64),
                ("dots", ctypes.c_int64), ("relres_true", ctypes.c_double),
                ("relres_implicit", ctypes.c_double), ("t_total", ctypes.c_double),
                ("t_poly", ctypes.c_double), ("t_chain", ctypes.c_double),
                ("t_spmv", ctypes.c_double), ("t_orth", ctypes.c_double),
                ("t_host", ctypes.c_double), ("bytes_chain", ctypes.c_double),
                ("bytes_spmv", ctypes.c_double), ("bytes_orth", ctypes.c_double),
                ("launches_chain", ctypes.c_int64), ("relres_original", ctypes.c_double),
                ("layout_used", ctypes.c_int32), ("nnz_stored", ctypes.c_int64),
                ("chain_slab_rows", ctypes.c_int32), ("chain_cached", ctypes.c_int32)]


_lib = None


def lib():
    """Load libpp.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpp.so not built ({LIB_PATH}); run "
                          "`python -m paper_1907_00072_amd.csrc.build`")
    # torch first: its wheel carries its own HIP runtime (libamdhip64, same soname
    # as the system's), and the library's dependency then resolves to that copy.
    # Loaded before torch, the library would bring in the system runtime and torch
    # its own: two runtimes in one process, and the second to start finds no device.
    _torch()
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, D, VP = (ctypes.POINTER, ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                        ctypes.c_void_p)
    CSRP = P(pp_csr)
    L.pp_build_poly.argtypes = [CSRP, VP, I, VP, P(VP)]
    L.pp_build_poly_power.argtypes = [CSRP, VP, I, I, VP, P(VP), P(I)]
    L.pp_poly_coeffs.argtypes = [VP, P(D), I, P(I)]
    L.pp_apply.argtypes = [CSRP, VP, VP, VP, VP]
    L.pp_apply_noalloc.argtypes = [CSRP, VP, VP, VP, VP]
    L.pp_gmres_solve.argtypes = [CSRP, VP, VP, I, I, D, P(pp_opts), VP, P(pp_stats)]
    L.pp_poly_roots.argtypes = [VP, P(D), P(D), I, P(I)]
    L.pp_poly_from_roots.argtypes = [I64, P(D), P(D), I, I, P(VP)]
    L.pp_poly_free.argtypes = [VP]
    L.pp_poly_free.restype = None
    L.pp_roots_from_hessenberg.argtypes = [P(D), I, I, P(D), P(D)]
    L.pp_csr_transpose.argtypes = [CSRP, VP, VP, VP, VP]
    L.pp_csr_grad.argtypes = [CSRP, VP, VP, VP, VP]
    L.pp_release_workspace.argtypes = []
    L.pp_release_workspace.restype = None
    L.pp_status_string.argtypes = [I]
    L.pp_status_string.restype = ctypes.c_char_p
    L.pp_version.argtypes = []
    L.pp_version.restype = ctypes.c_char_p
    L.pp_last_error.argtypes = []
    L.pp_last_error.restype = ctypes.c_char_p
    I32 = ctypes.c_int32
    L.pp_ilu0_factor.argtypes = [CSRP, VP, P(VP)]
    L.pp_ilu0_apply.argtypes = [VP, VP, VP, VP]
    L.pp_ilu0_values.argtypes = [VP, VP, VP]
    L.pp_ilu0_levels.argtypes = [VP, P(I32), P(I32), P(I32)]
    L.pp_ilu0_free.argtypes = [VP]
    L.pp_ilu0_free.restype = None
    L.pp_uniform_vector.argtypes = [I64, ctypes.c_uint64, VP, VP]
    for name in ("pp_build_poly", "pp_build_poly_power", "pp_poly_coeffs", "pp_apply",
                 "pp_apply_noalloc",
                 "pp_gmres_solve", "pp_poly_roots",
                 "pp_poly_from_roots", "pp_roots_from_hessenberg", "pp_csr_transpose",
                 "pp_csr_grad", "pp_ilu0_factor", "pp_ilu0_apply", "pp_ilu0_values",
                 "pp_ilu0_levels", "pp_uniform_vector"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class PPError(RuntimeError):
    def __init__(self, code: int, where: str):
        detail = lib().pp_last_error().decode() if code < 0 else ""
        super().__init__(f"{where}: {pp_status_string(code)} (code {code})"
                         + (f" at {detail}" if detail else ""))
        self.code = code
        self.detail = detail


class PPWarning(UserWarning):
    pass


def _check(code: int, where: str) -> int:
    if code < 0:
        raise PPError(code, where)
    if code > 0:
        warnings.warn(f"{where}: {pp_status_string(code)}", PPWarning, stacklevel=3)
    return code


def pp_status_string(code: int) -> str:
    return lib().pp_status_string(int(code)).decode()


def pp_version() -> str:
    return lib().pp_version().decode()


def pp_release_workspace() -> None:
    lib().pp_release_workspace()


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev_vec(t, dtype, n, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype or t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor with {n} entries")
    return t


class CSRMatrix:
    """Square CSR matrix whose arrays live in device memory (torch tensors).

    ``layout`` ("auto", "csr" or "sell") is the storage the library uses for its
    sparse products (``pp_csr.layout``): "auto" builds a sliced copy per call
    unless its padding would be large.
    """

    def __init__(self, row_ptr, col_ind, vals, layout: str = "auto"):
        torch = _torch()
        if row_ptr.dtype != torch.int32 or col_ind.dtype != torch.int32:
            raise ValueError("row_ptr and col_ind must be int32")
        if vals.dtype not in (torch.float64, torch.float32):
            raise ValueError("vals must be float64 or float32")
        for t in (row_ptr, col_ind, vals):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("CSR arrays must be contiguous CUDA tensors")
        if col_ind.numel() != vals.numel():
            raise ValueError("col_ind and vals differ in length")
        if layout not in LAYOUTS:
            raise ValueError(f"layout must be one of {sorted(LAYOUTS)}")
        self.row_ptr, self.col_ind, self.vals = row_ptr, col_ind, vals
        self.layout = layout
        self.n = row_ptr.numel() - 1
        self.nnz = vals.numel()

    @property
    def dtype(self):
        return self.vals.dtype

    @classmethod
    def from_host(cls, A, device="cuda", dtype=None, validate=True, layout="auto"):
        """Upload a host CSR (``workloads.CSR`` or scipy csr_matrix).

        ``validate`` checks the structure on the host first (row pointers
        nondecreasing from 0 to nnz, column indices in range), so that a
        malformed matrix is rejected before any kernel reads it.
        """
        torch = _torch()
        if hasattr(A, "indptr"):
            rp, ci, va, n = A.indptr, A.indices, A.data, A.shape[0]
        else:
            rp, ci, va, n = A.row_ptr, A.col_ind, A.vals, A.n
        rp = np.ascontiguousarray(rp, dtype=np.int32)
        ci = np.ascontiguousarray(ci, dtype=np.int32)
        va = np.ascontiguousarray(va, dtype=np.float64)
        if validate:
            check_csr_host(rp, ci, n)
        dt = dtype or torch.float64
        return cls(torch.from_numpy(rp).to(device), torch.from_numpy(ci).to(device),
                   torch.from_numpy(va).to(device=device, dtype=dt), layout=layout)

    def with_vals(self, vals):
        return CSRMatrix(self.row_ptr, self.col_ind, vals, layout=self.layout)

    def with_layout(self, layout: str):
        return CSRMatrix(self.row_ptr, self.col_ind, self.vals, layout=layout)

    def c(self) -> pp_csr:
        torch = _torch()
        return pp_csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_ind.data_ptr(),
                      self.vals.data_ptr(), PP_F64 if self.vals.dtype == torch.float64 else PP_F32,
                      LAYOUTS[self.layout])


def check_csr_host(rp: np.ndarray, ci: np.ndarray, n: int) -> None:
    if rp.size != n + 1 or n <= 0:
        raise ValueError("row_ptr must have n+1 entries, n > 0")
    if rp[0] != 0 or rp[-1] != ci.size:
        raise ValueError("row_ptr must start at 0 and end at nnz")
    if np.any(np.diff(rp) < 0):
        raise ValueError("row_ptr must be nondecreasing")
    if ci.size and (ci.min() < 0 or ci.max() >= n):
        raise ValueError("column index out of range")


class Poly:
    """Owner of a pp_poly handle."""

    def __init__(self, handle: ctypes.c_void_p, n: int):
        self._h = handle
        self.n = n

    @property
    def handle(self):
        return self._h

    def roots(self) -> np.ndarray:
        return pp_poly_roots(self)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.pp_poly_free(h)
            self._h = None


class ILU0:
    """Owner of a pp_ilu handle: the ILU(0) factorisation of one matrix."""

    def __init__(self, handle: ctypes.c_void_p, n: int, nnz: int, device):
        self._h = handle
        self.n = n
        self.nnz = nnz
        self.device = device

    @property
    def handle(self):
        return self._h

    def levels(self):
        """(forward levels, backward levels, launches per apply)."""
        f, b, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().pp_ilu0_levels(self._h, ctypes.byref(f), ctypes.byref(b), ctypes.byref(k)),
               "pp_ilu0_levels")
        return f.value, b.value, k.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.pp_ilu0_free(h)
            self._h = None


def pp_ilu0_factor(A: CSRMatrix, stream=None) -> ILU0:
    """ILU(0) of an FP64 matrix with sorted columns and a stored diagonal in every row."""
    h = ctypes.c_void_p()
    _check(lib().pp_ilu0_factor(ctypes.byref(A.c()), _stream(stream), ctypes.byref(h)),
           "pp_ilu0_factor")
    return ILU0(h, A.n, A.nnz, A.vals.device)


def pp_ilu0_apply(M: ILU0, r, z=None, stream=None):
    """z = M^-1 r (z may be r)."""
    torch = _torch()
    _dev_vec(r, torch.float64, M.n, "r")
    if z is None:
        z = torch.empty_like(r)
    _dev_vec(z, torch.float64, M.n, "z")
    _check(lib().pp_ilu0_apply(M.handle, _ptr(r), _ptr(z), _stream(stream)), "pp_ilu0_apply")
    return z


def pp_ilu0_values(M: ILU0, stream=None):
    """The factors in the matrix's CSR order (L strictly below the diagonal, U on and above)."""
    torch = _torch()
    lu = torch.empty(M.nnz, dtype=torch.float64, device=M.device)
    _check(lib().pp_ilu0_values(M.handle, _ptr(lu), _stream(stream)), "pp_ilu0_values")
    return lu


def pp_uniform_vector(n: int, seed: int = 0, out=None, device="cuda", stream=None):
    """The seeded U(-1, 1) start vector the library draws when given no v0."""
    torch = _torch()
    if out is None:
        out = torch.empty(int(n), dtype=torch.float64, device=device)
    _dev_vec(out, torch.float64, int(n), "out")
    _check(lib().pp_uniform_vector(int(n), int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(out),
                                   _stream(stream)), "pp_uniform_vector")
    return out


def pp_build_poly(A: CSRMatrix, v0, d: int, stream=None) -> Poly:
    """Polynomial with d roots from start vector v0 (None: the seeded vector, seed 0)."""
    torch = _torch()
    if v0 is not None:
        _dev_vec(v0, torch.float64, A.n, "v0")
    h = ctypes.c_void_p()
    _check(lib().pp_build_poly(ctypes.byref(A.c()), _ptr(v0), int(d), _stream(stream),
                               ctypes.byref(h)), "pp_build_poly")
    return Poly(h, A.n)


def pp_build_poly_power(A: CSRMatrix, v0, deg: int, auto_degree: bool = False, stream=None):
    """The paper's power-basis polynomial; returns (Poly, info) with info = POTRF's status."""
    torch = _torch()
    if v0 is not None:
        _dev_vec(v0, torch.float64, A.n, "v0")
    h = ctypes.c_void_p()
    info = ctypes.c_int()
    _check(lib().pp_build_poly_power(ctypes.byref(A.c()), _ptr(v0), int(deg),
                                     1 if auto_degree else 0, _stream(stream), ctypes.byref(h),
                                     ctypes.byref(info)), "pp_build_poly_power")
    return Poly(h, A.n), info.value


def pp_poly_coeffs(poly: Poly) -> np.ndarray:
    c = np.zeros(64)
    k = ctypes.c_int()
    _check(lib().pp_poly_coeffs(poly.handle, c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 64,
                                ctypes.byref(k)), "pp_poly_coeffs")
    return c[: k.value].copy()


def pp_apply(A: CSRMatrix, poly: Poly, v, y=None, stream=None):
    _dev_vec(v, A.dtype, A.n, "v")
    if y is None:
        y = _torch().empty_like(v)
    _dev_vec(y, A.dtype, A.n, "y")
    _check(lib().pp_apply(ctypes.byref(A.c()), poly.handle, _ptr(v), _ptr(y), _stream(stream)),
           "pp_apply")
    return y


def pp_apply_noalloc(A: CSRMatrix, poly: Poly, v, y, stream=None):
    """y = p(A) v without allocation (the library's fixed per-GPU scratch array;
    n <= 2^21 rows in FP64, 2^22 in FP32).  ``y`` is caller-allocated."""
    _dev_vec(v, A.dtype, A.n, "v")
    _dev_vec(y, A.dtype, A.n, "y")
    _check(lib().pp_apply_noalloc(ctypes.byref(A.c()), poly.handle, _ptr(v), _ptr(y),
                                  _stream(stream)), "pp_apply_noalloc")
    return y


@dataclass
class Stats:
    status: int
    iters: int
    cycles: int
    outer: int
    nroots: int
    spmvs: int
    dots: int
    relres_true: float
    relres_implicit: float
    t_total: float
    t_poly: float
    t_chain: float
    t_spmv: float
    t_orth: float
    t_host: float
    bytes_chain: float = 0.0
    bytes_spmv: float = 0.0
    bytes_orth: float = 0.0
    launches_chain: int = 0
    relres_original: float = float("nan")
    history: Optional[np.ndarray] = None
    layout_used: str = ""
    nnz_stored: int = 0
    chain_slab_rows: int = 0  # slab-skewed chain schedule's slab rows (0: full-range)
    chain_cached: bool = False  # chain launches through the caches


def pp_gmres_solve(A: CSRMatrix, b, x=None, m: int = 50, d: int = 10, tol: float = 1e-8,
                   v0=None, poly: Optional[Poly] = None, precision: str = "f64",
                   max_iters: int = 0, inner_tol: float = 0.0, max_outer: int = 0,
                   vals_f32=None, history: int = 0, timing: bool = False, op_form: str = "pi",
                   left_jacobi: bool = False, left_ilu: Optional[ILU0] = None,
                   chain_group: int = 0, chain_slab_rows: int = 0, v0_seed: int = 0,
                   stream=None):
    """Solve A x = b; returns (x, Stats).  ``x`` (if given) is the start guess and is overwritten.

    ``v0``: start vector of the polynomial; None draws the seeded U(-1, 1) vector
    ``pp_uniform_vector(n, v0_seed)`` on the device.

    ``op_form``: "pi" applies A p(A) v as v - pi(A) v (default), "p" as A (p(A) v).
    ``left_ilu``: an ILU(0) of A (pp_ilu0_factor) applied on the left, the
    polynomial built for M^-1 A on the right.
    ``chain_group``: the chain's schedule (pp_opts.chain_group): 0 automatic, 1
    full-range non-temporal, >= 2 slab-skewed over slabs of ``chain_slab_rows`` rows.
    """
    torch = _torch()
    _dev_vec(b, torch.float64, A.n, "b")
    if x is None:
        x = torch.zeros_like(b)
    _dev_vec(x, torch.float64, A.n, "x")
    o = pp_opts()
    o.max_iters = int(max_iters)
    o.precision = {"f64": PP_PREC_F64, "f32_ir": PP_PREC_F32_IR}[precision]
    o.inner_tol = float(inner_tol)
    o.max_outer = int(max_outer)
    if v0 is not None:
        _dev_vec(v0, torch.float64, A.n, "v0")
        o.v0 = v0.data_ptr()
    if poly is not None:
        o.poly = poly.handle.value
    if vals_f32 is not None:
        _dev_vec(vals_f32, torch.float32, A.nnz, "vals_f32")
        o.vals_f32 = vals_f32.data_ptr()
    hist = None
    if history:
        hist = np.zeros(int(history), dtype=np.float64)
        o.history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        o.history_cap = int(history)
    o.timing = 1 if timing else 0
    o.op_form = {"pi": PP_OP_RESIDUAL_POLY, "p": PP_OP_PRODUCT}[op_form]
    o.left_jacobi = 1 if left_jacobi else 0
    if left_ilu is not None:
        o.left_ilu = left_ilu.handle.value
    o.chain_group = int(chain_group)
    o.chain_slab_rows = int(chain_slab_rows)
    o.v0_seed = int(v0_seed) & 0xFFFFFFFFFFFFFFFF
    st = pp_stats()
    rc = lib().pp_gmres_solve(ctypes.byref(A.c()), _ptr(b), _ptr(x), int(m), int(d), float(tol),
                              ctypes.byref(o), _stream(stream), ctypes.byref(st))
    _check(rc, "pp_gmres_solve")
    s = Stats(st.status, st.iters, st.cycles, st.outer, st.nroots, st.spmvs, st.dots,
              st.relres_true, st.relres_implicit, st.t_total, st.t_poly, st.t_chain, st.t_spmv,
              st.t_orth, st.t_host, st.bytes_chain, st.bytes_spmv, st.bytes_orth,
              st.launches_chain, st.relres_original,
              hist[: st.history_len].copy() if hist is not None else None,
              {PP_LAYOUT_CSR: "csr", PP_LAYOUT_SELL: "sell"}.get(st.layout_used, ""),
              st.nnz_stored, st.chain_slab_rows, bool(st.chain_cached))
    return x, s


def pp_poly_roots(poly: Poly) -> np.ndarray:
    cap = 512
    re = np.zeros(cap)
    im = np.zeros(cap)
    d = ctypes.c_int()
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().pp_poly_roots(poly.handle, re.ctypes.data_as(dp), im.ctypes.data_as(dp), cap,
                               ctypes.byref(d)), "pp_poly_roots")
    return re[: d.value] + 1j * im[: d.value]


def pp_poly_from_roots(n: int, roots, dtype: str = "f64") -> Poly:
    roots = np.asarray(roots, dtype=np.complex128)
    re = np.ascontiguousarray(roots.real)
    im = np.ascontiguousarray(roots.imag)
    dp = ctypes.POINTER(ctypes.c_double)
    h = ctypes.c_void_p()
    _check(lib().pp_poly_from_roots(int(n), re.ctypes.data_as(dp), im.ctypes.data_as(dp),
                                    roots.size, PP_F64 if dtype == "f64" else PP_F32,
                                    ctypes.byref(h)), "pp_poly_from_roots")
    return Poly(h, n)


def pp_roots_from_hessenberg(Hbar: np.ndarray) -> np.ndarray:
    """Host-only: Leja-ordered harmonic Ritz values of an (s+1) x s Hessenberg matrix."""
    H = np.asfortranarray(np.asarray(Hbar, dtype=np.float64))
    s = H.shape[1]
    if H.shape[0] != s + 1:
        raise ValueError("Hbar must be (s+1) x s")
    re = np.zeros(s)
    im = np.zeros(s)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().pp_roots_from_hessenberg(H.ctypes.data_as(dp), s + 1, s,
                                          re.ctypes.data_as(dp), im.ctypes.data_as(dp)),
           "pp_roots_from_hessenberg")
    return re + 1j * im


def pp_csr_transpose(A: CSRMatrix, stream=None) -> CSRMatrix:
    torch = _torch()
    rp = torch.empty(A.n + 1, dtype=torch.int32, device=A.vals.device)
    ci = torch.empty(A.nnz, dtype=torch.int32, device=A.vals.device)
    va = torch.empty(A.nnz, dtype=A.vals.dtype, device=A.vals.device)
    _check(lib().pp_csr_transpose(ctypes.byref(A.c()), _ptr(rp), _ptr(ci), _ptr(va),
                                  _stream(stream)), "pp_csr_transpose")
    return CSRMatrix(rp, ci, va, layout=A.layout)


def pp_csr_grad(A: CSRMatrix, lam, x, g=None, stream=None):
    torch = _torch()
    _dev_vec(lam, torch.float64, A.n, "lam")
    _dev_vec(x, torch.float64, A.n, "x")
    if g is None:
        g = torch.empty(A.nnz, dtype=torch.float64, device=A.vals.device)
    _check(lib().pp_csr_grad(ctypes.byref(A.c()), _ptr(lam), _ptr(x), _ptr(g), _stream(stream)),
           "pp_csr_grad")
    return g
