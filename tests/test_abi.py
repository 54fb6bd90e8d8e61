"""CPU tests of the C ABI: the library loads, exports every declared symbol, and
its host-only numerics (harmonic Ritz eigenproblem, Leja order, root tables)
agree with numpy / the oracle.  No device work is done here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import poly as opoly
from paper_1907_00072_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(not os.path.exists(B.LIB_PATH), reason="libpp.so not built")


def _declared():
    src = open(os.path.join(ROOT, "include", "pp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?(pp_[a-z0-9_]+)\(", src, re.M)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) == 22
    L = B.lib()
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(names) == set(B.EXPORTS)


def test_version_and_status_strings():
    assert "gfx950" in B.pp_version()
    for code in (0, -1, -2, -3, -4, -5, 1, 2, 3):
        assert B.pp_status_string(code) != "unknown status"
    assert B.pp_status_string(99) == "unknown status"
    # no device call has failed on this thread: the failure record is empty
    assert B.lib().pp_last_error() == b""


def _rand_hess(s, seed, sub_scale=1.0):
    rng = np.random.default_rng(seed)
    H = np.triu(rng.standard_normal((s + 1, s)), -1)
    H[np.arange(1, s + 1), np.arange(s)] *= sub_scale
    return H


def _sorted(z):
    return np.array(sorted(np.asarray(z, complex), key=lambda t: (round(t.real, 9), t.imag)))


@pytest.mark.parametrize("s", [1, 2, 3, 5, 8, 13, 21, 40, 64, 100])
def test_francis_qr_eigenvalues_match_numpy(s):
    """h_{s+1,s} = 0: the harmonic Ritz matrix is H_s itself, so the roots are eig(H_s)."""
    for seed in range(4):
        H = _rand_hess(s, 100 * s + seed)
        H[s, s - 1] = 0.0
        got = B.pp_roots_from_hessenberg(H)
        ref = np.linalg.eigvals(H[:s, :s])
        # match every eigenvalue to its nearest reference value
        ref_l = list(ref)
        for g in got:
            j = int(np.argmin([abs(g - r) for r in ref_l]))
            assert abs(g - ref_l[j]) <= 1e-9 * max(1.0, abs(ref_l[j])), (s, seed, g, ref_l[j])
            ref_l.pop(j)


def test_complex_roots_are_exact_conjugate_pairs():
    H = _rand_hess(30, 7)
    got = B.pp_roots_from_hessenberg(H)
    i = 0
    while i < got.size:
        if got[i].imag != 0:
            assert got[i].imag > 0 and got[i + 1] == np.conj(got[i])
            i += 2
        else:
            i += 1


@pytest.mark.parametrize("seed,n,d", [(1, 60, 6), (2, 90, 10), (3, 200, 25)])
def test_harmonic_ritz_and_leja_match_oracle(seed, n, d):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) / np.sqrt(n) + 1.5 * np.eye(n)
    Q, Hbar, s = opoly.arnoldi(A, rng.uniform(-1, 1, n), d)
    got = B.pp_roots_from_hessenberg(Hbar)
    ref = opoly.leja_order(opoly.harmonic_ritz(Hbar))
    assert got.size == ref.size
    # same set, and the same Leja sequence unless two candidates nearly tie
    assert np.allclose(_sorted(got), _sorted(ref), rtol=1e-9, atol=1e-12)
    assert np.allclose(got, ref, rtol=1e-8, atol=1e-12)


def test_symmetric_hessenberg_gives_real_roots():
    rng = np.random.default_rng(4)
    n = 80
    M = rng.standard_normal((n, n))
    A = M @ M.T / n + np.eye(n)
    Q, Hbar, s = opoly.arnoldi(A, rng.uniform(-1, 1, n), 12)
    got = B.pp_roots_from_hessenberg(Hbar)
    assert np.all(got.imag == 0) and np.all(got.real > 0)


def test_singular_hessenberg_is_an_error():
    H = np.zeros((4, 3))
    H[0, 0] = 1.0
    H[1, 0] = 1.0
    with pytest.raises(B.PPError) as e:
        B.pp_roots_from_hessenberg(H)
    assert e.value.code == B.PP_ERR_SINGULAR


def test_poly_from_roots_roundtrip_and_validation():
    roots = np.array([3.0, 1.0 + 2.0j, 1.0 - 2.0j, -0.5])
    p = B.pp_poly_from_roots(100, roots)
    assert np.array_equal(B.pp_poly_roots(p), roots)
    with pytest.raises(B.PPError) as e:
        B.pp_poly_from_roots(100, np.array([1.0 - 2.0j, 1.0 + 2.0j]))
    assert e.value.code == B.PP_ERR_ARG
    with pytest.raises(B.PPError):
        B.pp_poly_from_roots(100, np.array([1.0 + 2.0j, 1.1 - 2.0j]))
    with pytest.raises(B.PPError) as e:
        B.pp_poly_from_roots(100, np.array([0.0, 2.0]))
    assert e.value.code == B.PP_ERR_SINGULAR
    empty = B.pp_poly_from_roots(10, np.array([], dtype=complex))
    assert B.pp_poly_roots(empty).size == 0


def test_host_validation_rejects_malformed_csr():
    with pytest.raises(ValueError):
        B.check_csr_host(np.array([0, 2, 1], np.int32), np.array([0, 1], np.int32), 2)
    with pytest.raises(ValueError):
        B.check_csr_host(np.array([0, 1, 2], np.int32), np.array([0, 2], np.int32), 2)
    with pytest.raises(ValueError):
        B.check_csr_host(np.array([0, 1, 3], np.int32), np.array([0, 1], np.int32), 2)
    B.check_csr_host(np.array([0, 1, 1, 2], np.int32), np.array([0, 2], np.int32), 3)


def _c_layout(struct, fields):
    """sizeof and offsetof of a pp.h struct, measured by compiling a tiny C program."""
    import shutil
    import subprocess
    import tempfile
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    body = "".join(f'  printf("%zu\\n", offsetof({struct}, {f}));\n' for f in fields)
    src = ("#include <stddef.h>\n#include <stdio.h>\n#include \"pp.h\"\nint main(void) {\n"
           f'  printf("%zu\\n", sizeof({struct}));\n{body}  return 0;\n}}\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(root, "include"), c, "-o", exe],
                       check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(v) for v in out[1:]]


@pytest.mark.parametrize("name", ["pp_csr", "pp_opts", "pp_stats"])
def test_ctypes_structs_match_the_c_header(name):
    from paper_1907_00072_amd import binding
    cls = getattr(binding, name)
    fields = [f[0] for f in cls._fields_]
    size, offsets = _c_layout(name, fields)
    assert ctypes.sizeof(cls) == size
    assert [getattr(cls, f).offset for f in fields] == offsets


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
