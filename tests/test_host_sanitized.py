"""The library's host numerics (Francis QR, harmonic Ritz values, modified Leja
order, the chain's step table, the power basis' Cholesky) built for the CPU with
AddressSanitizer and UndefinedBehaviorSanitizer, run on random and degenerate
inputs, and checked against NumPy and the oracle.  Any sanitizer report fails
the test (-fno-sanitize-recover)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import poly as opoly

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1907_00072_amd", "csrc", "host_numerics.cpp")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "host_numerics.h"
// stdin: number of cases, then per case: kind s, and the data
//   kind 0: harmonic Ritz + Leja + step table of an (s+1) x s Hessenberg (column-major)
//   kind 1: Cholesky of an s x s symmetric matrix (column-major), then a solve
int main() {
  int ncase = 0;
  if (scanf("%d", &ncase) != 1) return 2;
  for (int c = 0; c < ncase; ++c) {
    int kind = 0, s = 0;
    if (scanf("%d %d", &kind, &s) != 2) return 2;
    if (kind == 0) {
      std::vector<double> H((size_t)(s + 1) * s);
      for (double &v : H) if (scanf("%lf", &v) != 1) return 2;
      std::vector<double> wr, wi, lr, li;
      int rc = ppn::harmonic_ritz(H.data(), s + 1, s, wr, wi);
      if (rc == 0) rc = ppn::leja_order(wr, wi, lr, li);
      std::vector<ppn::Step> steps;
      if (rc == 0) rc = ppn::step_table(lr, li, steps);
      printf("%d %zu\n", rc, lr.size());
      for (size_t k = 0; k < lr.size(); ++k) printf("%.17g %.17g\n", lr[k], li[k]);
      printf("%zu\n", steps.size());
    } else {
      std::vector<double> G((size_t)s * s), rhs(s), y(s);
      for (double &v : G) if (scanf("%lf", &v) != 1) return 2;
      for (double &v : rhs) if (scanf("%lf", &v) != 1) return 2;
      std::vector<double> R;
      const int info = ppn::cholesky_upper(G.data(), s, s, R);
      printf("%d\n", info);
      if (info == 0) {
        ppn::cholesky_solve(R, s, rhs.data(), y.data());
        for (double v : y) printf("%.17g\n", v);
      }
    }
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("hostsan")
    drv = d / "driver.cpp"
    drv.write_text(DRIVER)
    exe = d / "driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I" + os.path.join(ROOT, "paper_1907_00072_amd", "csrc"),
           "-I" + os.path.join(ROOT, "include"), SRC, str(drv), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer build failed: " + r.stderr[-400:])
    return str(exe)


def _hess(s, rng, sub=1.0):
    H = np.triu(rng.standard_normal((s + 1, s)), -1)
    H[np.arange(1, s + 1), np.arange(s)] = sub * (0.5 + rng.random(s))
    return H


def _run(exe, cases):
    lines = [str(len(cases))]
    for kind, s, data in cases:
        lines.append(f"{kind} {s}")
        lines.append(" ".join(repr(float(v)) for v in data))
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout.split()


def test_roots_match_oracle_under_sanitizers(driver):
    rng = np.random.default_rng(2024)
    shapes = [1, 2, 3, 5, 8, 13, 21, 40, 64]
    Hs = [_hess(s, rng) for s in shapes]
    # exact symmetric tridiagonal (real roots) and a repeated-eigenvalue case
    T = np.zeros((7, 6))
    for j in range(6):
        T[j, j] = 2.0
        T[j + 1, j] = 1.0
        if j > 0:
            T[j - 1, j] = 1.0
    Hs.append(T)
    out = _run(driver, [(0, H.shape[1], H.T.ravel()) for H in Hs])
    k = 0
    for H in Hs:
        s = H.shape[1]
        rc, cnt = int(out[k]), int(out[k + 1])
        k += 2
        got = np.array([float(out[k + 2 * i]) + 1j * float(out[k + 2 * i + 1])
                        for i in range(cnt)])
        k += 2 * cnt
        nsteps = int(out[k])
        k += 1
        assert rc == 0 and cnt == s
        ref = opoly.harmonic_ritz(H)
        a = np.sort_complex(got)
        b = np.sort_complex(np.asarray(ref, complex))
        assert np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)) <= 1e-8, s
        # Leja: the first root has the largest modulus; conjugate pairs adjacent
        assert abs(abs(got[0]) - np.max(np.abs(got))) <= 1e-12 * np.max(np.abs(got))
        i = 0
        while i < cnt:
            if got[i].imag != 0.0:
                assert got[i].imag > 0 and got[i + 1] == np.conj(got[i])
                i += 2
            else:
                i += 1
        assert nsteps == cnt - int(np.sum(got.imag > 0))


def test_cholesky_under_sanitizers(driver):
    rng = np.random.default_rng(7)
    cases, refs = [], []
    for s in (1, 2, 5, 12, 30):
        M = rng.standard_normal((s, s))
        G = M @ M.T + s * np.eye(s)
        rhs = rng.standard_normal(s)
        cases.append((1, s, np.concatenate([G.T.ravel(), rhs])))
        refs.append(("ok", np.linalg.solve(G, rhs)))
    # indefinite: the first non-positive pivot is reported (POTRF's info)
    G = np.diag([4.0, 1.0, -2.0, 3.0])
    cases.append((1, 4, np.concatenate([G.ravel(), np.ones(4)])))
    refs.append(("info", 3))
    out = _run(driver, cases)
    k = 0
    for kind, ref in refs:
        info = int(out[k])
        k += 1
        if kind == "ok":
            assert info == 0
            y = np.array([float(v) for v in out[k:k + ref.size]])
            k += ref.size
            assert np.max(np.abs(y - ref)) <= 1e-10 * np.max(np.abs(ref))
        else:
            assert info == ref
