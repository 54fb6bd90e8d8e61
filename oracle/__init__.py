"""CPU FP64 oracle for polynomial-preconditioned GMRES(m).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, obviously
correct reference that the HIP path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the library (``paper_1907_00072_amd``) never does, and the two
share no code: the only common module is the seeded input generator
``paper_1907_00072_amd.workloads``, which holds none of the method's
arithmetic.

Contents
--------
poly     -- Arnoldi on v0, harmonic Ritz values, modified Leja order,
            p(A)v in complex arithmetic, and the paper's power-basis /
            normal-equation construction (Section II, eqs. (1)-(2)).
gmres    -- right-preconditioned restarted GMRES(m) with two-pass classical
            Gram-Schmidt (Section III), and the FP32-inside-FP64 iterative
            refinement loop.
adjoint  -- direct-solve adjoint gradient and Sherman-Morrison central
            differences for dL/dA_ij and dL/db.
ilu      -- ILU(0) factors, their triangular solves and dependency levels,
            and GMRES(m) with ILU(0) on the left and the polynomial on the
            right (Section VI, second example).
rng      -- the seeded U(-1, 1) start vector (Section V) drawn when the
            caller gives none: Philox4x64-10, written from its published
            definition.

Every function works in the floating-point type of its vector inputs
(float64 unless a float32 vector is passed), with all small dense algebra
(Hessenberg, least squares, eigenvalues) in float64.

Pins: every function is checked in ``tests/test_oracle_*.py`` against
closed forms, brute force, library routines on special cases and the
numbers printed in Section V (the Laplacian worked example).  Parity
unpinned: Table I and the counts of Sections III-IV (their Matrix Market
matrices and random vectors are not available).
"""
from . import poly, gmres, adjoint, ilu, rng  # noqa: F401
