"""Write tests/golden/fullsize_refs.json: oracle results at the full workload sizes.

Runs only the CPU oracle (oracle/) on the seeded workloads: the full solves are
too slow to repeat inside a GPU test, so their iteration counts and sampled
solution entries are stored here once.  Usage (from the repository root):

    python tests/golden/make_fullsize_refs.py [--only NAME ...]

Takes tens of minutes on an 8-core host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import adjoint as oa  # noqa: E402
from oracle import gmres as og  # noqa: E402
from oracle import ilu as oi  # noqa: E402
from oracle import poly as op  # noqa: E402
from paper_1907_00072_amd import workloads as W  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "fullsize_refs.json")
NSAMPLE = 64


def sample_idx(n, seed=11):
    return np.sort(np.random.default_rng(seed).choice(n, size=NSAMPLE, replace=False))


def record(name, P, d, x, st, t, extra=None):
    idx = sample_idx(P.A.n)
    rec = {"workload": P.name, "n": P.A.n, "nnz": P.A.nnz, "m": P.m, "d": d, "tol": P.tol,
           "iters": st.iters, "cycles": st.cycles, "spmvs": st.spmvs, "dots": st.dots,
           "relres_true": st.relres_true, "converged": st.converged,
           "x_norm": float(np.linalg.norm(x)), "x_absmax": float(np.max(np.abs(x))),
           "sample_idx": idx.tolist(), "x_sample": x[idx].tolist(),
           "roots_re": [] if st.roots is None else np.real(st.roots).tolist(),
           "roots_im": [] if st.roots is None else np.imag(st.roots).tolist(),
           "seconds": t}
    if extra:
        rec.update(extra)
    print(f"{name}: iters {st.iters} cycles {st.cycles} relres {st.relres_true:.3e} "
          f"({t:.0f}s)", flush=True)
    return rec


def run(names):
    refs = json.load(open(OUT)) if os.path.exists(OUT) else {}
    jobs = []
    for d in (25, 10, 40, 0):
        jobs.append((f"cd3d_128_pe50_d{d}", 2, d))
    jobs.append(("stencil27_96_ir_d25", 3, 25))
    jobs.append(("stencil27_96_f64_d25", 3, -25))
    jobs.append(("cd3d_256_pe100_d40", 5, 40))
    jobs.append(("recirc2d_257_eps200_ilu0_d13", "ilu", 13))
    jobs.append(("cd2d_512_pe20_adjoint_d15", "adjoint", 15))
    jobs.append(("cd3d_128_pe50_ir_d25", "ir128", 25))
    for name, cfg, d in jobs:
        if names and name not in names:
            continue
        if cfg == "ilu":
            # Section VI's second example: ILU(0) left, polynomial of M^-1 A right
            wl = W.ILU_WORKLOAD
            Ah, b = W.recirculating_flow(wl["N"], wl["eps"])
            P = W.Problem(wl["name"], Ah, b, W.uniform(Ah.n, wl["v0_seed"]), m=wl["m"], d=d,
                          tol=wl["tol"])
            t0 = time.time()
            x, st = oi.pp_gmres_left_ilu0(Ah.to_scipy(), b, P.m, P.tol, v0=P.v0, d=d,
                                          max_iters=20000)
            refs[name] = record(name, P, d, x, st, time.time() - t0,
                                {"relres_original": st.relres_original})
            json.dump(refs, open(OUT, "w"), indent=1)
            continue
        if cfg == "adjoint":
            # the backward solve of the 512^2 adjoint: PP-GMRES on A^T with its own
            # polynomial (d = 15, v0 seed 204), right-hand side dL/dx = x - x_t for
            # L = 0.5 ||x - x_t||^2 at the direct solution x = A^-1 b
            P = W.config(4)
            A = P.A.to_scipy()
            xd = oa.DirectSolver(A).solve(P.b)
            rhs = xd - P.extra["x_target"]
            At = A.T.tocsr()
            t0 = time.time()
            lam, st = og.pp_gmres(At, rhs, P.m, P.tol, v0=P.extra["v0_adjoint"], d=d,
                                  max_iters=5000)
            stop = ("converged" if st.converged else
                    "iteration cap" if st.iters >= 5000 else "stagnation")
            rec = record(name, P, d, lam, st, time.time() - t0,
                         {"stop": stop, "true_history": st.true_history,
                          "relres_implicit": st.relres_implicit,
                          "rhs": "x - x_t, x = A^-1 b by SuperLU"})
            refs[name] = rec
            json.dump(refs, open(OUT, "w"), indent=1)
            continue
        if cfg == "ir128":
            # FP32 inner PP-GMRES inside FP64 refinement on the 128^3 problem
            P = W.config(2)
            A = P.A.to_scipy()
            t0 = time.time()
            x, st = og.pp_gmres_ir(A, P.b, P.m, d, P.tol, P.v0, inner_tol=1e-5, max_outer=50)
            rec = record(name, P, d, x, st, time.time() - t0,
                         {"outer": st.outer, "inner_tol": 1e-5,
                          "true_history": st.true_history})
            refs[name] = rec
            json.dump(refs, open(OUT, "w"), indent=1)
            continue
        P = W.config(cfg)
        A = P.A.to_scipy()
        t0 = time.time()
        if cfg == 3 and d > 0:
            x, st = og.pp_gmres_ir(A, P.b, P.m, d, P.tol, P.v0,
                                   inner_tol=P.extra["inner_tol"], max_outer=50)
            rec = record(name, P, d, x, st, time.time() - t0, {"outer": st.outer})
        else:
            dd = abs(d)
            x, st = og.pp_gmres(A, P.b, P.m, P.tol, v0=P.v0, d=dd, max_iters=20000)
            rec = record(name, P, dd, x, st, time.time() - t0)
        refs[name] = rec
        json.dump(refs, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None)
    run(ap.parse_args().only)
