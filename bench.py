#!/usr/bin/env python3
"""Benchmark: polynomial-preconditioned GMRES time-to-tolerance on one MI355X.

Workload (default): 3D convection-diffusion, 7-point central differences on a
256^3 grid (n = 16.8M, 117M nonzeros, FP64), Peclet 100, wind (1, .5, .25),
b ~ N(0,1) seed 7, polynomial start vector U(-1,1) seed 105; PP-GMRES(30) with
d = 40 roots, tol 1e-8.  Inputs are generated on the host, uploaded once, and
resident in HBM before the timed region.

One step = one complete solve from x0 = 0: the polynomial build (40 Arnoldi
steps on v0, harmonic Ritz eigenproblem, Leja order), then restarted GMRES(30)
with the p(A) chain, the outer product and CGS2 in every Arnoldi step, to the
true relative residual < 1e-8.  `value` is the mean time-to-tolerance (s).

Extra legs on the same matrix: the FP32-inside-FP64 refinement solve and plain
GMRES(30) (no polynomial), each one timed solve after a warm-up.

The library runs its sparse products on a sliced copy of the CSR matrix that
it builds on the device at the start of each solve (64-row slices stored by
diagonal: values plus a 64-byte descriptor per slice, no column indices; 0.11% padding on
this stencil); the copy is part of every timed solve.  The `csr` leg times the
same solve on the caller's CSR arrays.

The chain's launches follow the library's automatic schedule: at this size a
launch's working set (73 B a row) is far beyond the 256 MiB Infinity Cache, so
each Arnoldi step's launches run in the slab-skewed order (Section VII) over
3.1M-row slabs with cached loads, every slab's matrix read from HBM once and
re-read from the cache by the following launches.  The `fullrange` leg times
the same solve with full-range, non-temporal launches (identical results).

roofline: the fused product + root-update chain kernel dominates (39 of every
40 products).  Its achieved bandwidth is the algorithmic bytes of the
event-timed chain launches (8 nnz_stored + n bytes of matrix: the values and
one 64-byte descriptor per 64-row slice; plus 16 n of vectors for a middle
real-root step) over their event-timed duration, both accumulated by the
library over the timed solves; a launch is one kernel launch (one slab's part
of a product under the slab-skewed schedule).  With the cache re-reads this
rate can exceed what HBM alone delivers.

cpu_baseline: the CPU oracle (NumPy/SciPy, complex-arithmetic product form) on
a bounded sample of the same solve (one p(A)v with the GPU's roots, one product,
one Gram-Schmidt column unit, all on the full matrix), scaled to the GPU solve's
step, cycle, build-product and CGS2 column counts; `cores` is the number of
threads the sample kept busy (CPU time over wall time).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-1e-8 rel. residual (s) PP-GMRES vs GMRES; SpMV HBM GB/s % of peak"
HBM_PEAK_GBPS = 8000.0
# measured on MI355X with a flat FP64 copy kernel (one element per thread): buffers far
# larger than the 256 MiB Infinity Cache, and two 128 MiB buffers that stay in it
HBM_COPY_GBPS = 6310.0
CACHE_COPY_GBPS = 7370.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=256, help="grid points per axis (256 = headline)")
    ap.add_argument("--config", type=int, default=5,
                    help="workload configuration (5 = the headline 256^3 problem; 1-4 time the "
                         "same kind of line on the others, at their own m, d and tol)")
    ap.add_argument("--legs", default="ir,plain,power,csr,jacobi,fullrange,ilu,adjoint",
                    help="comma list of extra legs: ir, plain, power, csr, jacobi, fullrange, ilu, "
                         "adjoint, none")
    ap.add_argument("--plain-max-iters", type=int, default=30000)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-full-solve", metavar="OUT_JSON", default=None,
                    help="instead of the default line: time the oracle's complete solve of the "
                         "workload on this host (minutes at 256^3; no GPU used), then the "
                         "cpu_baseline estimator on the same host, and write both to OUT_JSON")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the default line: time-to-tol on every workload configuration "
                         "(one JSON object)")
    ap.add_argument("--copy-check", type=int, default=1,
                    help="also time torch's 2 GiB device copy (the reference kernel that scales "
                         "the rocprofv3 byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1907_00072_amd import binding as B
    from paper_1907_00072_amd import workloads as W

    if args.cpu_full_solve:
        P = W.config(5, N=args.grid)
        As = P.A.to_scipy()
        log(f"cpu full solve: oracle on {P.name} grid {args.grid}^3, n={P.A.n}")
        full, roots = cpu_full_solve(P, As, args.grid)
        log(f"cpu full solve: {full['value']:.1f}s, {full['iters']} steps, "
            f"{full['cycles']} cycles, relres {full['relres']:.2e}")
        est, parts, wall, busy = cpu_estimate(P, As, roots, full["iters"], full["cycles"])
        rec = {"full_solve": full, "estimate_s": est, "estimate_parts": parts,
               "estimate_sample_s": wall, "command": "python bench.py --cpu-full-solve OUT_JSON"}
        with open(args.cpu_full_solve, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec), flush=True)
        return
    dev = torch.device("cuda:0")
    if args.sweep:
        print(json.dumps(sweep(B, W, torch, dev, args.steps)), flush=True)
        return
    t0 = time.perf_counter()
    if args.config != 5:
        args.grid = 0   # the configuration's own size; no stored 256^3 references apply
    P = W.config(5, N=args.grid) if args.config == 5 else W.config(args.config)
    log(f"generated {P.name} grid {args.grid}^3: n={P.A.n} nnz={P.A.nnz} "
        f"in {time.perf_counter() - t0:.1f}s")
    A = B.CSRMatrix.from_host(P.A, device=dev)
    b = torch.from_numpy(P.b).to(dev)
    v0 = torch.from_numpy(P.v0).to(dev)
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    log("uploaded")

    def solve(**kw):
        x.zero_()
        return B.pp_gmres_solve(A, b, x, m=P.m, d=P.d, tol=P.tol, v0=v0, timing=True, **kw)[1]

    for i in range(args.warmup):
        st = solve()
        log(f"warmup {i}: {st.t_total:.3f}s iters {st.iters} relres {st.relres_true:.2e}")
    torch.cuda.synchronize()
    times, stats = [], []
    tstart = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        st = solve()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        stats.append(st)
        log(f"step {i}: {times[-1]:.3f}s iters {st.iters} cycles {st.cycles} "
            f"relres {st.relres_true:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - tstart
    t_solve = elapsed / args.steps
    st = stats[-1]
    converged = all(s.relres_true < P.tol for s in stats)

    # independent host check of the last solution
    x_default = x.clone()
    xs = x.cpu().numpy()
    As = P.A.to_scipy()
    relres_host = float(np.linalg.norm(P.b - As @ xs) / np.linalg.norm(P.b))
    ref = oracle_reference(args.grid)

    bc = sum(s.bytes_chain for s in stats)
    tc = sum(s.t_chain for s in stats)
    nl = sum(s.launches_chain for s in stats)
    bs = sum(s.bytes_spmv for s in stats)
    tsp = sum(s.t_spmv for s in stats)
    bo = sum(s.bytes_orth for s in stats)
    to = sum(s.t_orth for s in stats)
    chain_gbps = bc / tc / 1e9 if tc > 0 else None
    layout_name = {"sell": "sliced (diagonal slices)", "csr": "CSR"}.get(st.layout_used,
                                                                       st.layout_used)
    # a middle real-root step on the sliced copy: stored values, one 64-byte descriptor per
    # 64-row slice, the gathered input and the output (explicit-column slices add 4 B a slot)
    per_row_layout = ((8.0 * st.nnz_stored + 64.0 * ((P.A.n + 63) // 64) + 16.0 * P.A.n) / P.A.n
                      if st.layout_used == "sell" else None)
    cached = bool(st.chain_slab_rows or st.chain_cached)
    roofline = {
        "kernel": f"k_chain (fused {layout_name} product + Leja root update), FP64, "
                  + (f"slab-skewed over {st.chain_slab_rows:,}-row slabs, cached loads"
                     if st.chain_slab_rows else
                     "full-range, " + ("cached" if st.chain_cached else "non-temporal") + " loads"),
        "bound": "hbm",
        "achieved": round(chain_gbps, 1) if chain_gbps else None,
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(chain_gbps / HBM_PEAK_GBPS, 4) if chain_gbps else None,
        "traffic": pmc_traffic(args.grid, bc / nl if nl else None),
        "rate_basis": (
            "achieved = the layout's algorithmic bytes per launch (its values, slice descriptors "
            "and vectors) over the launches' event-timed duration.  "
            + ("Under this schedule a slab's later launches re-read it from the 256 MiB Infinity "
               "Cache, so achieved is a cache-assisted rate and frac is NOT a fraction of HBM "
               "bandwidth: hbm_only gives that (the same solve with every launch streaming from "
               "HBM), frac_of_cache_resident_copy compares achieved with a copy whose buffers "
               "sit in the cache" if cached else
               "Every launch streams from HBM: frac is a fraction of the HBM peak.")),
        "frac_of_cache_resident_copy": (round(chain_gbps / CACHE_COPY_GBPS, 4)
                                        if chain_gbps and cached else None),
        "cache_resident_copy_GBps": CACHE_COPY_GBPS,
        "hbm_copy_GBps": HBM_COPY_GBPS,
        "hbm_only": None,
        "dram_bytes": None,
        "dram_bytes_note": ("not measurable on gfx950: rocprofv3 lists no counter behind the "
                            "Infinity Cache (TCC_EA0_RDREQ_DRAM / WRREQ_DRAM count the L2's requests "
                            "to DRAM addresses, Infinity Cache hits included); traffic is those "
                            "L2-miss bytes"),
        "bytes_per_launch": bc / nl if nl else None,
        "bytes_per_row": {"sliced_copy_real_root_step": per_row_layout,
                          "csr_formula_12nnz_36n": (12.0 * P.A.nnz + 36.0 * P.A.n) / P.A.n},
        "avg_launch_us": tc / nl * 1e6 if nl else None,
        "launches": nl,
        "schedule": {"slab_rows": st.chain_slab_rows, "cached": st.chain_cached},
    }
    phases = {
        "chain_GBps": chain_gbps,
        "spmv_GBps": bs / tsp / 1e9 if tsp > 0 else None,
        "orth_GBps": bo / to / 1e9 if to > 0 else None,
        "t_chain_s": tc / args.steps, "t_spmv_s": tsp / args.steps, "t_orth_s": to / args.steps,
        "t_host_s": sum(s.t_host for s in stats) / args.steps,
        "t_poly_s": sum(s.t_poly for s in stats) / args.steps,
    }
    legs = {"pp_fp64": {"time_s": t_solve, "iters": st.iters, "cycles": st.cycles,
                        "spmvs": st.spmvs, "dots": st.dots, "relres": st.relres_true,
                        "nroots": st.nroots, "err_vs_oracle": error_vs_oracle(ref, xs)}}
    wanted = [s for s in args.legs.split(",") if s and s != "none"]
    if "ir" in wanted:
        solve(precision="f32_ir")
        torch.cuda.synchronize()
        ts = time.perf_counter()
        s2 = solve(precision="f32_ir")
        torch.cuda.synchronize()
        tir = time.perf_counter() - ts
        xir = x.cpu().numpy()
        legs["pp_fp32_ir"] = {"time_s": tir, "outer": s2.outer, "inner_iters": s2.iters,
                              "relres": s2.relres_true,
                              "rel_diff_vs_fp64": float(np.linalg.norm(xir - xs) /
                                                        np.linalg.norm(xs)),
                              "err_vs_oracle": error_vs_oracle(ref, xir),
                              "chain_GBps": s2.bytes_chain / s2.t_chain / 1e9
                              if s2.t_chain > 0 else None}
        log(f"fp32-ir: {tir:.3f}s outer {s2.outer} inner {s2.iters} relres {s2.relres_true:.2e}")
    if "plain" in wanted:
        import warnings
        ts = time.perf_counter()
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            x.zero_()
            _, s3 = B.pp_gmres_solve(A, b, x, m=P.m, d=0, tol=P.tol,
                                     max_iters=args.plain_max_iters, timing=True)
        torch.cuda.synchronize()
        tpl = time.perf_counter() - ts
        legs["gmres_fp64"] = {"time_s": tpl, "iters": s3.iters, "cycles": s3.cycles,
                              "dots": s3.dots, "relres": s3.relres_true,
                              "converged": bool(s3.relres_true < P.tol),
                              "max_iters": args.plain_max_iters,
                              "spmv_GBps": s3.bytes_spmv / s3.t_spmv / 1e9
                              if s3.t_spmv > 0 else None,
                              "orth_GBps": s3.bytes_orth / s3.t_orth / 1e9
                              if s3.t_orth > 0 else None}
        legs["speedup_pp_vs_gmres"] = tpl / t_solve
        log(f"plain gmres: {tpl:.3f}s iters {s3.iters} relres {s3.relres_true:.2e}")

    if "csr" in wanted:
        A_csr = A.with_layout("csr")
        B.pp_gmres_solve(A_csr, b, x.zero_(), m=P.m, d=P.d, tol=P.tol, v0=v0)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        _, s5 = B.pp_gmres_solve(A_csr, b, x.zero_(), m=P.m, d=P.d, tol=P.tol, v0=v0,
                                 timing=True)
        torch.cuda.synchronize()
        tcsr = time.perf_counter() - ts
        legs["pp_fp64_csr_layout"] = {"time_s": tcsr, "iters": s5.iters,
                                      "relres": s5.relres_true,
                                      "chain_GBps": s5.bytes_chain / s5.t_chain / 1e9
                                      if s5.t_chain > 0 else None}
        log(f"csr layout: {tcsr:.3f}s iters {s5.iters} relres {s5.relres_true:.2e}")

    if "jacobi" in wanted:
        # composition with a left Jacobi preconditioner (the polynomial is built for D^-1 A);
        # the stencil's diagonal is constant, so this measures the composition's overhead
        solve(left_jacobi=True)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        s6 = solve(left_jacobi=True)
        torch.cuda.synchronize()
        tj = time.perf_counter() - ts
        legs["pp_fp64_left_jacobi"] = {"time_s": tj, "iters": s6.iters,
                                       "relres_preconditioned": s6.relres_true,
                                       "relres_original": s6.relres_original}
        log(f"left jacobi: {tj:.3f}s iters {s6.iters} relres {s6.relres_original:.2e}")

    if "fullrange" in wanted:
        # the chain without Section VII's reuse: every launch over all rows, with
        # non-temporal loads and stores; identical results
        kwb = dict(chain_group=1)
        solve(**kwb)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        s7 = solve(**kwb)
        torch.cuda.synchronize()
        tb = time.perf_counter() - ts
        legs["pp_fp64_chain_fullrange"] = {
            "time_s": tb, "iters": s7.iters, "relres": s7.relres_true, **kwb,
            "chain_GBps": s7.bytes_chain / s7.t_chain / 1e9 if s7.t_chain > 0 else None,
            "same_x_as_default": bool(torch.equal(x, x_default))}
        if s7.t_chain > 0 and s7.launches_chain:
            hb = s7.bytes_chain / s7.t_chain / 1e9
            roofline["hbm_only"] = {
                "schedule": "full-range launches, non-temporal loads and stores (chain_group 1)",
                "achieved": round(hb, 1), "frac": round(hb / HBM_PEAK_GBPS, 4),
                "frac_of_hbm_copy": round(hb / HBM_COPY_GBPS, 4), "unit": "GB/s",
                "avg_launch_us": s7.t_chain / s7.launches_chain * 1e6}
        log(f"full-range non-temporal chain: {tb:.3f}s iters {s7.iters}")

    if "ilu" in wanted:
        legs["ilu0_left_recirc_257"] = ilu_leg(B, W, torch, dev)
        li = legs["ilu0_left_recirc_257"]
        log(f"ILU(0) + d={li['d']}: {li['time_s']:.3f}s iters {li['iters']}; ILU(0) alone "
            f"{li['ilu_only']['iters']} iters relres {li['ilu_only']['relres']:.2e}; "
            f"M^-1 r {li['apply_ms']:.3f} ms ({li['us_per_level']:.2f} us per level)")

    if "adjoint" in wanted:
        legs["adjoint_512"] = adjoint_leg(B, W, torch, dev)
        log(f"adjoint 512^2: {legs['adjoint_512']['time_s']:.3f}s")

    if args.copy_check:
        # torch's own device copy: context only (it is not a ceiling; a flat HIP copy
        # kernel reaches more), and the reference kernel for the counter scaling
        phases["torch_copy_GBps"] = torch_copy_rate(torch)
        log(f"torch device copy {phases['torch_copy_GBps']:.0f} GB/s")

    if "power" in wanted:
        # the paper's own construction: power basis + normal equations, degree chosen by
        # Section IV's heuristic (highest degree whose Gram matrix factors), then the solve
        import warnings
        def power_solve():
            ts = time.perf_counter()
            p, info = B.pp_build_poly_power(A, v0, 30, auto_degree=True)
            x.zero_()
            with warnings.catch_warnings():
                warnings.simplefilter("ignore")
                _, s4 = B.pp_gmres_solve(A, b, x, m=P.m, d=0, tol=P.tol, poly=p,
                                         max_iters=args.plain_max_iters)
            torch.cuda.synchronize()
            return time.perf_counter() - ts, p, info, s4
        power_solve()
        tpw, p, info, s4 = power_solve()
        legs["pp_power_auto"] = {"time_s": tpw, "degree": len(B.pp_poly_coeffs(p)) - 1,
                                 "potrf_info": info, "iters": s4.iters, "cycles": s4.cycles,
                                 "relres": s4.relres_true,
                                 "converged": bool(s4.relres_true < P.tol)}
        log(f"power-basis auto degree {legs['pp_power_auto']['degree']}: {tpw:.3f}s "
            f"iters {s4.iters} relres {s4.relres_true:.2e}")

    cpu = None
    if args.cpu_baseline:
        cpu = cpu_baseline(P, As, st, args.grid)

    out = {
        "metric": METRIC,
        "value": t_solve,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_solve * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"cd3d_{args.grid}_pe100" if args.config == 5 and args.grid != 256
                                else P.name),
                   "n": P.A.n, "nnz": P.A.nnz, "m": P.m, "d": P.d, "tol": P.tol,
                   "solver": "PP-GMRES(m), Leja-ordered harmonic Ritz roots, CGS2",
                   "layout": st.layout_used, "nnz_stored": st.nnz_stored},
        "converged": converged,
        "check": {"relres_lib": st.relres_true, "relres_host_scipy": relres_host},
        "roofline": roofline,
        "phases": phases,
        "legs": legs,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def sweep(B, W, torch, dev, steps):
    """Time-to-tol (mean of `steps` solves after one warm-up, build included) on each
    workload configuration: PP-GMRES at the configuration's d (and every d it lists),
    plain GMRES, and FP32 inside FP64 refinement where the configuration asks for it."""
    import warnings
    out = {}
    for k in sorted(W.CONFIG_NAMES):
        P = W.config(k)
        A = B.CSRMatrix.from_host(P.A, device=dev)
        b = torch.from_numpy(P.b).to(dev)
        v0 = torch.from_numpy(P.v0).to(dev)
        x = torch.zeros_like(b)
        rec = {"n": P.A.n, "nnz": P.A.nnz, "m": P.m, "tol": P.tol}

        def timed(tol=P.tol, **kw):
            with warnings.catch_warnings():
                warnings.simplefilter("ignore")
                x.zero_()
                B.pp_gmres_solve(A, b, x, m=P.m, tol=tol, v0=v0, **kw)
                torch.cuda.synchronize()
                ts = time.perf_counter()
                for _ in range(steps):
                    x.zero_()
                    _, st = B.pp_gmres_solve(A, b, x, m=P.m, tol=tol, v0=v0, **kw)
                torch.cuda.synchronize()
            return {"time_s": (time.perf_counter() - ts) / steps, "iters": st.iters,
                    "relres": st.relres_true, "layout": st.layout_used}
        for d in P.extra.get("degrees", [P.d]):
            rec[f"pp_d{d}" if d else "gmres"] = timed(d=d)
        if P.tol < 1e-8:
            # the metric's time-to-1e-8 on a configuration with a tighter tolerance:
            # the same solve stopped at 1e-8
            rec[f"pp_d{P.d}_to_1e-8"] = timed(tol=1e-8, d=P.d)
            rec["gmres_to_1e-8"] = timed(tol=1e-8, d=0, max_iters=30000)
        if "gmres" not in rec:
            rec["gmres"] = timed(d=0, max_iters=30000)
        if "inner_tol" in P.extra:
            rec[f"pp_d{P.d}_f32_ir"] = timed(d=P.d, precision="f32_ir",
                                            inner_tol=P.extra["inner_tol"])
        out[P.name] = rec
        log(f"{P.name}: " + ", ".join(f"{key} {v['time_s']:.4f}s/{v['iters']}it"
                                      for key, v in rec.items() if isinstance(v, dict)))
        del A, b, v0, x
        torch.cuda.empty_cache()
    out[W.EX1_WORKLOAD["name"]] = example1(B, W, torch, dev, steps)
    out.update(permuted_legs(B, W, torch, dev))
    return {"sweep": out, "steps": steps, "data": "synthetic"}


def permuted_legs(B, W, torch, dev, grid=256):
    """The headline solve on matrices without diagonal structure: the 256^3 problem
    under a seeded symmetric permutation P A P^T (b and v0 permuted alike), uniform
    over all rows (the worst case: every gather a random cache line) and within
    blocks of 4096 rows (an unstructured matrix whose ordering keeps locality, as a
    bandwidth-reducing ordering of a finite-element mesh would).  One timed solve
    after a warm-up each, with the library's automatic layout and schedule, and the
    chain kernel's per-product time and algorithmic rate beside the stencil's."""
    import warnings
    P = W.config(5, N=grid)
    out = {}
    for name, block in (("cd3d_256_pe100_perm", None), ("cd3d_256_pe100_perm4096", 4096)):
        if grid != 256:
            name = name.replace("256", str(grid))
        t0 = time.perf_counter()
        perm = W.permutation(P.A.n, 17, block)
        Ap = W.permuted(P.A, perm)
        log(f"{name}: permuted in {time.perf_counter() - t0:.1f}s")
        A = B.CSRMatrix.from_host(Ap, device=dev)
        del Ap
        b = torch.from_numpy(P.b[perm]).to(dev)
        v0 = torch.from_numpy(P.v0[perm]).to(dev)
        x = torch.zeros_like(b)

        def run():
            x.zero_()
            with warnings.catch_warnings():
                warnings.simplefilter("ignore")
                return B.pp_gmres_solve(A, b, x, m=P.m, d=P.d, tol=P.tol, v0=v0, timing=True)[1]
        run()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        st = run()
        torch.cuda.synchronize()
        t = time.perf_counter() - ts
        out[name] = {"time_s": t, "iters": st.iters, "relres": st.relres_true,
                     "layout": st.layout_used, "nnz_stored": st.nnz_stored,
                     "chain_slab_rows": st.chain_slab_rows, "chain_cached": st.chain_cached,
                     "chain_us_per_launch": st.t_chain / st.launches_chain * 1e6
                     if st.launches_chain else None,
                     "chain_GBps": st.bytes_chain / st.t_chain / 1e9 if st.t_chain > 0 else None,
                     "t_chain_s": st.t_chain, "t_orth_s": st.t_orth, "t_poly_s": st.t_poly}
        log(f"{name}: {t:.3f}s, {st.iters} steps, layout {st.layout_used}, chain "
            f"{out[name]['chain_us_per_launch']:.0f} us per launch, "
            f"{out[name]['chain_GBps']:.0f} GB/s")
        del A, b, v0, x
        torch.cuda.empty_cache()
    return out


def example1(B, W, torch, dev, steps):
    """Section VI's first example: recirculating flow, eps = 1/2, 1025^2, GMRES(50) to
    1e-8 without a preconditioner and with the paper's degrees 4 and 9 (d = 5, 10),
    and with the power basis at Section IV's automatic degree.  Besides time-to-tol,
    one extra solve with phase timing gives the share of GPU time in orthogonalisation
    (CGS2 dots and updates) against the application of A p(A), the split the paper
    plots."""
    import warnings
    wl = W.EX1_WORKLOAD
    Ah, bh = W.recirculating_flow(wl["N"], wl["eps"])
    A = B.CSRMatrix.from_host(Ah, device=dev)
    b = torch.from_numpy(bh).to(dev)
    v0 = torch.from_numpy(W.uniform(Ah.n, wl["v0_seed"])).to(dev)
    x = torch.zeros_like(b)
    rec = {"n": Ah.n, "nnz": Ah.nnz, "m": wl["m"], "tol": wl["tol"]}

    def run(cap=60000, **kw):
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            x.zero_()
            B.pp_gmres_solve(A, b, x, m=wl["m"], tol=wl["tol"], v0=v0, max_iters=cap, **kw)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            for _ in range(steps):
                x.zero_()
                _, st = B.pp_gmres_solve(A, b, x, m=wl["m"], tol=wl["tol"], v0=v0,
                                         max_iters=cap, **kw)
            torch.cuda.synchronize()
            t = (time.perf_counter() - ts) / steps
            x.zero_()
            _, sp = B.pp_gmres_solve(A, b, x, m=wl["m"], tol=wl["tol"], v0=v0, max_iters=cap,
                                     timing=True, **kw)
        busy = sp.t_chain + sp.t_spmv + sp.t_orth
        return {"time_s": t, "iters": st.iters, "relres": st.relres_true,
                "converged": bool(st.relres_true < wl["tol"]), "max_iters": cap,
                "orth_share": sp.t_orth / busy if busy > 0 else None,
                "apply_share": (sp.t_chain + sp.t_spmv) / busy if busy > 0 else None}
    for d in wl["degrees"]:
        rec[f"pp_d{d}" if d else "gmres"] = run(d=d)
    # the paper's power basis: at Section IV's automatic degree (the highest whose Gram
    # matrix factors; where that lands depends on the Gram's last digits), capped at
    # 5000 steps since a polynomial at the onset may not precondition at all; and at
    # degree 9, the degree the paper reports its heuristic chose for this example
    p, info = B.pp_build_poly_power(A, v0, 30, auto_degree=True)
    deg = len(B.pp_poly_coeffs(p)) - 1
    rec["power_auto"] = dict(run(d=0, poly=p, cap=5000), degree=deg, potrf_info=info)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        p9, info9 = B.pp_build_poly_power(A, v0, 9)
    rec["power_deg9"] = dict(run(d=0, poly=p9, cap=5000), degree=9, potrf_info=info9)
    log(f"{wl['name']}: " + ", ".join(
        f"{key} {v['time_s']:.3f}s/{v['iters']}it orth {v['orth_share']:.2f}"
        for key, v in rec.items() if isinstance(v, dict)))
    return rec


def ilu_leg(B, W, torch, dev, ilu_only_cap=1000):
    """Section VI's second example: ILU(0) on the left, the polynomial of M^-1 A on
    the right (recirculating wind, eps = 1/200, 257^2, GMRES(50), d = 13, tol
    1e-8).  Times the factorisation, one M^-1 r (two level-scheduled sweeps; wall
    time of a synchronised call, mean of 100 after 5 warm-ups) and the composed
    solve (one warm-up, one timed), and runs ILU(0) alone up to `ilu_only_cap`
    iterations (it stalls on this problem, as the paper reports)."""
    import warnings

    wl = W.ILU_WORKLOAD
    Ah, bh = W.recirculating_flow(wl["N"], wl["eps"])
    A = B.CSRMatrix.from_host(Ah, device=dev)
    b = torch.from_numpy(bh).to(dev)
    v0 = torch.from_numpy(W.uniform(Ah.n, wl["v0_seed"])).to(dev)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    M = B.pp_ilu0_factor(A)
    t_factor = time.perf_counter() - ts
    nf, nb, launches = M.levels()
    r = torch.from_numpy(W.normal(Ah.n, 1)).to(dev)
    z = torch.empty_like(r)
    for _ in range(5):
        B.pp_ilu0_apply(M, r, z)
    reps = 100
    ts = time.perf_counter()
    for _ in range(reps):
        B.pp_ilu0_apply(M, r, z)
    t_apply = (time.perf_counter() - ts) / reps

    def solve(**kw):
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            _, st = B.pp_gmres_solve(A, b, x, m=wl["m"], tol=wl["tol"], v0=v0, left_ilu=M, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, x, st
    solve(d=wl["d"])
    t_pp, x, st = solve(d=wl["d"])
    t_alone, _, s0 = solve(d=0, max_iters=ilu_only_cap)
    # algorithmic bytes of one M^-1 r: per sweep the level order and row pointers
    # (8 n), the waited-for entries (12 each, nnz - n in all), right-hand side,
    # solution written and gathered (24 n); the backward sweep's pivots (8 n)
    sweep_bytes = 72.0 * Ah.n + 12.0 * (Ah.nnz - Ah.n)
    ref = oracle_reference_named("recirc2d_257_eps200_ilu0_d13")
    return {"workload": wl["name"], "n": Ah.n, "nnz": Ah.nnz, "m": wl["m"], "d": wl["d"],
            "tol": wl["tol"], "time_s": t_pp, "iters": st.iters, "cycles": st.cycles,
            "relres_preconditioned": st.relres_true, "relres_original": st.relres_original,
            "err_vs_oracle": error_vs_oracle(ref, x.cpu().numpy()) if ref else None,
            "oracle_iters": ref["iters"] if ref else None,
            "factor_s": t_factor, "levels_forward": nf, "levels_backward": nb,
            "launches_per_apply": launches, "apply_ms": t_apply * 1e3,
            "us_per_level": t_apply * 1e6 / (nf + nb),
            "apply_alg_GBps": sweep_bytes / t_apply / 1e9,
            "ilu_only": {"time_s": t_alone, "iters": s0.iters, "relres": s0.relres_true,
                         "converged": bool(s0.relres_true < wl["tol"]), "cap": ilu_only_cap}}


def adjoint_leg(B, W, torch, dev):
    """Forward solve, adjoint solve on A^T and the gradient on the CSR pattern
    (2D convection-diffusion 512^2, Pe 20, L = 0.5 ||x - x_t||^2, forward and
    adjoint d = 15, tol 1e-12), through the torch autograd wrapper; one warm-up,
    then one timed forward + backward."""
    import warnings

    from paper_1907_00072_amd.autograd import SolveConfig, pp_solve
    P = W.config(4)
    pattern = B.CSRMatrix.from_host(P.A, device=dev)
    xt = torch.from_numpy(P.extra["x_target"]).to(dev)

    def once():
        vals = torch.from_numpy(P.A.vals).to(dev).requires_grad_(True)
        bb = torch.from_numpy(P.b).to(dev).requires_grad_(True)
        cfg = SolveConfig(m=P.m, d=P.d, tol=P.tol, v0=torch.from_numpy(P.v0).to(dev),
                          adj_v0=torch.from_numpy(P.extra["v0_adjoint"]).to(dev))
        torch.cuda.synchronize()
        ts = time.perf_counter()
        x = pp_solve(pattern, vals, bb, cfg)
        loss = 0.5 * ((x - xt) ** 2).sum()
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")  # the adjoint may end on the stagnation test
            loss.backward()
        torch.cuda.synchronize()
        return time.perf_counter() - ts, cfg
    once()
    t, cfg = once()
    fwd, adj = cfg.stats[0][1], cfg.stats[1][1]
    return {"time_s": t, "n": P.A.n, "nnz": P.A.nnz, "forward_iters": fwd.iters,
            "adjoint_iters": adj.iters, "forward_relres": fwd.relres_true,
            "adjoint_relres": adj.relres_true}


def oracle_reference(grid):
    """The oracle's own solve of the default workload (sampled entries), stored by
    tests/golden/make_fullsize_refs.py; None for other grids."""
    if grid != 256:
        return None
    return oracle_reference_named("cd3d_256_pe100_d40")


def oracle_reference_named(name):
    """A stored oracle solve (tests/golden/fullsize_refs.json), or None."""
    try:
        refs = json.load(open(os.path.join(ROOT, "tests", "golden", "fullsize_refs.json")))
    except OSError:
        return None
    return refs.get(name)


def error_vs_oracle(ref, x):
    """Max |x - x_oracle| over the oracle's 64 sampled entries, relative to max |x_oracle|
    (the oracle ran the same PP-GMRES(30), d = 40 to 1e-8 in FP64 on the host)."""
    import numpy as np
    if ref is None:
        return None
    idx = np.asarray(ref["sample_idx"])
    return float(np.max(np.abs(x[idx] - np.asarray(ref["x_sample"]))) / ref["x_absmax"])


def kernels_code_hash():
    """sha256 prefix of kernels.hip with comments and blank lines removed, so the
    counters stay valid across comment-only edits."""
    import hashlib
    import re
    src = open(os.path.join(ROOT, "paper_1907_00072_amd", "csrc", "kernels.hip")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in src.splitlines()]
    code = "\n".join(ln for ln in lines if ln.strip())
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def pmc_traffic(grid, bytes_per_launch):
    """L2-miss bytes per chain launch from the committed rocprofv3 counter runs:
    the dominant kernel's FETCH_SIZE + WRITE_SIZE per row over its algorithmic
    bytes per row (the launches are slabs of different sizes), times this run's
    algorithmic bytes per launch.

    Only reported while kernels.hip's code is what those counters were taken
    from (kernels_code_hash is recorded with them); otherwise None.
    """
    if grid != 256 or not bytes_per_launch:
        return None
    path = os.path.join(ROOT, "profiles", "k_chain_cd3d_256_pe100_traffic.json")
    try:
        rec = json.load(open(path))
        sha = kernels_code_hash()
    except OSError:
        return None
    if rec.get("kernels_code_sha256_16") != sha:
        return None
    return rec["traffic_ratio"] * bytes_per_launch


def torch_copy_rate(torch, nbytes=2 << 30, reps=5):
    """Bandwidth of torch's device copy of nbytes (read + write), event-timed."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 2.0 * nbytes / sec / 1e9


def host_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def oracle_roots(P, grid):
    """Roots of the oracle's own polynomial for the workload: the stored oracle run's
    at 256^3 (written by tests/golden/make_fullsize_refs.py), else built here by the
    oracle (small grids)."""
    import numpy as np

    from oracle import poly as op
    ref = oracle_reference(grid)
    if ref is not None and len(ref["roots_re"]) == P.d:
        return np.asarray(ref["roots_re"]) + 1j * np.asarray(ref["roots_im"]), "stored oracle run"
    roots, _ = op.build_poly(P.A.to_scipy(), P.v0, P.d)
    return roots, "oracle build_poly"


def cpu_estimate(P, As, roots, st_iters, st_cycles):
    """The oracle's time for the whole solve, from timings of its own functions on
    the full matrix: one p(A)v (complex arithmetic, one root at a time), and the
    Arnoldi process (one product + CGS2 per step) to k1 and k2 steps.  The Arnoldi
    prefixes give the per-step cost t(j) = c0 + c1 j at j basis columns (least
    squares on T(k) = k c0 + c1 k(k+1)/2); a GMRES step at column j costs one p(A)v
    plus t(j), a cycle end one p(A)v plus one product, the build T(d).  Returns
    (estimate_s, parts, sample_wall_s, threads_busy)."""
    import numpy as np

    from oracle import poly as op
    r0 = P.b / np.linalg.norm(P.b)
    c0w, w0 = time.process_time(), time.perf_counter()
    ts = time.perf_counter()
    op.apply_poly(As, roots, r0)
    t_apply = time.perf_counter() - ts
    ks, Ts = (4, 8), []
    for k in ks:
        ts = time.perf_counter()
        op.arnoldi(As, P.v0, k)
        Ts.append(time.perf_counter() - ts)
    M = np.array([[k, k * (k + 1) / 2.0] for k in ks])
    c0, c1 = np.linalg.solve(M, np.asarray(Ts))
    c1 = max(c1, 0.0)
    c0 = max(c0, 0.0)
    ts = time.perf_counter()
    As @ r0
    t_mv = time.perf_counter() - ts
    wall = time.perf_counter() - w0
    busy = (time.process_time() - c0w) / wall

    def T(k):
        return k * c0 + c1 * k * (k + 1) / 2.0
    steps = sum(t_apply + c0 + c1 * (j % P.m + 1) for j in range(st_iters))
    est = T(P.d) + steps + st_cycles * (t_apply + t_mv) + t_mv
    parts = {"p_of_A_v_s": t_apply, "arnoldi_prefix_s": dict(zip(map(str, ks), Ts)),
             "step_cost_s": [c0, c1], "product_s": t_mv, "build_s_est": T(P.d)}
    return est, parts, wall, busy


class _CountedOperator:
    """The matrix with a count of its products, printing a progress line every 200
    (a whole oracle solve at 256^3 runs for minutes)."""

    def __init__(self, A):
        self.A, self.k, self.shape = A, 0, A.shape

    def __matmul__(self, x):
        self.k += 1
        if self.k % 200 == 0:
            log(f"cpu full solve: {self.k} products")
        return self.A @ x


def cpu_full_solve(P, As, grid):
    """The oracle's complete solve of the workload, timed: its polynomial build
    (d Arnoldi steps, harmonic Ritz values, Leja order) and PP-GMRES(m) to tol."""
    from oracle import gmres as og
    from oracle import poly as op
    A = _CountedOperator(As)
    c0, w0 = time.process_time(), time.perf_counter()
    roots, _ = op.build_poly(A, P.v0, P.d)
    t_build = time.perf_counter() - w0
    log(f"cpu full solve: build {t_build:.1f}s")
    _, so = og.pp_gmres(A, P.b, P.m, P.tol, roots=roots, max_iters=20000)
    wall = time.perf_counter() - w0
    return {"value": wall, "unit": "s", "build_s": t_build, "iters": so.iters,
            "cycles": so.cycles, "relres": so.relres_true, "converged": so.converged,
            "threads_busy": (time.process_time() - c0) / wall, "products": A.k,
            "host": host_model(), "logical_cpus": os.cpu_count(),
            "workload": P.name if grid == 256 else f"cd3d_{grid}_pe100"}, roots


def cpu_baseline(P, As, st, grid):
    """Oracle time for the whole solve on this host: an estimate from timings of the
    oracle's own functions on the full matrix (cpu_estimate), with the oracle's own
    roots, scaled to the oracle's step and cycle counts (the GPU's, equal within 2%).
    The complete oracle solve measured once on a host of the GPU machine is quoted beside it
    (profiles/oracle_cpu_cd3d_256_pe100.json, written by `bench.py --cpu-full-solve`),
    with the estimator's value from that same run as its calibration."""
    roots, src = oracle_roots(P, grid)
    log("cpu baseline: timing the oracle's p(A)v and Arnoldi prefixes on the full matrix")
    est, parts, wall, busy = cpu_estimate(P, As, roots, st.iters, st.cycles)
    cal = None
    path = os.path.join(ROOT, "profiles", "oracle_cpu_cd3d_256_pe100.json")
    if grid == 256 and os.path.exists(path):
        rec = json.load(open(path))
        full = rec["full_solve"]
        cal = {"measured_full_solve_s": full["value"], "estimate_same_run_s": rec["estimate_s"],
               "measured_over_estimate": full["value"] / rec["estimate_s"],
               "host": full["host"], "threads_busy": full["threads_busy"],
               "source": "profiles/oracle_cpu_cd3d_256_pe100.json"}
    log(f"cpu baseline: estimated oracle solve {est:.0f}s (sample {wall:.1f}s, {busy:.1f} "
        f"threads busy)")
    return {"value": est, "unit": "s", "cores": max(1, round(busy)), "kind": "oracle",
            "sample": (f"the oracle's own functions on the full n={P.A.n} matrix: one p(A)v with "
                       f"{len(roots)} roots ({src}; complex arithmetic) {parts['p_of_A_v_s']:.1f}s, "
                       f"Arnoldi (product + CGS2) to 4 and 8 steps "
                       f"{parts['arnoldi_prefix_s']['4']:.1f}s / "
                       f"{parts['arnoldi_prefix_s']['8']:.1f}s; scaled to the build's {P.d} "
                       f"steps and the solve's {st.iters} steps and {st.cycles} cycle ends "
                       f"({wall:.0f}s of sampling, {busy:.1f} threads busy: SciPy's sparse "
                       f"products are single-threaded, NumPy's Gram-Schmidt products are not).  "
                       f"Host: {host_model()}, {os.cpu_count()} logical CPUs visible."),
            "parts": parts, "calibration": cal}


if __name__ == "__main__":
    main()
