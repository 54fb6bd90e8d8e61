/*
 * pp.h -- C ABI of libpp: polynomial-preconditioned GMRES(m) on MI355X (gfx950).
 *
 * Method: Loe, Thornquist & Boman, "Polynomial Preconditioned GMRES to Reduce
 * Communication in Parallel Computing" (arXiv 1907.00072).  The preconditioner
 * is the GMRES minimum-residual polynomial p(A) of Section II, used on the right
 * of GMRES(m) with two-pass classical Gram-Schmidt (Section III): solve
 * A p(A) y = b, then x = p(A) y.
 *
 * Degree convention.  d = number of roots of the residual polynomial
 * pi(alpha) = 1 - alpha p(alpha); p has degree d-1.  The paper's degree deg is d-1
 * (its power basis has deg+1 columns and costs deg+1 products, Sections II-III).
 * Applying p costs d-1 sparse products; one preconditioned step A p(A) v costs d.
 *
 * Root form.  The paper forms p from a power basis and the normal equations
 * (Section II, eqs. (1)-(2)) and notes that this is unstable at higher degree
 * (Section IV) and that more stable constructions exist (end of Section II,
 * Section VIII).  This library uses the stable product form: the zeros of pi are
 * the harmonic Ritz values theta_i of A on K_d(A, v0), the eigenvalues of
 * H_d + h_{d+1,d}^2 H_d^{-T} e_d e_d^T from d Arnoldi steps on v0; they are
 * applied in modified Leja order, a conjugate pair as one real quadratic factor.
 * Both forms are the same polynomial in exact arithmetic.
 *
 * Conventions for every entry point
 *  - Device pointers are HIP device (or managed) memory on the current device;
 *    the caller owns them and the library keeps none of them past the call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is ordered on that stream.  Calls that return results to the
 *    host (build, solve) synchronise the stream before returning; pp_apply,
 *    pp_csr_transpose and pp_csr_grad also synchronise, so every call is
 *    complete on return and its temporaries can be reused.
 *  - Internal temporaries (Krylov basis, chain vectors, reduction partials) come
 *    from a per-device arena owned by the library, grown on demand and kept
 *    until pp_release_workspace() or process exit.  Calls are serialised by a
 *    library-wide lock.
 *  - Return value: 0 = success; > 0 = warning, outputs are valid (see codes);
 *    < 0 = error, outputs are unspecified (inputs are never modified, except x
 *    in pp_gmres_solve, which then holds the last finite iterate).
 *  - Reductions are two-stage in a fixed order without floating-point atomics,
 *    so repeated calls with the same inputs give bitwise-identical results.  With
 *    PP_LAYOUT_AUTO, calls that run different numbers of products (a separate
 *    pp_build_poly and a solve) may pick different layouts and so round
 *    differently; fix pp_csr.layout when their results must agree bit for bit.
 *  - Checkpoint / resume: a solve interrupted at a restart-cycle boundary
 *    (max_iters a multiple of m) resumes exactly from the saved x (as x0) and the
 *    polynomial rebuilt from pp_poly_roots by pp_poly_from_roots.
 *  - Tracing: the environment variable PP_LOG=1 prints one line per restart cycle
 *    (or refinement step), per ILU(0) factorisation and per solve's chain schedule
 *    to stderr, PP_LOG=2 also every Arnoldi step's implicit residual; unset or 0
 *    prints nothing.
 */
#ifndef PP_H
#define PP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define PP_OK 0
#define PP_ERR_ARG (-1)       /* null pointer, n <= 0, d < 0, m < 1, tol <= 0, dtype or size mismatch */
#define PP_ERR_HIP (-2)       /* a HIP runtime call failed */
#define PP_ERR_NOMEM (-3)     /* device or pinned-host allocation failed */
#define PP_ERR_EIG (-4)       /* Hessenberg QR iteration did not converge */
#define PP_ERR_SINGULAR (-5)  /* H_d singular, or a zero / non-finite root */
#define PP_WARN_DEGREE_REDUCED 1 /* Arnoldi on v0 broke down after s < d steps: s roots */
#define PP_WARN_NOT_CONVERGED 2  /* iteration cap reached, or the true residual stagnated
                                    within 100 x tol while the implicit estimate reached
                                    tol (the attainable accuracy); x is the last iterate */
#define PP_WARN_NONFINITE 3      /* NaN/Inf met; x is the last finite iterate */
#define PP_WARN_CHOLESKY 4       /* power basis: Gram matrix not numerically positive definite */

/* ---- value types ----------------------------------------------------- */
#define PP_F64 0
#define PP_F32 1

/* ---- solve precision -------------------------------------------------- */
#define PP_PREC_F64 0    /* everything in FP64 */
#define PP_PREC_F32_IR 1 /* FP32 chain + CGS2 inside an FP64 refinement loop */

/* ---- how an Arnoldi step applies the preconditioned operator ------------ */
#define PP_OP_RESIDUAL_POLY 0 /* w = v - pi(A) v: d fused root updates (default) */
#define PP_OP_PRODUCT 1       /* w = A (p(A) v): d-1 fused updates, then one product */

/* ---- storage of A for the sparse products --------------------------- */
#define PP_LAYOUT_AUTO 0 /* the sliced copy unless it would stream more bytes (below), else CSR */
#define PP_LAYOUT_CSR 1  /* run the products on the caller's CSR arrays */
#define PP_LAYOUT_SELL 2 /* always the sliced copy (unless its offsets would overflow int32) */

/* Square sparse matrix in CSR form, all arrays in device memory.
 * row_ptr[n+1] int32, row_ptr[0] = 0, nondecreasing, row_ptr[n] = nnz < 2^31;
 * col_ind[nnz] int32 in [0, n) (any order inside a row; sorted is fastest);
 * vals[nnz] of type dtype.  Duplicate (row, col) entries are summed.
 *
 * layout: with PP_LAYOUT_AUTO (0, the zero-initialised default) or
 * PP_LAYOUT_SELL, each call first copies A, in library memory, into a sliced
 * form: slices of 64 consecutive rows, each stored column-major (slot-major).
 * A slice whose rows have strictly increasing columns and use at most 1.5 x
 * (longest row) distinct diagonals (col - row) is stored by diagonal: slot j
 * holds diagonal d_j for all 64 rows (0 where a row has no entry there) and
 * only the offsets d_j are kept, no column indices.  Any other slice keeps
 * explicit columns, padded to its longest row (column -1, value 0).  The
 * products then run on the copy: one wavefront owns a slice, and each load of
 * the vector reads one diagonal (or one entry) of 64 consecutive rows.  The
 * copy costs about two passes over A per call.  AUTO keeps CSR when one product
 * on the copy would stream more than 1.25 x the bytes of the CSR product
 * (irregular row lengths), or when the call runs too few products to repay
 * the copy (e.g. pp_apply with a handful of roots: each product is credited
 * with the bytes it saves, at least 5% of a CSR product, against the bytes the
 * conversion moves).  Both layouts give the same products up to the
 * rounding of the summation; an entry stored as an explicit 0 and an absent
 * one are treated alike. */
typedef struct pp_csr {
  int64_t n;
  int64_t nnz;
  const int32_t *row_ptr;
  const int32_t *col_ind;
  const void *vals;
  int32_t dtype;  /* PP_F64 or PP_F32 */
  int32_t layout; /* PP_LAYOUT_AUTO (0), PP_LAYOUT_CSR or PP_LAYOUT_SELL */
} pp_csr;

/* Opaque polynomial: n, the Leja-ordered roots (host, FP64) and the dtype it was
 * built in.  Library-owned; free with pp_poly_free.  It holds no device memory
 * and no pointer into A: pass the same A it was built from to pp_apply. */
typedef struct pp_poly pp_poly;

/* Opaque ILU(0) factorisation M = L U of a matrix (pp_ilu0_factor): the factors
 * and their level schedules in device memory on the device that was current when
 * it was made.  Library-owned; free with pp_ilu0_free.  It keeps no pointer into
 * the matrix it was made from. */
typedef struct pp_ilu pp_ilu;

/* Optional solver controls.  Zero-initialise and set what you need; zero
 * fields take the defaults shown. */
typedef struct pp_opts {
  int32_t max_iters;      /* cap on Arnoldi steps (inner steps for F32_IR); 0 -> 100000 */
  int32_t precision;      /* PP_PREC_F64 (0) or PP_PREC_F32_IR */
  double inner_tol;       /* F32_IR: inner cycle stops at this relative reduction; 0 ->
                             automatic: 1e-5, or 0.5 tol / relres when that is larger (a
                             refinement step needing less reduction stops earlier) */
  int32_t max_outer;      /* F32_IR: cap on refinement steps; 0 -> 100 */
  const double *v0;       /* device[n] start vector for the polynomial; NULL -> the
                             seeded U(-1, 1) vector pp_uniform_vector(n, v0_seed) drawn
                             on the device.  Section V shows why not b: the polynomial
                             built from b can swing far below zero on the spectrum
                             (GMRES(50) then stalls), one from a random vector does not. */
  const pp_poly *poly;    /* reuse this polynomial instead of building one (d ignored) */
  const float *vals_f32;  /* F32_IR: device[nnz] FP32 copy of A's values; NULL -> made internally */
  double *history;        /* host[history_cap]: implicit relative residual after each step */
  int32_t history_cap;
  int32_t timing;         /* nonzero: fill the per-phase times in pp_stats (adds events) */
  int32_t op_form;        /* PP_OP_RESIDUAL_POLY (0) or PP_OP_PRODUCT; the same operator
                             A p(A) in exact arithmetic (pi(alpha) = 1 - alpha p(alpha)) */
  int32_t left_jacobi;    /* nonzero: compose with a left Jacobi preconditioner (Section II:
                             the polynomial is built for the preconditioned operator).
                             GMRES runs on D^-1 A p(D^-1 A) y = D^-1 b, x = p(D^-1 A) y, and
                             stops on ||D^-1 (b - A x)|| / ||D^-1 b|| < tol; D = diag(A)
                             (zero or missing diagonal -> PP_ERR_SINGULAR).  The scaled
                             copy of A's values is made once per call. */
  const pp_ilu *left_ilu; /* non-NULL: compose with this ILU(0) factorisation M of A
                             (pp_ilu0_factor of the same matrix) on the left, Section VI's
                             second example: GMRES runs on M^-1 A p(M^-1 A) y = M^-1 b,
                             x = p(M^-1 A) y, the polynomial is built for M^-1 A, and the
                             solve stops on ||M^-1 (b - A x)|| / ||M^-1 b|| < tol.  FP64
                             only; not together with left_jacobi or F32_IR (PP_ERR_ARG). */
  int32_t chain_group;    /* Schedule of the solve's chains (each Arnoldi step's operator,
                             the cycle-end update, the power basis' Horner chain; pp_apply
                             always chooses automatically); every choice gives
                             bit-identical results.  Section VII's reuse of
                             the matrix across products: a launch's working set is its
                             matrix rows plus two vectors (73 B a row for a 7-point
                             stencil in FP64, 37 B in FP32), against a budget of 216 MiB
                             of MI355X's 256 MiB Infinity Cache.
                             0 (automatic): if the working set fits the budget, full-range
                               launches with cached loads and stores; else the slab-skewed
                               order below over all of a chain's launches with slabs that
                               fit the budget, when the matrix bandwidth is at most 1/8 of
                               a slab; else full-range non-temporal launches.
                             1: full-range launches, non-temporal loads and stores.
                             >= 2: the slab-skewed order, chain_group launches at a time
                               over row slabs of chain_slab_rows rows, each launch one
                               matrix bandwidth behind the previous: a slab's matrix and
                               vectors are read chain_group times in a row while cached.
                             Negative: PP_ERR_ARG.  Ignored with left_ilu (M^-1 couples all
                             rows).  pp_stats reports the choice. */
  int32_t chain_slab_rows; /* rows per slab (rounded down to whole launch tiles, at least
                              one); 0 -> the budget over the working set per row.
                              Negative: PP_ERR_ARG */
  uint64_t v0_seed;        /* seed of the start vector drawn when v0 is NULL (0 default) */
} pp_opts;

/* Solve statistics (all counts follow Section III: a dot is one block inner
 * product or norm, three per Arnoldi step with CGS2). */
typedef struct pp_stats {
  int32_t status;          /* same as the return value */
  int32_t iters;           /* Arnoldi steps of the (inner) GMRES */
  int32_t cycles;          /* GMRES(m) cycles (restarts + 1) */
  int32_t outer;           /* F32_IR refinement steps (0 in FP64 mode) */
  int32_t nroots;          /* roots used (<= d; 0 = no polynomial) */
  int32_t history_len;     /* entries written to opts->history */
  int64_t spmvs;           /* sparse products with A, including the build */
  int64_t dots;            /* block inner products and norms, including the build */
  double relres_true;      /* ||b - A x|| / ||b|| at return (FP64) */
  double relres_implicit;  /* last implicit (least-squares) estimate */
  double t_total;          /* seconds, wall clock of the call */
  double t_poly;           /* seconds building the polynomial (wall clock) */
  /* Phase times of the Arnoldi steps (the build's and the solve's), measured
   * with HIP events on the stream when timing != 0: */
  double t_chain;          /* seconds in the p(A) chain kernels */
  double t_spmv;           /* seconds in the operator product A z */
  double t_orth;           /* seconds in CGS2 kernels and reductions */
  double t_host;           /* step wall time not covered by the three above: launch
                              latency, the per-step copy and synchronisation, host
                              least squares */
  /* Algorithmic HBM bytes of the launches inside the timed phases above (the
   * Arnoldi steps' chains, operator products and CGS2 sweeps), from the
   * per-launch traffic model: a chain launch reads the matrix once (CSR: vals,
   * col_ind, row_ptr, 12 nnz + 4 n bytes in FP64; sliced copy: the stored values,
   * the columns of explicit-column slices, a 64-byte descriptor per 64-row slice
   * and any diagonal offsets past the descriptor's first 8, 8 nnz_stored + n
   * bytes for a stencil), the gathered vector once and the accumulator / partner
   * vectors once, and writes its outputs once.  Divided by t_chain / t_spmv /
   * t_orth they give achieved bandwidth. */
  double bytes_chain;
  double bytes_spmv;
  double bytes_orth;
  int64_t launches_chain;  /* chain launches inside t_chain */
  double relres_original;  /* ||b - A x|| / ||b|| of the unpreconditioned system (equals
                              relres_true unless left_jacobi or left_ilu is set) */
  int32_t layout_used;     /* PP_LAYOUT_CSR or PP_LAYOUT_SELL: what the products ran on */
  int64_t nnz_stored;      /* values one product streams: nnz (CSR) or the sliced copy's
                              stored values, padding included */
  int32_t chain_slab_rows; /* the chain schedule used (the inner solve's with F32_IR): rows
                              per slab of the slab-skewed order, 0 = full-range launches */
  int32_t chain_cached;    /* 1: the chain's launches load and store through the caches;
                              0: non-temporal (see pp_opts.chain_group) */
} pp_stats;

/* Build the polynomial for (A, v0) with d roots.
 * Passage: Section II (the minimum-residual polynomial for a start vector v0),
 * Section V (v0 random rather than b); root form as described above.
 * Runs d Arnoldi steps (CGS2) on v0 in A's dtype on the device, then on the host
 * in FP64 the harmonic Ritz eigenproblem (Francis double-shift QR) and the
 * modified Leja order.
 *   A   : matrix (PP_F64 or PP_F32)
 *   v0  : device[n] FP64 start vector (cast to A's dtype for the Arnoldi); not
 *         modified.  NULL -> the seeded vector pp_uniform_vector(n, 0).
 *   d   : 1 <= d <= min(n, 256)
 *   out : receives a new pp_poly on success or warning
 * Returns PP_OK, PP_WARN_DEGREE_REDUCED (fewer roots), PP_ERR_ARG, PP_ERR_SINGULAR
 * (H_d singular, zero v0, or a zero/non-finite root), PP_ERR_EIG, PP_ERR_HIP, PP_ERR_NOMEM. */
int pp_build_poly(const pp_csr *A, const double *v0, int d, void *stream, pp_poly **out);

/* y = p(A) v.  Passage: Section II (the polynomial object applies p(A) to a vector).
 * Product form in Leja order: for a real root theta, y += prod/theta and
 * prod -= A prod / theta; a pair a +- ib is one real quadratic step with
 * c1 = 2a/|theta|^2, c2 = 1/|theta|^2.  d-1 fused sparse-product + update kernels,
 * in the schedule pp_opts.chain_group = 0 would choose (bit-identical results).
 *   v, y : device[n] of A's dtype; may not alias.  y is overwritten.
 * Returns PP_OK, PP_ERR_ARG (poly built for another n), PP_ERR_HIP, PP_ERR_NOMEM. */
int pp_apply(const pp_csr *A, const pp_poly *p, const void *v, void *y, void *stream);

/* pp_apply without allocation, for callers that cannot allocate: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Computes
 * y = p(A) v as pp_apply does, and calls no hipMalloc, hipFree, hipHostMalloc or
 * other allocating routine (the caller still owns A, v and y).
 *   Scratch: the chain's three n-entry temporaries and the CSR check's flag live
 *   in a fixed device array of the library, 48 MiB + 4 KiB on each GPU it runs
 *   on, held from the library's load until the process ends.  Hence
 *   n <= 2^21 = 2,097,152 rows in FP64 (2^22 in FP32); a larger n is PP_ERR_ARG,
 *   and pp_last_error() states the limit.
 *   Layout: the products run on A's CSR arrays whatever A->layout asks (the
 *   sliced copy would need memory in proportion to nnz), in full-range launches
 *   (cached when a product's working set fits the last-level cache); the result
 *   equals pp_apply's on PP_LAYOUT_CSR bit for bit.
 *   Sharing: every call on a GPU uses that GPU's one array, which keeps the last
 *   call's contents (the flag is cleared by a fill kernel each call; the
 *   temporaries are written before they are read).  Calls that overlapped on one
 *   GPU would race on it: the library lock serialises the calls of a process and
 *   each call synchronises its stream before it returns, so they do not overlap.
 * Returns PP_OK, PP_ERR_ARG (as pp_apply, or n above the limit), PP_ERR_HIP. */
int pp_apply_noalloc(const pp_csr *A, const pp_poly *p, const void *v, void *y, void *stream);

/* Solve A x = b with GMRES(m) right-preconditioned by the d-root polynomial.
 * Stopping: the true relative residual below tol, the iteration cap, or, once it
 * is below 100 * tol, three consecutive restart cycles that each fail to reduce
 * it by 10% (FP64 rounding floor; PP_WARN_NOT_CONVERGED).
 * Passage: Section III (GMRES(m), two-pass classical Gram-Schmidt, relative
 * residual ||b - A x|| / ||b|| < tol, polynomial on the right), Section V
 * (start vector), Section II (the polynomial).  d = 0 runs plain GMRES(m).
 *   A   : PP_F64 matrix (F32_IR makes or takes an FP32 copy of the values)
 *   b   : device[n] FP64; x: device[n] FP64, in: x0, out: solution
 *   m   : restart length, 1 <= m <= 256; tol > 0
 *   opt : may be NULL (defaults); st: may be NULL
 * A cycle ends early when the implicit residual drops below tol; convergence
 * is decided on the true residual recomputed in FP64 after each cycle.
 * F32_IR: the outer FP64 loop computes r = b - A x; an inner FP32 GMRES cycle
 * (at most m steps, stop at relative reduction inner_tol) solves for the
 * correction of r/||r||, and x += ||r|| * correction in FP64.
 * Returns PP_OK, PP_WARN_DEGREE_REDUCED, PP_WARN_NOT_CONVERGED, PP_WARN_NONFINITE,
 * or an error code. */
int pp_gmres_solve(const pp_csr *A, const double *b, double *x, int m, int d, double tol,
                   const pp_opts *opt, void *stream, pp_stats *st);

/* The paper's own construction of the polynomial (Section II, eqs. (1)-(2)):
 * the power basis V = [v0, A v0, ..., A^deg v0] (left unnormalised), W = A V, and
 * the normal equations (W^T W) y = W^T v0 solved by a Cholesky factorisation on
 * the host; p(A) = sum_{k=0}^{deg} y_k A^k, applied by Horner's rule (deg fused
 * product + axpy launches).  deg+1 products and two block inner products build it.
 *   A, v0    : as for pp_build_poly (v0 device FP64, not normalised; NULL -> the
 *              seeded vector pp_uniform_vector(n, 0))
 *   deg      : 0 <= deg <= 62 and deg + 1 <= n
 *   auto_degree : nonzero -> Section IV's heuristic: factor the Gram matrices of
 *              degrees 0, 1, ..., deg (leading blocks of one matrix) and keep the
 *              highest degree before the first Cholesky failure; returns PP_OK.
 *              zero -> use degree deg; a Cholesky failure at column k keeps the
 *              coefficients of the leading (k-1) block with zeros above (the
 *              plateau of Table I) and returns PP_WARN_CHOLESKY.
 *   info_out : optional; the 1-based column where the Cholesky failed (POTRF's
 *              info), 0 if none.
 * The polynomial is usable in pp_apply and as pp_opts.poly of pp_gmres_solve.
 * Returns PP_OK, PP_WARN_CHOLESKY, PP_ERR_ARG, PP_ERR_SINGULAR (A v0 = 0 or a
 * non-finite Gram matrix), PP_ERR_HIP, PP_ERR_NOMEM. */
int pp_build_poly_power(const pp_csr *A, const double *v0, int deg, int auto_degree,
                        void *stream, pp_poly **out, int *info_out);

/* Copy a power-basis polynomial's coefficients (y_0 .. y_deg) to host c[cap];
 * *n_out = deg + 1.  Passage: Section II eq. (2) (the coefficients y of
 * p(A) = sum_k y_k A^k that the normal equations give).  PP_ERR_ARG for a
 * root-form polynomial or a short buffer. */
int pp_poly_coeffs(const pp_poly *p, double *c, int cap, int *n_out);

/* Copy the Leja-ordered roots to host arrays re[cap], im[cap]; *d_out = number
 * of roots.  Passage: the paper does not define this call.  The roots are the
 * harmonic Ritz values that define the polynomial (root form above); exporting
 * them serves checkpoint/resume (save the roots with x at a restart boundary) and
 * inspection of alpha p(alpha) on the spectrum as in Section V's figures.  A complex pair appears as (Im > 0, its conjugate) in adjacent slots.
 * Returns PP_ERR_ARG if cap is too small, a pointer is NULL, or p is a
 * power-basis polynomial. */
int pp_poly_roots(const pp_poly *p, double *re, double *im, int cap, int *d_out);

/* Make a polynomial from given roots (host arrays), e.g. to resume a solve with
 * the roots of an earlier build.  Passage: not defined by the paper; the inverse
 * of pp_poly_roots for checkpoint/resume (p(alpha) is fixed by its roots through
 * pi(alpha) = prod (1 - alpha/theta_i) = 1 - alpha p(alpha)).  The roots are used in the order given; a
 * complex root must be immediately followed by its exact conjugate, with the
 * Im > 0 member first.  dtype is the value type it will be applied in.
 * Returns PP_ERR_ARG on malformed pairs, PP_ERR_SINGULAR on a zero or
 * non-finite root. */
int pp_poly_from_roots(int64_t n, const double *re, const double *im, int d, int dtype,
                       pp_poly **out);

/* Free a polynomial (NULL is ignored).  Passage: not in the paper (ownership of
 * the pp_poly object). */
void pp_poly_free(pp_poly *p);

/* Harmonic Ritz values from a host Hessenberg matrix, in modified Leja order.
 * Passage: the roots of the minimum-residual polynomial (Section II, the root
 * form described above): the zeros of pi(alpha) = 1 - alpha p(alpha) are the
 * harmonic Ritz values of the Arnoldi process.  Host only, no device work.  Hbar is (s+1) x s, column-major with leading
 * dimension ldh >= s+1 (the Arnoldi relation A Q_s = Q_{s+1} Hbar).  Outputs
 * re[s], im[s].  Returns PP_ERR_SINGULAR if H_s is singular or a root is zero,
 * PP_ERR_EIG if the QR iteration fails. */
int pp_roots_from_hessenberg(const double *Hbar, int ldh, int s, double *re, double *im);

/* Transpose of A in CSR form (the adjoint operator for the backward solve).
 * Passage: not in the paper.  The backward (adjoint) solve A^T lam = dL/dx of a
 * differentiable solve is an addition to the paper's method; it runs the same
 * PP-GMRES on A^T with a polynomial built for A^T.
 * Outputs are caller-allocated device arrays: rp_t[n+1], ci_t[nnz], vals_t[nnz]
 * (A's dtype).  Columns of each output row come out sorted ascending, entries
 * with equal columns (duplicates) in A's row order, so the output is the same
 * on every call.  A column index outside [0, n) is PP_ERR_ARG (checked on the
 * device before any entry is placed).
 * Returns PP_OK, PP_ERR_ARG, PP_ERR_HIP, PP_ERR_NOMEM. */
int pp_csr_transpose(const pp_csr *A, int32_t *rp_t, int32_t *ci_t, void *vals_t, void *stream);

/* Gradient of a loss with respect to A's stored values, given the adjoint
 * solution lam (A^T lam = dL/dx) and the forward solution x:
 * g_vals[k] = -lam[row(k)] * x[col(k)] for every stored entry k.
 * Passage: not in the paper (the adjoint of x = A^-1 b: dL/dA = -lam x^T,
 * taken on A's stored pattern).
 * All pointers device FP64 (lam[n], x[n], g_vals[nnz]); A's dtype is ignored
 * (only the pattern is read).  Returns PP_OK, PP_ERR_ARG, PP_ERR_HIP. */
int pp_csr_grad(const pp_csr *A, const double *lam, const double *x, double *g_vals,
                void *stream);

/* ---- ILU(0), the second preconditioner of Section VI's second example ----
 * ILU(0) (the incomplete LU factorisation with no fill, Saad, "Iterative
 * Methods for Sparse Linear Systems", Section 10.3): L unit lower and U upper
 * triangular on A's pattern with (L U)_ij = a_ij for every stored (i, j).  The
 * rows keep A's order.  The factorisation and both triangular sweeps run level
 * by level on the device (the rows of a level wait only for earlier levels);
 * runs of narrow levels go to a single workgroup, wider levels to a launch
 * each, so the cost of a sweep grows with its number of levels (2N-1 for an
 * N x N grid in natural order, 3N-2 for N^3). */

/* Factor A (PP_F64; every row's columns strictly increasing, in [0, n), with a
 * stored diagonal).  Passage: Section VI, second example (ILU(0) as the left
 * preconditioner, the polynomial of M^-1 A on the right).  out receives a new pp_ilu.  Synchronises the stream.
 * Returns PP_OK; PP_ERR_ARG for a bad pattern, a non-FP64 A or null pointers;
 * PP_ERR_SINGULAR for a zero pivot or a non-finite factor entry; PP_ERR_HIP;
 * PP_ERR_NOMEM.  Not serialised with the other calls: it uses no shared
 * workspace. */
int pp_ilu0_factor(const pp_csr *A, void *stream, pp_ilu **out);

/* z = M^-1 r = U^-1 (L^-1 r) (Section VI, second example: applying the ILU(0)
 * preconditioner): device FP64 vectors of n entries; z may equal r
 * (in place).  Synchronises the stream.  A pp_ilu holds one work vector, so the
 * calls that use it (this one, and solves with it as left_ilu) are serialised on
 * it.  Returns PP_OK, PP_ERR_ARG (also when the current device is not the one M
 * was made on), PP_ERR_HIP. */
int pp_ilu0_apply(const pp_ilu *M, const double *r, double *z, void *stream);

/* Copy the factors into lu (device FP64[nnz], A's CSR order; inspection of the
 * ILU(0) of Section VI's second example, not defined by the paper): the strictly lower
 * entries hold L (its unit diagonal implied), the others U.  Synchronises.
 * Returns PP_OK, PP_ERR_ARG (null pointer, or M made on another device),
 * PP_ERR_HIP. */
int pp_ilu0_values(const pp_ilu *M, double *lu, void *stream);

/* Levels of the forward and backward sweeps, and the launches one pp_ilu0_apply
 * makes (any output pointer may be NULL; the paper defines no such call: it
 * reports the dependency chains that bound a sweep's cost).  Host only.  Returns PP_OK, or
 * PP_ERR_ARG when M is NULL. */
int pp_ilu0_levels(const pp_ilu *M, int32_t *nlev_forward, int32_t *nlev_backward,
                   int32_t *launches);

/* Free a factorisation (NULL is ignored); waits for the device first.  Passage:
 * not in the paper (ownership of the pp_ilu object). */
void pp_ilu0_free(pp_ilu *M);

/* The seeded random start vector of Section V (entries uniform on (-1, 1)), the
 * one the build and the solve draw when they are given no v0.  Generator:
 * Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC 2011), a counter-based generator: entry i is word i mod 4 of
 * the block at counter floor(i/4) + 1 with key (seed, 0) -- the stream of
 * numpy's Philox(key=(seed, 0)) bit generator -- mapped to 2 (w >> 11) 2^-53 - 1,
 * so the vector is a pure function of (n, seed), bit for bit on any device.
 *   out : device[n] FP64, written; 0 < n < 2^40
 * Synchronises the stream.  Returns PP_OK, PP_ERR_ARG, PP_ERR_HIP. */
int pp_uniform_vector(int64_t n, uint64_t seed, double *out, void *stream);

/* Free the library's device and pinned-host arena on every device.  Passage: not
 * in the paper (workspace ownership). */
void pp_release_workspace(void);

/* Human-readable name of a status code (static string).  Passage: not in the
 * paper; the warning codes follow its POTRF-style convention (results still
 * returned, Section IV). */
const char *pp_status_string(int code);

/* Where the calling thread's last PP_ERR_HIP came from: "file:line: call ->
 * hipErrorName" of the first HIP call that failed inside the library since the
 * thread's last entry into a device call, or the reason for an argument error
 * that has one (pp_apply_noalloc's size limit); "" if none.  Static per-thread
 * string, valid until the thread's next library call.  Every device entry point
 * first clears any HIP error left pending by earlier runtime calls of the
 * process (PP_LOG >= 1 reports one on stderr), so a PP_ERR_HIP always names a
 * call of the library's own.  Passage: not in the paper (error reporting). */
const char *pp_last_error(void);

/* Library version string, e.g. "libpp 0.4.0 gfx950" (not in the paper).  The minor version changes
 * whenever a struct of this header changes size or layout or an entry point is
 * added (0.2.0: pp_stats gained chain_slab_rows and chain_cached; 0.3.0: pp_opts
 * gained v0_seed, and a NULL v0 draws the seeded vector instead of using b;
 * 0.4.0: pp_last_error, pp_apply_noalloc), so a caller can check it matches the
 * header it was built with. */
const char *pp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PP_H */
