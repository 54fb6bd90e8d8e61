// Host-side dense numerics for the polynomial build (FP64, no device code).
#pragma once

#include <vector>

namespace ppn {

// One step of the product-form chain in Leja order.
//  kind == 0 (real root theta): c1 = 1/theta
//  kind == 1 (pair a +- ib):   c1 = 2a/|theta|^2, c2 = 1/|theta|^2
struct Step {
  int kind;
  double c1, c2;
};

// Eigenvalues of an s x s upper Hessenberg matrix (column-major, ld = s) by
// Francis double-shift QR.  H is overwritten.  Complex eigenvalues come out as
// exact conjugate pairs, real ones with wi == 0 exactly.  Returns 0 or a
// negative PP_ERR_* code.
int hessenberg_eigvals(int s, double *H, double *wr, double *wi);

// Harmonic Ritz values of the (s+1) x s Hessenberg Hbar (column-major, ld):
// eigenvalues of H_s + h^2 f e_s^T with H_s^T f = e_s, h = Hbar(s, s-1).
int harmonic_ritz(const double *Hbar, int ldh, int s, std::vector<double> &wr,
                  std::vector<double> &wi);

// Modified Leja order (largest modulus first; then maximal product of
// distances to the roots taken so far; complex roots as (Im>0, conjugate);
// repeats last; ties to the earlier root in (Re, Im) order).
int leja_order(const std::vector<double> &wr, const std::vector<double> &wi,
               std::vector<double> &or_, std::vector<double> &oi);

// Chain steps for roots already in order (pairs adjacent, Im>0 first).
// Returns 0, or PP_ERR_ARG for a malformed pair, PP_ERR_SINGULAR for a zero or
// non-finite root.
int step_table(const std::vector<double> &re, const std::vector<double> &im,
               std::vector<Step> &steps);

// Cholesky factor R (upper, k x k, column-major) of the leading k x k block of the
// symmetric matrix G (column-major, leading dimension ldg), column by column.
// Returns 0, or the 1-based column of the first pivot that is not positive
// (LAPACK POTRF's `info`), in which case R is unspecified.
int cholesky_upper(const double *G, int ldg, int k, std::vector<double> &R);

// Solve R^T R y = rhs (R from cholesky_upper, k x k).
void cholesky_solve(const std::vector<double> &R, int k, const double *rhs, double *y);

// One launch of a slab-skewed chain schedule: chain launch k over tiles [t0, t1).
struct SlabPart {
  int k, t0, t1;
};

// The slab-skewed order of K chain launches over ntile tiles (a matrix-powers
// style schedule, Section VII): the launches are taken `group` at a time; inside a
// group, slab b of the group's i-th launch covers the tiles [b S - i w, (b+1) S - i w)
// clipped to [0, ntile), for b = 0, 1, ... with the group's launches in order inside
// each slab (S >= 1 tiles a slab, w >= 0 tiles of bandwidth, group >= 1).  Every
// launch covers each tile exactly once, and launch k reaches a tile only after
// launch k - 1 has covered every tile within w of it.
void slab_order(int ntile, int S, int w, int K, int group, std::vector<SlabPart> &out);

}  // namespace ppn
