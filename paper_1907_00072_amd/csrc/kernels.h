// Launch wrappers for the gfx950 kernels (internal to libpp).
//
// Every wrapper enqueues on `stream` and returns the hipError_t of the launch.
// Vectors are device arrays of T (double or float) unless stated; "scale"
// pointers are device doubles multiplying the vector they belong to (nullptr
// = 1).  Basis matrices V are column-major with leading dimension ldv.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ppk {

constexpr int kBlock = 256;   // threads per workgroup (4 wavefronts of 64)
constexpr int kMaxCols = 64;  // columns handled by one fused CGS2 sweep
constexpr int kSlice = 64;    // rows per slice of the sliced copy (one wavefront)
constexpr int kSellBatch = 8; // slots per row whose loads are in flight together

// Sparse matrix view on the device: CSR, plus an optional sliced copy.
// The sliced copy groups the rows in slices of kSlice.  Slice s is described by
// kDesc ints at sdesc[s * kDesc]: its value offset b_s, its slot count w_s, its
// kind (1 = diagonal slice), 0, then the first kSellBatch diagonal offsets
// (zeros past w_s or for explicit-column slices).  Its values are stored
// column-major: slot j of row kSlice*s + l at b_s + kSlice*j + l.  A diagonal
// slice holds in slot j the entries on diagonal soff[s*dmax + j] (column = row
// + offset), zero where a row has none; an explicit-column slice holds row l's
// entries in order with their columns in sci, padded with column -1 and value
// 0.  When sdesc != nullptr the product kernels read only the sliced arrays and
// never rp/ci/va.
constexpr int kDesc = 16;  // ints per slice descriptor (one 64-byte scalar load)
template <typename T>
struct SpMat {
  int n;
  int nnz;
  const int32_t *rp;
  const int32_t *ci;
  const T *va;
  const int32_t *sdesc = nullptr; // [ceil(n / kSlice) * kDesc]
  const int32_t *soff = nullptr;  // [ns * dmax + kSellBatch slack]
  const int32_t *sci = nullptr;   // [snnz] (nullptr when every slice is diagonal)
  const T *sva = nullptr;         // [snnz]
  int snnz = 0;                   // stored slots x kSlice, padding included
  int snnz_ell = 0;               // the part in explicit-column slices
  int dmax = 0;                   // most slots of a diagonal slice (soff stride)
  int soff_extra = 0;             // diagonal offsets read from soff (past the descriptors)
};

// One launch of the fused product + root-update chain.
// Accumulating form (y = p(A) v):
//  kind 0 (real root): y = y_in + c1*p; p' = p - c1*A p  (fold: y += cf*p', p' not stored)
//  kind 1 (pair, first half): t = A p; y = y_in + c1*p - c2*t (t stored unless `last`)
//  kind 2 (pair, second half): p' = p - c1*t + c2*A t (fold: y = y_in + cf*p', p' not stored)
// Operator form (w = A p(A) v = v - pi(A) v, no accumulator):
//  kind 3 (real root): p' = p - c1*A p
//  kind 2 with `last`: as above, then out = ys*y_in - p'
//  kind 3 with `last`: out = ys*y_in - p'   (y_in is the chain's input vector v)
// Power-basis (Horner) form:
//  kind 4: out = c2*gs*A g + c1*ss*self   (one Horner step z <- A z + y_k v)
// g is the gathered vector (p for kinds 0/1/3, t for kind 2), self is p for kind 2.
template <typename T>
struct ChainArgs {
  const T *g;
  const double *gscale;
  const T *self;
  const double *sscale;
  T *out;
  const T *y_in;  // nullptr = zero
  T *y_out;
  double c1, c2, cf;
  const double *yscale;  // scale of y_in in the operator form's last step (nullptr = 1)
  int tile0 = 0;         // first tile (chain_tile_rows rows each) the launch covers
  int ntiles = 0;        // tiles it covers (0 = through the last row)
  // host-side choice of the cache policy: false = non-temporal loads and stores of
  // A and the vectors (a pass that touches each once), true = ordinary ones (the
  // next launch re-reads them soon)
  bool cached = false;
};

// Rows of one tile of the product launches (one workgroup): 256, or 512 for FP32
// products on the sliced copy (two slices per wavefront).
template <typename T>
inline int chain_tile_rows(const SpMat<T> &A) {
  return (A.sdesc && sizeof(T) == sizeof(float)) ? 2 * kBlock : kBlock;
}

// `fold` and `last` select the variants above (fold: kinds 0 and 2; last: kinds 1, 2, 3).
template <typename T>
hipError_t launch_chain(const SpMat<T> &A, int kind, bool fold, bool last, const ChainArgs<T> &a,
                        hipStream_t stream);

// y_out = y_in + c * (gscale * g) elementwise (a degree-0 polynomial step).
template <typename T>
hipError_t launch_axpy(int n, double c, const T *g, const double *gscale, const T *y_in, T *y_out,
                       hipStream_t stream);

// out = A * (gscale * g), on the rows of tiles [tile0, tile0 + ntiles) (ntiles = 0:
// through the last row); `cached` as ChainArgs::cached.
template <typename T>
hipError_t launch_spmv(const SpMat<T> &A, const T *g, const double *gscale, T *out,
                       hipStream_t stream, int tile0 = 0, int ntiles = 0, bool cached = false);

// *bad |= 1 when the CSR structure is malformed (row_ptr[0] != 0, row_ptr[n] !=
// nnz, a decreasing row_ptr, or a column outside [0, n)); *bad zeroed by the
// caller.  Reads only inside row_ptr[n + 1] and col_ind[nnz].
hipError_t launch_check_csr(int n, int nnz, const int32_t *rp, const int32_t *ci, int32_t *bad,
                            hipStream_t stream);

// *out = max over stored entries of |column - row| (the matrix bandwidth); *out
// zeroed by the caller.
hipError_t launch_bandwidth(int n, const int32_t *rp, const int32_t *ci, int32_t *out,
                            hipStream_t stream);

// out = b - A x (out may be a T-typed vector of the same type as A), and
// partial[tile] = sum over the tile of out^2 (double).  Returns the tile count.
template <typename T>
hipError_t launch_residual(const SpMat<T> &A, const T *b, const T *x, T *out, double *partial,
                           int *ntiles, hipStream_t stream);

// Workgroups G of a sweep of n rows at rpt rows per thread; its partials are
// laid out [column][G].
int orth_grid(int n, int rpt);

// The second stage of a sweep's reduction done inside the sweep: its last
// workgroup to finish (an atomic ticket on `counter`, a device int that is 0
// between launches and is set back to 0) sums the partials exactly as
// launch_reduce_cols (colscale, h, coef) or launch_reduce_norm (nrm, inv) would,
// so the results are bitwise the same with one launch fewer.  Worth it when the
// partials are few (the last workgroup sums them alone).
// Largest partial count a folded second stage takes: one partial per thread of the
// 256-thread reduction it reproduces.
constexpr int kFoldMaxG = kBlock;
struct FoldOut {
  int *counter = nullptr;
  const double *colscale = nullptr;
  double *h = nullptr;
  double *coef = nullptr;
  double *nrm = nullptr;
  double *inv = nullptr;
  // norm stage only (optional): after nrm, copy_src[0..copy_n) -> copy_dst, where
  // copy_dst may be pinned host memory and copy_src + nrm_at is where nrm lives
  const double *copy_src = nullptr;
  double *copy_dst = nullptr;
  int copy_n = 0;
  int nrm_at = 0;
};

// partial[(c0+c) * G + g] = sum over block g's rows of V(i, c0+c) * w(i), c < nc <= kMaxCols,
// G = orth_grid(n, rpt).  fold (optional): then also launch_reduce_cols(partial, G, c0, nc,
// fold->colscale, fold->h, fold->coef).
// cached: ordinary loads of V and w (a basis whose sweeps' working set fits the
// caches, re-read by the next sweep), else non-temporal ones.
template <typename T>
hipError_t launch_dots(int n, int rpt, const T *V, int64_t ldv, int c0, int nc, const T *w,
                       double *partial, hipStream_t stream, const FoldOut *fold = nullptr,
                       bool cached = false);

// out = w_in - sum_c V(:, c) * coef(c),  coef(c) = sign * a(c) * (b ? b(c) : 1), nc <= kMaxCols.
// w_in may be nullptr (zero) and may equal out.  With dots: partial dots of the
// new vector with V(:, 0..nc) as in launch_dots.  With norm: partial[g] = sum of
// out^2 over block g (double).  G = orth_grid(n, rpt).  fold (with dots or norm only):
// then also the matching second stage, as for launch_dots.
template <typename T>
hipError_t launch_update(int n, int rpt, const T *V, int64_t ldv, int nc, const double *coef_a,
                         const double *coef_b, double sign, const T *w_in, T *out, bool dots,
                         bool norm, double *partial, hipStream_t stream,
                         const FoldOut *fold = nullptr, bool cached = false);

// partial[g] = sum over block g of (scale*x(i))^2 in double; optionally also
// writes out32 = (float)(scale * x) when out32 != nullptr (the refinement cast).
template <typename T>
hipError_t launch_norm2(int n, int rpt, const T *x, const double *scale, float *out32,
                        double *partial, hipStream_t stream);

// Second stage of the column reductions:
//   h[c] = colscale[c0+c] * sum_g partial[(c0+c)*G + g];  coef[c] = colscale[c0+c] * h[c].
hipError_t launch_reduce_cols(const double *partial, int G, int c0, int nc, const double *colscale,
                              double *h, double *coef, hipStream_t stream);

// Norm finalisation: nrm[0] = sqrt(sum_g partial[g]); if inv != nullptr,
// inv[0] = 1/nrm (0 when nrm == 0).  With copy_dst (pinned host memory, say): then
// also copy_dst[i] = copy_src[i] for i < copy_n, where copy_src + nrm_at is nrm
// (a small result block handed to the host without a separate copy).
hipError_t launch_reduce_norm(const double *partial, int G, double *nrm, double *inv,
                              hipStream_t stream, const double *copy_src = nullptr,
                              double *copy_dst = nullptr, int copy_n = 0, int nrm_at = 0);

// Fill a device array with a value.
template <typename T>
hipError_t launch_fill(int64_t n, T value, T *x, hipStream_t stream);

// x (double) += alpha * (double) d (float or double); alpha from device (*alpha_dev).
template <typename T>
hipError_t launch_axpy_f64(int n, const double *alpha_dev, const T *d, double *x,
                           hipStream_t stream);

// out32 = (float) in64
hipError_t launch_cast_f32(int64_t n, const double *in, float *out, hipStream_t stream);

// out = (T) in64 (copy when T == double)
template <typename T>
hipError_t launch_copy_from_f64(int n, const double *in, T *out, hipStream_t stream);

// CSR transpose helpers and gradient.
hipError_t launch_count_cols(int nnz, const int32_t *ci, int32_t *cnt, hipStream_t stream);
hipError_t launch_exclusive_scan(int n, const int32_t *in, int32_t *out, int32_t *tmp,
                                 hipStream_t stream);  // out[0..n], tmp >= scan_tmp_size(n)
int64_t scan_tmp_size(int n);
// scatter: entry k of A goes to row ci[k] of the transpose (slot order set by
// atomics), with k recorded in src_t; sort_rows then orders each row by src,
// i.e. by column and duplicates by their position in A (deterministic).
template <typename T>
hipError_t launch_scatter_transpose(int n, const int32_t *rp, const int32_t *ci, const T *va,
                                    const int32_t *rp_t, int32_t *cursor, int32_t *ci_t, T *va_t,
                                    int32_t *src_t, hipStream_t stream);
template <typename T>
hipError_t launch_sort_rows(int n, const int32_t *rp, int32_t *ci, T *va, int32_t *src,
                            hipStream_t stream);
hipError_t launch_csr_grad(int n, const int32_t *rp, const int32_t *ci, const double *lam,
                           const double *x, double *g, hipStream_t stream);

// Sliced-copy construction from CSR (ns = ceil(n / kSlice) slices).
// plan: wlen[s] = kSlice * (slots of slice s), flag[s] (1 = diagonal slice),
//       wrow[s] = longest row of slice s, and (a second, one-workgroup kernel)
//       stat[0] = longest row, stat[1] = kSlice * slots of the explicit-column
//       slices, stat[2] = most slots of a diagonal slice, stat[3] = slots of
//       diagonal slices past the descriptor's first kSellBatch (sums saturate at
//       INT_MAX; the caller rejects the copy when 96 * stat[0] * ns >= 2^31,
//       which also covers any wrap).
// Then sp = exclusive scan of wlen (launch_exclusive_scan), fill_idx writes the
// slice descriptors, the diagonal offsets (soff[s * dmax + j], dmax = stat[2])
// and the explicit columns, and fill_vals the values (padding included).
hipError_t launch_slice_plan(int n, int ns, const int32_t *rp, const int32_t *ci, int32_t *wlen,
                             int32_t *flag, int32_t *wrow, int32_t *stat, hipStream_t stream);
hipError_t launch_slice_fill_idx(int n, int ns, int dmax, const int32_t *rp, const int32_t *ci,
                                 const int32_t *sp, const int32_t *flag, int32_t *sdesc,
                                 int32_t *soff, int32_t *sci, hipStream_t stream);
// sva = (D) va in sliced order (S, D in {float, double}).
template <typename S, typename D>
hipError_t launch_slice_fill_vals(int n, int ns, const int32_t *rp, const int32_t *ci, const S *va,
                                  const int32_t *sp, const int32_t *flag, D *sva,
                                  hipStream_t stream);

// out[i] = the seeded U(-1, 1) vector: entry i is word i mod 4 of the
// Philox4x64-10 block at counter floor(i/4) + 1 with key (seed, 0), mapped to
// 2 (w >> 11) 2^-53 - 1.  n < 2^40.
hipError_t launch_uniform_pm1(int64_t n, uint64_t seed, double *out, hipStream_t stream);

// Left Jacobi scaling: va_out[k] = va[k] / a_ii and b_out[i] = b[i] / a_ii for the
// row i of entry k (a_ii the sum of the row's diagonal entries); *bad is set to 1
// when a row has a zero or missing diagonal.
hipError_t launch_jacobi_scale(int n, const int32_t *rp, const int32_t *ci, const double *va,
                               const double *b, double *va_out, double *b_out, int32_t *bad,
                               hipStream_t stream);

}  // namespace ppk
