// gfx950 kernels of the polynomial-preconditioned GMRES hot path.
//
// Every kernel here is bandwidth-bound (sparse products, GEMV-shaped
// orthogonalisation), so there is no MFMA: the design goal is coalesced
// streaming of the matrix and the Krylov basis from HBM and a single pass over
// each per step.
//
// * Sparse products (the polynomial chain, the outer product, the residual)
//   run by default on a sliced copy of A: 64-row slices, one per wavefront,
//   stored slot-major, so lane l owns row 64 s + l and the loads of slot j of
//   the slice's 64 rows are one contiguous burst.  A slice whose rows use few
//   distinct diagonals (col - row) is stored by diagonal: slot j holds one
//   diagonal for all 64 rows (zero where a row lacks it), no column indices are
//   stored, and the gather becomes a contiguous shifted load.  Other slices
//   keep explicit columns; their gather for slot j still touches one entry of
//   64 consecutive rows.  A 64-byte descriptor per slice (value offset, slot
//   count, kind, first diagonal offsets) arrives in one scalar burst; each
//   batch of up to 8 slots issues all its loads before the first use.  No row
//   pointers, no LDS, no barrier.  FP32 products take two slices per wavefront
//   to keep more bytes in flight.  The root update of the polynomial chain is
//   fused into the epilogue, so one launch reads A once and the chain vectors
//   once; streamed data use non-temporal loads and stores so the L2 keeps the
//   gathered vector.  A launch may cover a range of tiles only (one slab of a
//   slab-skewed chain schedule); such launches, and launches over a matrix that
//   fits the Infinity Cache, take the KEEP instances, whose ordinary loads and
//   stores leave the slab in the cache for the next launch of the chain.
// * The CSR path (matrices whose slices would need heavy padding) is a
//   "CSR-stream" tile: a workgroup owns 256 consecutive rows; its threads
//   stream the tile's nonzeros contiguously (all index and value loads of a
//   chunk issued before any gather), write the products into LDS, then each
//   thread sums its own row.
// * Workgroups of the sparse products take their 256-row tiles in groups of 16
//   consecutive tiles per XCD (workgroups are dealt to the 8 XCDs round-robin),
//   so most of a tile's neighbouring rows were fetched into the same XCD's L2.
// * The Gram-Schmidt kernels keep one basis row per thread in registers (a
//   template bound on the column count, in steps of 8), so each sweep reads
//   every basis column once and updates the vector and accumulates the next
//   pass's dot products in the same sweep.  Column loads are branch-free (the
//   index is clamped to the last live column and the extra products carry a
//   zero coefficient), so all of a row's loads are in flight together.  Rows
//   per thread are chosen per sweep kind (orth_rpt).
// * All reductions are two-stage in a fixed order (per-workgroup partials in
//   memory, then a second kernel), with no floating-point atomics, so results
//   are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <climits>

#include "kernels.h"

namespace ppk {

namespace {

template <typename T>
struct LdsCap;
template <>
struct LdsCap<double> {
  static constexpr int value = 2048;
};
template <>
struct LdsCap<float> {
  static constexpr int value = 2048;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums over the 64 lanes of a wavefront of NCB per-lane values (one per basis
// column), by recursive halving: in round r (lane distance d = 32 >> r) a lane keeps
// one half of its current values, the lower half when bit d of its lane is clear,
// and adds its partner's (lane ^ d) copy of that half, so after H rounds each lane
// holds NCB >> H values, and a butterfly over the remaining low lane bits completes
// them.  H is the number of times NCB halves evenly (at most 6).  On return a[k],
// k < NCB >> H, is the wavefront's sum of column first + k, first being returned;
// the lanes that differ only in the low 6 - H bits hold the same columns and the
// same bits (a + b == b + a).  About NCB shuffles in all, against 6 per column for
// a butterfly per column.
constexpr int halvings(int ncb) {
  int h = 0;
  while (h < 6 && ncb % 2 == 0) {
    ncb /= 2;
    ++h;
  }
  return h;
}

// Round R of wave_col_sums (a template per round, so every array index is a
// compile-time constant and the values stay in registers).
template <int NCB, int R>
__device__ __forceinline__ void col_halve(double (&a)[NCB], int lane, int &first) {
  if constexpr (R < halvings(NCB)) {
    constexpr int d = 32 >> R, half = NCB >> (R + 1);
    const bool up = (lane & d) != 0;
#pragma unroll
    for (int k = 0; k < half; ++k) {
      const double give = up ? a[k] : a[k + half];
      const double keep = up ? a[k + half] : a[k];
      a[k] = keep + __shfl_xor(give, d, 64);
    }
    first += up ? half : 0;
    col_halve<NCB, R + 1>(a, lane, first);
  } else if constexpr (R < 6) {
    constexpr int d = 32 >> R;
#pragma unroll
    for (int k = 0; k < (NCB >> halvings(NCB)); ++k) a[k] += __shfl_xor(a[k], d, 64);
    col_halve<NCB, R + 1>(a, lane, first);
  }
}

template <int NCB>
__device__ __forceinline__ int wave_col_sums(double (&a)[NCB], int lane) {
  int first = 0;
  col_halve<NCB, 0>(a, lane, first);
  return first;
}

// The per-workgroup partial dots of nc (<= NCB) columns from every thread's acc:
// the wavefront sums (wave_col_sums) into red[wave][column], then thread c adds
// the four waves' sums of column c in a fixed order and writes it to
// partial[(c0 + c) * gridDim.x + blockIdx.x].
template <int NCB, typename T>
__device__ __forceinline__ void block_col_partials(const T (&acc)[NCB], int nc, int c0,
                                                   double (*red)[NCB],
                                                   double *__restrict__ partial) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int H = halvings(NCB), M = NCB >> H;
  double a[NCB];
#pragma unroll
  for (int c = 0; c < NCB; ++c) a[c] = (double)acc[c];
  const int first = wave_col_sums<NCB>(a, lane);
  if ((lane & ((1 << (6 - H)) - 1)) == 0) {
#pragma unroll
    for (int k = 0; k < M; ++k) red[wv][first + k] = a[k];
  }
  __syncthreads();
  if ((int)threadIdx.x < nc) {
    const int c = threadIdx.x;
    partial[(int64_t)(c0 + c) * gridDim.x + blockIdx.x] =
        ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
  }
}

// Sum over the 256 threads of a workgroup, identical on every thread.
__device__ __forceinline__ double block_sum(double v, double *red4) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red4[wv] = v;
  __syncthreads();
  const double r = ((red4[0] + red4[1]) + red4[2]) + red4[3];
  __syncthreads();
  return r;
}

template <typename T>
__device__ __forceinline__ T ldnt(const T *p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void stnt(T v, T *p) {
  __builtin_nontemporal_store(v, p);
}
// The product kernels' streamed operands (A and the vectors of one pass):
// non-temporal by default, since a full-range pass touches each once; ordinary
// loads and stores under KEEP, for launches whose data the next launch re-reads
// while it may still sit in the L2 and the Infinity Cache.
template <bool KEEP, typename T>
__device__ __forceinline__ T ld_pass(const T *p) {
  if constexpr (KEEP) return *p;
  else return __builtin_nontemporal_load(p);
}
template <bool KEEP, typename T>
__device__ __forceinline__ void st_pass(T v, T *p) {
  if constexpr (KEEP) *p = v;
  else __builtin_nontemporal_store(v, p);
}

// Row sums of A * g for the tile [r0, r0 + nrows) (thread t -> row r0 + t).
// All threads of the workgroup must call it; rows past the tile return 0.
// rb/re are the calling thread's row bounds (0, 0 for threads past the tile).
template <typename T, bool KEEP = false>
__device__ __forceinline__ T tile_row_sum(const SpMat<T> &A, const T *__restrict__ g, int r0,
                                          int nrows, int rb, int re, T *s_buf) {
  constexpr int CAP = LdsCap<T>::value;
  constexpr int PER = CAP / kBlock;
  const int t = threadIdx.x;
  const int kb = A.rp[r0], ke = A.rp[r0 + nrows];
  T acc = T(0);
  for (int c0 = kb; c0 < ke; c0 += CAP) {
    const int c1 = min(c0 + CAP, ke);
    int cols[PER];
    T vals[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int k = c0 + q * kBlock + t;
      if (k < c1) {
        vals[q] = ld_pass<KEEP>(A.va + k);
        cols[q] = ld_pass<KEEP>(A.ci + k);
      }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int k = c0 + q * kBlock + t;
      if (k < c1) s_buf[k - c0] = vals[q] * g[cols[q]];
    }
    __syncthreads();
    const int lo = max(rb, c0), hi = min(re, c1);
    for (int k = lo; k < hi; ++k) acc += s_buf[k - c0];
    if (c0 + CAP < ke) __syncthreads();
  }
  return acc;
}


// Makes the first 12 descriptor words live at this point, so the compiler
// issues their scalar loads as one burst here instead of sinking each into the
// branch that first needs it (which costs one scalar-memory round trip per
// branch).  Emits no instruction.
__device__ __forceinline__ void desc_barrier(const int *d) {
  asm volatile("" ::"s"(d[0]), "s"(d[1]), "s"(d[2]), "s"(d[4]), "s"(d[5]), "s"(d[6]), "s"(d[7]),
               "s"(d[8]), "s"(d[9]), "s"(d[10]), "s"(d[11]));
}

// One batch of N slots of a diagonal slice: values at sva + 64 q, diagonal
// offsets o[q]; the shifted loads are unconditional and kept in range, and an
// absent entry (value 0) selects 0, so it never reaches the product.
template <typename T, int N, bool KEEP = false>
__device__ __forceinline__ T dia_batch(const T *__restrict__ sva, const T *__restrict__ g, int row,
                                       int last, const int *o, T acc) {
  T v[N], gl[N];
#pragma unroll
  for (int q = 0; q < N; ++q) {
    v[q] = ld_pass<KEEP>(sva + q * kSlice);
    // column in unsigned arithmetic: a present entry's column lies in [0, n); for an
    // absent one the sum may fall outside (or wrap) and is clamped to row n - 1
    const unsigned col = (unsigned)row + (unsigned)o[q];
    gl[q] = g[min(col, (unsigned)last)];
  }
#pragma unroll
  for (int q = 0; q < N; ++q) acc += v[q] * (v[q] != T(0) ? gl[q] : T(0));
  return acc;
}

// One batch of N slots of an explicit-column slice (padding: column -1).
template <typename T, int N, bool KEEP = false>
__device__ __forceinline__ T ell_batch(const T *__restrict__ sva, const int32_t *__restrict__ sci,
                                       const T *__restrict__ g, T acc) {
  int c[N];
  T v[N], gv[N];
#pragma unroll
  for (int q = 0; q < N; ++q) {
    v[q] = ld_pass<KEEP>(sva + q * kSlice);
    c[q] = ld_pass<KEEP>(sci + q * kSlice);
  }
#pragma unroll
  for (int q = 0; q < N; ++q) gv[q] = c[q] >= 0 ? g[c[q]] : T(0);
#pragma unroll
  for (int q = 0; q < N; ++q) acc += v[q] * gv[q];
  return acc;
}

// Row sum of A * g for `row` from the sliced copy (thread -> row, lanes of a
// wavefront -> the 64 rows of one slice).  Rows past n return 0.  Slot counts
// are uniform across the wavefront, so each batch of up to kSellBatch slots
// runs a specialisation whose loads are all issued before any is used.
template <typename T, bool KEEP = false>
__device__ __forceinline__ T sell_row_sum(const SpMat<T> &A, const T *__restrict__ g, int row) {
  // the slice is uniform across the wavefront (tiles are 64-row aligned); saying
  // so puts the slice metadata in scalar registers and makes the branches uniform
  const int s = __builtin_amdgcn_readfirstlane(row / kSlice);
  const int lane = row - s * kSlice;
  // the slice descriptor (value offset, slots, kind, first diagonal offsets) in
  // one scalar burst; slice clamped into range so the load is unconditional
  const int ns = (A.n + kSlice - 1) / kSlice;
  const int sc = min(s, ns - 1);
  const int32_t *__restrict__ dsc = A.sdesc + (int64_t)sc * kDesc;
  int dd[kDesc];
#pragma unroll
  for (int q = 0; q < kDesc; ++q) dd[q] = dsc[q];
  desc_barrier(dd);
  const int base = dd[0], w = dd[1], dia = dd[2];
  const int *__restrict__ offs = A.soff + (int64_t)sc * A.dmax;
  int o[kSellBatch];
#pragma unroll
  for (int q = 0; q < kSellBatch; ++q) o[q] = dd[4 + q];
  T acc = T(0);
  if (s >= ns) return acc;
  const int last = A.n - 1;
  for (int j0 = 0; j0 < w; j0 += kSellBatch) {
    const int cnt = min(kSellBatch, w - j0);
    const T *sv = A.sva + base + j0 * kSlice + lane;
    if (dia) {
      if (j0 > 0) {
#pragma unroll
        for (int q = 0; q < kSellBatch; ++q) o[q] = offs[j0 + q];
      }
#define PP_DIA(N)                                         \
  case N:                                                 \
    acc = dia_batch<T, N, KEEP>(sv, g, row, last, o, acc);\
    break;
      switch (cnt) { PP_DIA(8) PP_DIA(7) PP_DIA(6) PP_DIA(5) PP_DIA(4) PP_DIA(3) PP_DIA(2) PP_DIA(1) }
#undef PP_DIA
    } else {
      const int32_t *sc = A.sci + base + j0 * kSlice + lane;
#define PP_ELL(N)                                         \
  case N:                                                 \
    acc = ell_batch<T, N, KEEP>(sv, sc, g, acc);          \
    break;
      switch (cnt) { PP_ELL(8) PP_ELL(7) PP_ELL(6) PP_ELL(5) PP_ELL(4) PP_ELL(3) PP_ELL(2) PP_ELL(1) }
#undef PP_ELL
    }
  }
  return acc;
}

// Row sums for two rows of different slices (one per wavefront each), with the
// loads of both slices in flight together when both are diagonal slices of at
// most kSellBatch slots (a slice past n counts as an empty diagonal slice);
// otherwise one slice after the other.
template <typename T, bool KEEP = false>
__device__ __forceinline__ void sell_row_sum2(const SpMat<T> &A, const T *__restrict__ g,
                                              int rowA, int rowB, T *accA, T *accB) {
  const int sA = __builtin_amdgcn_readfirstlane(rowA / kSlice);
  const int sB = __builtin_amdgcn_readfirstlane(rowB / kSlice);
  const int ns = (A.n + kSlice - 1) / kSlice;
  const bool inA = sA < ns, inB = sB < ns;
  // both slice descriptors first, unconditionally (slices clamped into range)
  const int cA = min(sA, ns - 1), cB = min(sB, ns - 1);
  const int32_t *__restrict__ dscA = A.sdesc + (int64_t)cA * kDesc;
  const int32_t *__restrict__ dscB = A.sdesc + (int64_t)cB * kDesc;
  int ddA[kDesc], ddB[kDesc];
#pragma unroll
  for (int q = 0; q < kDesc; ++q) {
    ddA[q] = dscA[q];
    ddB[q] = dscB[q];
  }
  desc_barrier(ddA);
  desc_barrier(ddB);
  int oA[kSellBatch], oB[kSellBatch];
#pragma unroll
  for (int q = 0; q < kSellBatch; ++q) {
    oA[q] = ddA[4 + q];
    oB[q] = ddB[4 + q];
  }
  const int baseA = ddA[0], wA = inA ? ddA[1] : 0, dA = inA ? ddA[2] : 1;
  const int baseB = ddB[0], wB = inB ? ddB[1] : 0, dB = inB ? ddB[2] : 1;
  if (!(dA && dB && wA <= kSellBatch && wB <= kSellBatch)) {
    *accA = inA ? sell_row_sum<T, KEEP>(A, g, rowA) : T(0);
    *accB = inB ? sell_row_sum<T, KEEP>(A, g, rowB) : T(0);
    return;
  }
  const int laneA = rowA - sA * kSlice, laneB = rowB - sB * kSlice;
  const unsigned last = (unsigned)(A.n - 1);
  T vA[kSellBatch], gA[kSellBatch], vB[kSellBatch], gB[kSellBatch];
#pragma unroll
  for (int q = 0; q < kSellBatch; ++q) {
    vA[q] = gA[q] = vB[q] = gB[q] = T(0);
    if (q < wA) {  // uniform branches
      vA[q] = ld_pass<KEEP>(A.sva + baseA + q * kSlice + laneA);
      gA[q] = g[min((unsigned)rowA + (unsigned)oA[q], last)];
    }
    if (q < wB) {
      vB[q] = ld_pass<KEEP>(A.sva + baseB + q * kSlice + laneB);
      gB[q] = g[min((unsigned)rowB + (unsigned)oB[q], last)];
    }
  }
  T a0 = T(0), a1 = T(0);
#pragma unroll
  for (int q = 0; q < kSellBatch; ++q) {
    a0 += vA[q] * (vA[q] != T(0) ? gA[q] : T(0));
    a1 += vB[q] * (vB[q] != T(0) ? gB[q] : T(0));
  }
  *accA = a0;
  *accB = a1;
}

// Tile of workgroup b among G: groups of kXcdGroup consecutive tiles go to one
// XCD (b mod 8 is the XCD a workgroup lands on); a ragged last group keeps the
// identity, so the map is a bijection on [0, G).
constexpr int kXcdGroup = 16;
__device__ __forceinline__ int xcd_tile(int b, int G) {
  constexpr int span = 8 * kXcdGroup;
  const int grp = b / span, w = b - grp * span;
  if ((grp + 1) * span > G) return b;
  return grp * span + (w % 8) * kXcdGroup + w / 8;
}

// Row sum of A * g for the calling thread's row r0 + threadIdx.x from the view's
// layout.  All threads of the workgroup must call it.
template <typename T, bool SELL, bool KEEP = false>
__device__ __forceinline__ T row_product(const SpMat<T> &A, const T *__restrict__ g, int r0,
                                         int nrows, int rb, int re) {
  if constexpr (SELL) {
    return sell_row_sum<T, KEEP>(A, g, r0 + (int)threadIdx.x);
  } else {
    __shared__ T s_buf[LdsCap<T>::value];
    return tile_row_sum<T, KEEP>(A, g, r0, nrows, rb, re, s_buf);
  }
}

// ------------------------------------------------------------------ chain
// Epilogue of one chain row (see ChainArgs for the kinds): acc = (A g)(i).
template <typename T, int KIND, bool FOLD, bool LAST, bool KEEP = false>
__device__ __forceinline__ void chain_row(const ChainArgs<T> &a, int i, T acc, T own, T yv, T sf,
                                          T gs) {
  const T c1 = (T)a.c1, c2 = (T)a.c2, cf = (T)a.cf;
  if constexpr (KIND == 0) {
    const T p = gs * own;
    const T ap = gs * acc;
    T y = yv + c1 * p;
    const T pn = p - c1 * ap;
    if constexpr (FOLD) {
      y += cf * pn;
    } else {
      st_pass<KEEP>(pn, a.out + i);
    }
    st_pass<KEEP>(y, a.y_out + i);
  } else if constexpr (KIND == 1) {
    const T p = gs * own;
    const T tt = gs * acc;
    st_pass<KEEP>(yv + c1 * p - c2 * tt, a.y_out + i);
    if constexpr (!LAST) st_pass<KEEP>(tt, a.out + i);
  } else if constexpr (KIND == 2) {
    const T ss = a.sscale ? (T)(*a.sscale) : T(1);
    const T pn = ss * sf - c1 * (gs * own) + c2 * (gs * acc);
    if constexpr (FOLD) {
      st_pass<KEEP>(yv + cf * pn, a.y_out + i);
    } else if constexpr (LAST) {
      const T ys = a.yscale ? (T)(*a.yscale) : T(1);
      st_pass<KEEP>(ys * yv - pn, a.out + i);
    } else {
      st_pass<KEEP>(pn, a.out + i);
    }
  } else if constexpr (KIND == 4) {
    const T ss = a.sscale ? (T)(*a.sscale) : T(1);
    st_pass<KEEP>(c2 * (gs * acc) + c1 * (ss * sf), a.out + i);
  } else {
    const T pn = gs * own - c1 * (gs * acc);
    if constexpr (LAST) {
      const T ys = a.yscale ? (T)(*a.yscale) : T(1);
      st_pass<KEEP>(ys * yv - pn, a.out + i);
    } else {
      st_pass<KEEP>(pn, a.out + i);
    }
  }
}

// R rows per thread: rows r0 + t + 256 r of a tile of 256 R rows (R = 2 only on
// the sliced copy, where it lets a wavefront keep two slices' loads in flight).
template <typename T, int KIND, bool FOLD, bool LAST, bool SELL, int R, bool KEEP = false>
__global__ __launch_bounds__(kBlock) void k_chain(SpMat<T> A, ChainArgs<T> a) {
  static_assert(R == 1 || (R == 2 && SELL), "two rows per thread need the sliced copy");
  const int r0 = (a.tile0 + xcd_tile(blockIdx.x, gridDim.x)) * kBlock * R;
  const int t = threadIdx.x;
  constexpr bool kReadY = (KIND == 0) || (KIND == 1) || (KIND == 2 && (FOLD || LAST)) ||
                          (KIND == 3 && LAST);
  constexpr bool kReadSelf = (KIND == 2) || (KIND == 4);
  // own-row operands first, so their latency overlaps the product
  int rb = 0, re = 0;
  T own[R], yv[R], sf[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = r0 + r * kBlock + t;
    own[r] = yv[r] = sf[r] = T(0);
    if (i < A.n) {
      if constexpr (!SELL) {
        rb = A.rp[i];
        re = A.rp[i + 1];
      }
      own[r] = a.g[i];
      if (kReadY) yv[r] = a.y_in ? ld_pass<KEEP>(a.y_in + i) : T(0);
      if (kReadSelf) sf[r] = ld_pass<KEEP>(a.self + i);
    }
  }
  T acc[R];
  if constexpr (R == 1) {
    acc[0] = row_product<T, SELL, KEEP>(A, a.g, r0, min(kBlock, A.n - r0), rb, re);
  } else {
    sell_row_sum2<T, KEEP>(A, a.g, r0 + t, r0 + kBlock + t, &acc[0], &acc[1]);
  }
  // read after the product's loads are issued, so its latency is not on their path
  const T gs = a.gscale ? (T)(*a.gscale) : T(1);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = r0 + r * kBlock + t;
    if (i < A.n) chain_row<T, KIND, FOLD, LAST, KEEP>(a, i, acc[r], own[r], yv[r], sf[r], gs);
  }
}

// R rows per thread as in k_chain (R = 2 only on the sliced copy).
template <typename T, bool SELL, int R, bool KEEP = false>
__global__ __launch_bounds__(kBlock) void k_spmv(SpMat<T> A, const T *__restrict__ g,
                                                 const double *gscale, T *__restrict__ out,
                                                 int tile0) {
  static_assert(R == 1 || (R == 2 && SELL), "two rows per thread need the sliced copy");
  const int r0 = (tile0 + xcd_tile(blockIdx.x, gridDim.x)) * kBlock * R;
  const int t = threadIdx.x;
  T acc[R];
  if constexpr (R == 1) {
    const int nrows = min(kBlock, A.n - r0);
    int rb = 0, re = 0;
    if constexpr (!SELL) {
      if (t < nrows) {
        rb = A.rp[r0 + t];
        re = A.rp[r0 + t + 1];
      }
    }
    acc[0] = row_product<T, SELL, KEEP>(A, g, r0, nrows, rb, re);
  } else {
    sell_row_sum2<T, KEEP>(A, g, r0 + t, r0 + kBlock + t, &acc[0], &acc[1]);
  }
  const T gs = gscale ? (T)(*gscale) : T(1);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = r0 + r * kBlock + t;
    if (i < A.n) st_pass<KEEP>(gs * acc[r], out + i);
  }
}

template <typename T, bool SELL>
__global__ __launch_bounds__(kBlock) void k_residual(SpMat<T> A, const T *__restrict__ b,
                                                     const T *__restrict__ x, T *__restrict__ out,
                                                     double *__restrict__ partial) {
  __shared__ double red[4];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int r0 = tile * kBlock;
  const int nrows = min(kBlock, A.n - r0);
  const int i = r0 + threadIdx.x;
  int rb = 0, re = 0;
  T bi = T(0);
  if ((int)threadIdx.x < nrows) {
    if constexpr (!SELL) {
      rb = A.rp[i];
      re = A.rp[i + 1];
    }
    bi = ldnt(b + i);
  }
  const T acc = row_product<T, SELL>(A, x, r0, nrows, rb, re);
  double sq = 0.0;
  if ((int)threadIdx.x < nrows) {
    const T r = bi - acc;
    stnt(r, out + i);
    sq = (double)r * (double)r;
  }
  sq = block_sum(sq, red);
  if (threadIdx.x == 0) partial[tile] = sq;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpy(int n, double c, const T *__restrict__ g,
                                                 const double *gscale, const T *y_in, T *y_out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const T gs = gscale ? (T)(*gscale) : T(1);
  y_out[i] = (y_in ? y_in[i] : T(0)) + (T)c * (gs * g[i]);
}

// ------------------------------------------------------------------ CGS2
// Fixed-order sum of x[0..G) over the workgroup's threads (thread t takes
// t, t + 256, ...), with four loads in flight per thread.
__device__ __forceinline__ double strided_sum(const double *__restrict__ x, int G) {
  double s = 0.0;
  int g = threadIdx.x;
  for (; g + 3 * kBlock < G; g += 4 * kBlock) {
    const double a0 = x[g], a1 = x[g + kBlock], a2 = x[g + 2 * kBlock], a3 = x[g + 3 * kBlock];
    s += (a0 + a1) + (a2 + a3);
  }
  for (; g < G; g += kBlock) s += x[g];
  return s;
}

// Second stage of a column reduction (one workgroup): h[c] = colscale[c] * sum of
// the G partials of column c, coef[c] = colscale[c] * h[c].  The same arithmetic
// whether it runs in k_reduce_cols or in the producing sweep's last workgroup.
__device__ __forceinline__ void reduce_col_finish(const double *__restrict__ partial, int G,
                                                  int c, const double *colscale, double *h,
                                                  double *coef, double *red4) {
  double s = strided_sum(partial + (int64_t)c * G, G);
  s = block_sum(s, red4);
  if (threadIdx.x == 0) {
    const double sc = colscale ? colscale[c] : 1.0;
    const double hv = sc * s;
    h[c] = hv;
    if (coef) coef[c] = sc * hv;
  }
}

// Second stage of a norm: nrm = sqrt(sum of the G partials), inv = 1/nrm (0 for 0).
__device__ __forceinline__ void reduce_norm_finish(const double *__restrict__ partial, int G,
                                                   double *nrm, double *inv, double *red4) {
  double s = strided_sum(partial, G);
  s = block_sum(s, red4);
  if (threadIdx.x == 0) {
    const double r = sqrt(s);
    nrm[0] = r;
    if (inv) inv[0] = (r > 0.0) ? 1.0 / r : 0.0;
  }
}

// What block_sum(strided_sum(x, G)) returns in a 256-thread workgroup, for
// G <= 256, computed by one wavefront: lane l stands for threads l, l + 64,
// l + 128 and l + 192 in turn (each holds 0.0 + x[t] or 0.0, as strided_sum
// leaves it), each group is summed by the same butterfly as wave_sum, and the
// four group sums are added in block_sum's order.  Bitwise the same value.
__device__ __forceinline__ double col_sum_as_block(const double *__restrict__ x, int G) {
  const int lane = threadIdx.x & 63;
  double v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int t = 64 * k + lane;
    v[k] = 0.0;
    if (t < G) v[k] += x[t];
  }
  double r[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k] = wave_sum(v[k]);
  return ((r[0] + r[1]) + r[2]) + r[3];
}

// The folded column stage: wavefront w of the last workgroup finishes columns
// w, w + 4, ... (as reduce_col_finish, G <= kFoldMaxG).
__device__ __forceinline__ void fold_cols(const double *__restrict__ partial, int G, int c0,
                                          int nc, const FoldOut &f) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int c = c0 + wv; c < c0 + nc; c += 4) {
    const double s = col_sum_as_block(partial + (int64_t)c * G, G);
    if (lane == 0) {
      const double sc = f.colscale ? f.colscale[c] : 1.0;
      const double hv = sc * s;
      f.h[c] = hv;
      if (f.coef) f.coef[c] = sc * hv;
    }
  }
}

// The folded norm stage (as reduce_norm_finish, G <= kFoldMaxG), by wavefront 0.
// With copy_dst set, the workgroup then copies copy_src[0..copy_n) there, the norm
// itself written from the register (the other entries come from earlier launches).
// Called by every thread of the workgroup.
__device__ __forceinline__ void fold_norm(const double *__restrict__ partial, int G,
                                          const FoldOut &f) {
  __shared__ double s_r;
  if (threadIdx.x < 64) {
    const double s = col_sum_as_block(partial, G);
    if (threadIdx.x == 0) {
      const double r = sqrt(s);
      f.nrm[0] = r;
      if (f.inv) f.inv[0] = (r > 0.0) ? 1.0 / r : 0.0;
      s_r = r;
    }
  }
  if (f.copy_dst) {
    __syncthreads();
    const double r = s_r;
    for (int i = threadIdx.x; i < f.copy_n; i += kBlock)
      f.copy_dst[i] = (i == f.nrm_at) ? r : f.copy_src[i];
  }
}

// Called by every thread of a sweep's workgroup once wave 0 has stored the
// workgroup's partials (those stores all come from threads < 64).  Wave 0
// releases them at device scope and takes a ticket; the workgroup that draws
// the last ticket acquires every other workgroup's partials and returns true.
// The counter is re-armed (set back to 0) by that workgroup.
__device__ __forceinline__ bool last_to_arrive(int *counter) {
  __shared__ int s_last;
  if (threadIdx.x < 64) {
    __threadfence();
    if (threadIdx.x == 0) s_last = (atomicAdd(counter, 1) == (int)gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) {
    __threadfence();
    if (threadIdx.x == 0) *counter = 0;
  }
  return last;
}

// KEEP: ordinary loads (the basis re-read from the caches by the next sweep, for a
// working set that fits them); otherwise non-temporal.
template <typename T, int NCB, bool FOLD, bool KEEP>
__global__ __launch_bounds__(kBlock) void k_dots(int n, int rpt, const T *__restrict__ V,
                                                 int64_t ldv, int c0, int nc,
                                                 const T *__restrict__ w,
                                                 double *__restrict__ partial, FoldOut f) {
  __shared__ double red[4][NCB];
  T acc[NCB];
#pragma unroll
  for (int c = 0; c < NCB; ++c) acc[c] = T(0);
  const int64_t base = (int64_t)blockIdx.x * rpt * kBlock + threadIdx.x;
  const T *Vc = V + (int64_t)c0 * ldv;
  for (int r = 0; r < rpt; ++r) {
    const int64_t i = base + (int64_t)r * kBlock;
    if (i < n) {
      T v[NCB];
#pragma unroll
      for (int c = 0; c < NCB; ++c) v[c] = ld_pass<KEEP>(Vc + (int64_t)min(c, nc - 1) * ldv + i);
      const T wi = ld_pass<KEEP>(w + i);
      // keep every load of the row ahead of the arithmetic (the scheduler would
      // otherwise interleave load/wait/fma to save registers)
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int c = 0; c < NCB; ++c) acc[c] += v[c] * wi;
    }
  }
  block_col_partials<NCB>(acc, nc, c0, red, partial);
  if constexpr (FOLD) {
    if (last_to_arrive(f.counter)) fold_cols(partial, gridDim.x, c0, nc, f);
  }
}

template <typename T, int NCB, bool DOTS, bool NORM, bool FOLD, bool KEEP>
__global__ __launch_bounds__(kBlock) void k_update(int n, int rpt, const T *__restrict__ V,
                                                   int64_t ldv, int nc, const double *coef_a,
                                                   const double *coef_b, double sign,
                                                   const T *w_in, T *out,
                                                   double *__restrict__ partial, FoldOut f) {
  __shared__ T s_coef[NCB];
  __shared__ double red[4][DOTS ? NCB : 1];
  __shared__ double red4[4];
  if ((int)threadIdx.x < NCB) {
    const int c = threadIdx.x;
    s_coef[c] = c < nc ? (T)(sign * coef_a[c] * (coef_b ? coef_b[c] : 1.0)) : T(0);
  }
  __syncthreads();
  T coef[NCB];
#pragma unroll
  for (int c = 0; c < NCB; ++c) coef[c] = s_coef[c];
  T acc[DOTS ? NCB : 1];
#pragma unroll
  for (int c = 0; c < (DOTS ? NCB : 1); ++c) acc[c] = T(0);
  double nacc = 0.0;
  const int64_t base = (int64_t)blockIdx.x * rpt * kBlock + threadIdx.x;
  for (int r = 0; r < rpt; ++r) {
    const int64_t i = base + (int64_t)r * kBlock;
    if (i < n) {
      T v[NCB];
#pragma unroll
      for (int c = 0; c < NCB; ++c) v[c] = ld_pass<KEEP>(V + (int64_t)min(c, nc - 1) * ldv + i);
      T wi = w_in ? ld_pass<KEEP>(w_in + i) : T(0);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int c = 0; c < NCB; ++c) wi -= v[c] * coef[c];
      st_pass<KEEP>(wi, out + i);
      if constexpr (DOTS) {
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[c] += v[c] * wi;
      }
      if constexpr (NORM) nacc += (double)wi * (double)wi;
    }
  }
  if constexpr (DOTS) {
    block_col_partials<NCB>(acc, nc, 0, red, partial);
    if constexpr (FOLD) {
      if (last_to_arrive(f.counter)) fold_cols(partial, gridDim.x, 0, nc, f);
    }
  }
  if constexpr (NORM) {
    const double s = block_sum(nacc, red4);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
    if constexpr (FOLD) {
      if (last_to_arrive(f.counter)) fold_norm(partial, gridDim.x, f);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_norm2(int n, int rpt, const T *__restrict__ x,
                                                  const double *scale, float *out32,
                                                  double *__restrict__ partial) {
  __shared__ double red4[4];
  const double sc = scale ? *scale : 1.0;
  double acc = 0.0;
  const int64_t base = (int64_t)blockIdx.x * rpt * kBlock + threadIdx.x;
  for (int r = 0; r < rpt; ++r) {
    const int64_t i = base + (int64_t)r * kBlock;
    if (i < n) {
      const double v = (double)x[i] * sc;
      if (out32) {
        const float f = (float)v;
        out32[i] = f;
        acc += (double)f * (double)f;
      } else {
        acc += v * v;
      }
    }
  }
  acc = block_sum(acc, red4);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kBlock) void k_reduce_cols(const double *__restrict__ partial, int G,
                                                        int c0, const double *colscale, double *h,
                                                        double *coef) {
  __shared__ double red4[4];
  reduce_col_finish(partial, G, c0 + blockIdx.x, colscale, h, coef, red4);
}

// With copy_dst: then copy_src[0..copy_n) -> copy_dst (pinned host memory, say),
// the norm itself (copy_src[nrm_at]) written from the register.
__global__ __launch_bounds__(kBlock) void k_reduce_norm(const double *__restrict__ partial, int G,
                                                        double *nrm, double *inv,
                                                        const double *copy_src, double *copy_dst,
                                                        int copy_n, int nrm_at) {
  __shared__ double red4[4];
  __shared__ double s_r;
  reduce_norm_finish(partial, G, nrm, inv, red4);
  if (copy_dst) {
    if (threadIdx.x == 0) s_r = nrm[0];
    __syncthreads();
    const double r = s_r;
    for (int i = threadIdx.x; i < copy_n; i += kBlock)
      copy_dst[i] = (i == nrm_at) ? r : copy_src[i];
  }
}

// ------------------------------------------------------------ elementwise
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, T value, T *x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = value;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpy_f64(int n, const double *alpha,
                                                     const T *__restrict__ d, double *x) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] += (*alpha) * (double)d[i];
}

__global__ __launch_bounds__(kBlock) void k_cast_f32(int64_t n, const double *__restrict__ in,
                                                     float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy_from_f64(int n, const double *__restrict__ in,
                                                          T *__restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = (T)in[i];
}

// ------------------------------------------------------------- transpose
__global__ __launch_bounds__(kBlock) void k_count_cols(int nnz, const int32_t *__restrict__ ci,
                                                       int32_t *cnt) {
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < nnz; k += gridDim.x * kBlock)
    atomicAdd(&cnt[ci[k]], 1);
}

constexpr int kScanPerThread = 4;
constexpr int kScanPerBlock = kBlock * kScanPerThread;

// Exclusive scan of thread sums inside a workgroup; returns the workgroup total.
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t *s, int32_t *excl) {
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int32_t add = (t >= off) ? s[t - off] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  *excl = s[t] - v;
  const int32_t total = s[kBlock - 1];
  __syncthreads();
  return total;
}

// out[1 + i] = inclusive scan of in inside each 1024-element chunk; tmp[chunk] = chunk total.
__global__ __launch_bounds__(kBlock) void k_scan_chunks(int n, const int32_t *__restrict__ in,
                                                        int32_t *__restrict__ out,
                                                        int32_t *__restrict__ tmp) {
  __shared__ int32_t s[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanPerBlock + threadIdx.x * kScanPerThread;
  int32_t v[kScanPerThread];
  int32_t sum = 0;
#pragma unroll
  for (int q = 0; q < kScanPerThread; ++q) {
    v[q] = (base + q < n) ? in[base + q] : 0;
    sum += v[q];
  }
  int32_t excl;
  const int32_t total = block_exclusive_scan(sum, s, &excl);
  int32_t run = excl;
#pragma unroll
  for (int q = 0; q < kScanPerThread; ++q) {
    run += v[q];
    if (base + q < n) out[1 + base + q] = run;
  }
  if (threadIdx.x == 0) tmp[blockIdx.x] = total;
}

// Exclusive scan of the chunk totals in place (one workgroup).
__global__ __launch_bounds__(kBlock) void k_scan_tops(int nchunks, int32_t *tmp) {
  __shared__ int32_t s[kBlock];
  int32_t carry = 0;
  for (int c0 = 0; c0 < nchunks; c0 += kBlock) {
    const int i = c0 + threadIdx.x;
    const int32_t v = (i < nchunks) ? tmp[i] : 0;
    int32_t excl;
    const int32_t total = block_exclusive_scan(v, s, &excl);
    if (i < nchunks) tmp[i] = carry + excl;
    carry += total;
  }
}

__global__ __launch_bounds__(kBlock) void k_scan_add(int n, int32_t *out,
                                                     const int32_t *__restrict__ tmp) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i == 0) out[0] = 0;
  if (i < n) out[1 + i] += tmp[i / kScanPerBlock];
}

// Places entry k = (i, j) of A in row j of the transpose at a slot taken with an
// atomic cursor (so in no fixed order), recording k in src_t.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter_transpose(
    int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const T *__restrict__ va, const int32_t *__restrict__ rp_t, int32_t *cursor,
    int32_t *__restrict__ ci_t, T *__restrict__ va_t, int32_t *__restrict__ src_t) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int j = ci[k];
    const int pos = rp_t[j] + atomicAdd(&cursor[j], 1);
    ci_t[pos] = i;
    va_t[pos] = va[k];
    src_t[pos] = k;
  }
}

// Insertion sort of each row by A's entry index src (unique), which orders the
// row by column and duplicate columns by their position in A: the same output
// whatever order the scatter's atomics produced.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sort_rows(int n, const int32_t *__restrict__ rp,
                                                      int32_t *ci, T *va, int32_t *src) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int lo = rp[i], hi = rp[i + 1];
  for (int k = lo + 1; k < hi; ++k) {
    const int key = src[k];
    const int col = ci[k];
    const T val = va[k];
    int q = k - 1;
    while (q >= lo && src[q] > key) {
      src[q + 1] = src[q];
      ci[q + 1] = ci[q];
      va[q + 1] = va[q];
      --q;
    }
    src[q + 1] = key;
    ci[q + 1] = col;
    va[q + 1] = val;
  }
}

__global__ __launch_bounds__(kBlock) void k_csr_grad(int n, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     const double *__restrict__ lam,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ g) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double li = lam[i];
  for (int k = rp[i]; k < rp[i + 1]; ++k) g[k] = -li * x[ci[k]];
}

// ------------------------------------------------------- sliced copy
// Distinct diagonals of a slice in increasing order, one per call, by a k-way
// merge over the wavefront's rows (each row's columns strictly increasing):
// returns the next offset m = col - row (INT_MAX when all rows are consumed)
// and sets *take to the index (within the row) of this lane's entry on that
// diagonal, or -1.  All 64 lanes of the wavefront must call it together.
__device__ __forceinline__ int next_diagonal(const int32_t *__restrict__ ci, int rb, int len,
                                             int row, int *p, int *take) {
  const int cur = (*p < len) ? ci[rb + *p] - row : INT_MAX;
  int m = cur;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = min(m, __shfl_xor(m, off, 64));
  *take = -1;
  if (cur == m && m != INT_MAX) {
    *take = *p;
    ++*p;
  }
  return m;
}

// Rows of at most kRowRegs entries are staged in registers for the merge
// (one burst of loads per lane instead of one dependent load per step).
constexpr int kRowRegs = 32;

// This lane's row in registers: columns c[q] (INT_MAX past the row) and, when V
// is not void, values v[q].
template <typename S>
__device__ __forceinline__ void stage_row(const int32_t *__restrict__ ci, const S *__restrict__ va,
                                          int rb, int len, int *c, S *v) {
#pragma unroll
  for (int q = 0; q < kRowRegs; ++q) {
    c[q] = q < len ? ci[rb + q] : INT_MAX;
    if (va) v[q] = q < len ? va[rb + q] : S(0);
  }
}

// Register form of next_diagonal on a staged row: the lane's next column is
// c[0]; taking it shifts the row (and its values) left by one.  Returns m and
// sets *hit when this lane's entry lies on diagonal m.
template <typename S>
__device__ __forceinline__ int next_diagonal_regs(int *c, S *v, int row, bool *hit) {
  const int cur = c[0] == INT_MAX ? INT_MAX : c[0] - row;
  int m = cur;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = min(m, __shfl_xor(m, off, 64));
  *hit = cur == m && m != INT_MAX;
  if (*hit) {
#pragma unroll
    for (int q = 0; q + 1 < kRowRegs; ++q) {
      c[q] = c[q + 1];
      v[q] = v[q + 1];
    }
    c[kRowRegs - 1] = INT_MAX;
  }
  return m;
}

// Plan of the sliced copy: per slice, the longest row w and the slot count:
// the number of distinct diagonals when every row's columns strictly increase
// and that number is at most 1.5 w (then flag = 1: stored by diagonal), else w
// (flag = 0: explicit columns).  wlen[s] = 64 * slots (wrapping modulo 2^32),
// wrow[s] = w.  No atomics: k_slice_stats reduces the per-slice values.
__global__ __launch_bounds__(kBlock) void k_slice_plan(int n, int ns,
                                                       const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci,
                                                       int32_t *__restrict__ wlen,
                                                       int32_t *__restrict__ flag,
                                                       int32_t *__restrict__ wrow) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int s = i / kSlice;  // uniform across the wavefront
  const int lane = threadIdx.x & 63;
  int rb = 0, len = 0;
  if (i < n) {
    rb = rp[i];
    len = rp[i + 1] - rb;
  }
  int w = len;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) w = max(w, __shfl_xor(w, off, 64));
  const bool regs = w <= kRowRegs;  // uniform
  int c[kRowRegs];
  char nov[kRowRegs];  // no values needed here
  bool sorted = true;
  if (regs) {
    stage_row<char>(ci, nullptr, rb, len, c, nov);
#pragma unroll
    for (int q = 1; q < kRowRegs; ++q) sorted = sorted && (q >= len || c[q] > c[q - 1]);
  } else {
    for (int k = 1; k < len; ++k) sorted = sorted && (ci[rb + k] > ci[rb + k - 1]);
  }
  const bool all_sorted = __ballot(!sorted) == 0;
  int slots = w, dia = 0;
  if (s < ns && all_sorted && w > 0) {
    const int cap = w + w / 2;
    int p = 0, take = -1, cnt = 0;
    bool hit = false;
    while (cnt <= cap) {  // cnt and the returned m are uniform across the wavefront
      const int m = regs ? next_diagonal_regs<char>(c, nov, i, &hit)
                         : next_diagonal(ci, rb, len, i, &p, &take);
      if (m == INT_MAX) break;
      ++cnt;
    }
    if (cnt <= cap) {
      slots = cnt;
      dia = 1;
    }
  }
  if (lane == 0 && s < ns) {
    wlen[s] = (int32_t)((uint32_t)kSlice * (uint32_t)slots);
    flag[s] = dia;
    wrow[s] = w;
  }
}

// Totals of the plan in one workgroup, in a fixed order: stat[0] = longest row,
// stat[1] = 64 * slots of explicit-column slices, stat[2] = most slots of a
// diagonal slice, stat[3] = slots of diagonal slices past the descriptor's
// kSellBatch (sums saturate at INT_MAX; the caller rejects the copy when
// 96 * stat[0] * ns >= 2^31).
__global__ __launch_bounds__(1024) void k_slice_stats(int ns, const int32_t *__restrict__ wlen,
                                                      const int32_t *__restrict__ flag,
                                                      const int32_t *__restrict__ wrow,
                                                      int32_t *__restrict__ stat) {
  __shared__ int64_t red[4][1024 / 64];
  int64_t mrow = 0, ell = 0, dmax = 0, extra = 0;
  for (int s = threadIdx.x; s < ns; s += 1024) {
    const int64_t slots = (uint32_t)wlen[s] / kSlice;
    mrow = max(mrow, (int64_t)wrow[s]);
    if (flag[s]) {
      dmax = max(dmax, slots);
      extra += max(slots - kSellBatch, (int64_t)0);
    } else {
      ell += kSlice * slots;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mrow = max(mrow, (int64_t)__shfl_xor(mrow, off, 64));
    dmax = max(dmax, (int64_t)__shfl_xor(dmax, off, 64));
    ell += __shfl_xor(ell, off, 64);
    extra += __shfl_xor(extra, off, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = mrow;
    red[1][wv] = ell;
    red[2][wv] = dmax;
    red[3][wv] = extra;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int q = threadIdx.x;
    int64_t r = red[q][0];
    for (int k = 1; k < 1024 / 64; ++k) r = (q == 0 || q == 2) ? max(r, red[q][k]) : r + red[q][k];
    stat[q] = (int32_t)min(r, (int64_t)INT_MAX);
  }
}

// Index part of the sliced copy: the diagonal offsets of diagonal slices
// (soff[s * dmax + j]) and the columns of explicit-column slices (sci, -1 =
// padding; sci may be nullptr when every slice is diagonal).
__global__ __launch_bounds__(kBlock) void k_slice_fill_idx(int n, int ns, int dmax,
                                                           const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const int32_t *__restrict__ sp,
                                                           const int32_t *__restrict__ flag,
                                                           int32_t *__restrict__ sdesc,
                                                           int32_t *__restrict__ soff,
                                                           int32_t *__restrict__ sci) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int s = i / kSlice;
  if (s >= ns) return;  // whole wavefronts
  const int lane = i - s * kSlice;
  const int base = sp[s], w = (sp[s + 1] - base) / kSlice;
  int32_t *d = sdesc + (int64_t)s * kDesc;
  // descriptor: value offset, slots, kind; diagonal offsets below, zeros elsewhere
  if (lane < kDesc) d[lane] = lane == 0 ? base : lane == 1 ? w : lane == 2 ? flag[s] : 0;
  int rb = 0, len = 0;
  if (i < n) {
    rb = rp[i];
    len = rp[i + 1] - rb;
  }
  if (flag[s]) {
    int lw = len;  // longest row of the slice (uniform), to pick the register path
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lw = max(lw, __shfl_xor(lw, off, 64));
    int c[kRowRegs];
    char nov[kRowRegs];
    const bool regs = lw <= kRowRegs;
    if (regs) stage_row<char>(ci, nullptr, rb, len, c, nov);
    int p = 0, take = -1;
    bool hit = false;
    for (int j = 0; j < w; ++j) {
      const int m = regs ? next_diagonal_regs<char>(c, nov, i, &hit)
                         : next_diagonal(ci, rb, len, i, &p, &take);
      if (lane == 0) {
        soff[(int64_t)s * dmax + j] = m;
        if (j < kSellBatch) d[4 + j] = m;
      }
    }
  } else {
    for (int j = 0; j < w; ++j) sci[base + j * kSlice + lane] = j < len ? ci[rb + j] : -1;
  }
}

// Values of the sliced copy in D (zero where a row has no entry in the slot).
template <typename S, typename D>
__global__ __launch_bounds__(kBlock) void k_slice_fill_vals(int n, int ns,
                                                            const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ ci,
                                                            const S *__restrict__ va,
                                                            const int32_t *__restrict__ sp,
                                                            const int32_t *__restrict__ flag,
                                                            D *__restrict__ sva) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int s = i / kSlice;
  if (s >= ns) return;  // whole wavefronts
  const int lane = i - s * kSlice;
  const int base = sp[s], w = (sp[s + 1] - base) / kSlice;
  int rb = 0, len = 0;
  if (i < n) {
    rb = rp[i];
    len = rp[i + 1] - rb;
  }
  if (flag[s]) {
    int lw = len;  // longest row of the slice (uniform), to pick the register path
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lw = max(lw, __shfl_xor(lw, off, 64));
    if (lw <= kRowRegs) {
      int c[kRowRegs];
      S v[kRowRegs];
      stage_row<S>(ci, va, rb, len, c, v);
      bool hit = false;
      for (int j = 0; j < w; ++j) {
        const S head = v[0];  // the entry a hit takes, before the row shifts
        (void)next_diagonal_regs<S>(c, v, i, &hit);
        sva[base + j * kSlice + lane] = hit ? (D)head : D(0);
      }
    } else {
      int p = 0, take = -1;
      for (int j = 0; j < w; ++j) {
        (void)next_diagonal(ci, rb, len, i, &p, &take);
        sva[base + j * kSlice + lane] = take >= 0 ? (D)va[rb + take] : D(0);
      }
    }
  } else {
    for (int j = 0; j < w; ++j) sva[base + j * kSlice + lane] = j < len ? (D)va[rb + j] : D(0);
  }
}

__global__ __launch_bounds__(kBlock) void k_jacobi_scale(int n, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci,
                                                         const double *__restrict__ va,
                                                         const double *__restrict__ b,
                                                         double *__restrict__ va_out,
                                                         double *__restrict__ b_out,
                                                         int32_t *bad) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int lo = rp[i], hi = rp[i + 1];
  double dg = 0.0;
  for (int k = lo; k < hi; ++k)
    if (ci[k] == i) dg += va[k];
  if (dg == 0.0 || !isfinite(dg)) {
    *bad = 1;
    dg = 1.0;
  }
  const double inv = 1.0 / dg;
  for (int k = lo; k < hi; ++k) va_out[k] = va[k] * inv;
  b_out[i] = b[i] * inv;
}

inline int tiles_of(int n) { return (n + kBlock - 1) / kBlock; }
inline unsigned blocks_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

// ------------------------------------------------------------- wrappers
template <typename T>
hipError_t launch_chain(const SpMat<T> &A, int kind, bool fold, bool last, const ChainArgs<T> &a,
                        hipStream_t stream) {
  // FP32 on the sliced copy: two rows per thread (measured +8% on the FP32 step;
  // no gain in FP64, whose single-slice loads already fill the memory pipes)
  const bool two = A.sdesc && sizeof(T) == sizeof(float);
  const dim3 grid(a.ntiles > 0 ? a.ntiles : tiles_of(A.n) - a.tile0),
      grid2(a.ntiles > 0 ? a.ntiles : (A.n + 2 * kBlock - 1) / (2 * kBlock) - a.tile0),
      block(kBlock);
#define PP_CHAIN_P(K, F, L, C)                                                                \
  do {                                                                                        \
    if (two)                                                                                  \
      hipLaunchKernelGGL((k_chain<T, K, F, L, true, 2, C>), grid2, block, 0, stream, A, a);   \
    else if (A.sdesc)                                                                         \
      hipLaunchKernelGGL((k_chain<T, K, F, L, true, 1, C>), grid, block, 0, stream, A, a);    \
    else                                                                                      \
      hipLaunchKernelGGL((k_chain<T, K, F, L, false, 1, C>), grid, block, 0, stream, A, a);   \
  } while (0)
// cached (a.cached) or non-temporal loads and stores
#define PP_CHAIN(K, F, L)                          \
  do {                                             \
    if (a.cached) PP_CHAIN_P(K, F, L, true);       \
    else PP_CHAIN_P(K, F, L, false);               \
  } while (0)
  switch (kind) {
    case 0:
      if (fold) PP_CHAIN(0, true, false); else PP_CHAIN(0, false, false);
      break;
    case 1:
      if (last) PP_CHAIN(1, false, true); else PP_CHAIN(1, false, false);
      break;
    case 2:
      if (fold) PP_CHAIN(2, true, false);
      else if (last) PP_CHAIN(2, false, true);
      else PP_CHAIN(2, false, false);
      break;
    case 3:
      if (last) PP_CHAIN(3, false, true); else PP_CHAIN(3, false, false);
      break;
    case 4:
      PP_CHAIN(4, false, false);
      break;
    default:
      return hipErrorInvalidValue;
  }
#undef PP_CHAIN
#undef PP_CHAIN_P
  return hipGetLastError();
}

template <typename T>
hipError_t launch_axpy(int n, double c, const T *g, const double *gscale, const T *y_in, T *y_out,
                       hipStream_t stream) {
  hipLaunchKernelGGL((k_axpy<T>), dim3(blocks_of(n)), dim3(kBlock), 0, stream, n, c, g, gscale,
                     y_in, y_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spmv(const SpMat<T> &A, const T *g, const double *gscale, T *out,
                       hipStream_t stream, int tile0, int ntiles, bool cached) {
  const int all = (A.n + chain_tile_rows(A) - 1) / chain_tile_rows(A);
  const dim3 grid(ntiles > 0 ? ntiles : all - tile0), block(kBlock);
#define PP_SPMV(C)                                                                            \
  do {                                                                                        \
    if (A.sdesc && sizeof(T) == sizeof(float))                                                \
      hipLaunchKernelGGL((k_spmv<T, true, 2, C>), grid, block, 0, stream, A, g, gscale, out,  \
                         tile0);                                                              \
    else if (A.sdesc)                                                                         \
      hipLaunchKernelGGL((k_spmv<T, true, 1, C>), grid, block, 0, stream, A, g, gscale, out,  \
                         tile0);                                                              \
    else                                                                                      \
      hipLaunchKernelGGL((k_spmv<T, false, 1, C>), grid, block, 0, stream, A, g, gscale, out, \
                         tile0);                                                              \
  } while (0)
  if (cached) PP_SPMV(true);
  else PP_SPMV(false);
#undef PP_SPMV
  return hipGetLastError();
}

namespace {
// bad[0] = 1 if the CSR structure is malformed: row_ptr not starting at 0, not
// ending at nnz or decreasing, or a column index outside [0, n).  Only the rows
// whose bounds are valid have their columns read, so every access stays inside
// row_ptr[n + 1] and col_ind[nnz].
__global__ __launch_bounds__(kBlock) void k_check_csr(int n, int nnz,
                                                      const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci,
                                                      int32_t *bad) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int lo = rp[i], hi = rp[i + 1];
  bool ok = lo >= 0 && hi >= lo && hi <= nnz;
  if (i == 0) ok = ok && lo == 0;
  if (i == n - 1) ok = ok && hi == nnz;
  if (ok) {
    for (int p = lo; p < hi; ++p) {
      const int c = ci[p];
      ok = ok && c >= 0 && c < n;
    }
  }
  if (!ok) atomicOr(bad, 1);
}

// Largest |column - row| of the matrix into *out (zeroed by the caller).  A
// workgroup takes tiles of 256 rows in turn: their row pointers go to LDS, its
// threads stride over the tile's nonzeros (coalesced column loads) and find each
// one's row by binary search in LDS.  The workgroup's maximum reaches *out in one
// atomic: same-address atomics are serviced one at a time, and one per wavefront
// over 256^3 rows (262,144 of them) took 3 ms.
__global__ __launch_bounds__(kBlock) void k_bandwidth(int n, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci,
                                                      int32_t *out) {
  __shared__ int32_t s_rp[kBlock + 1];
  __shared__ int32_t s_w[kBlock / 64];
  const int ntiles = (n + kBlock - 1) / kBlock;
  int w = 0;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int r0 = tile * kBlock;
    const int rows = min(kBlock, n - r0);
    __syncthreads();  // the previous tile's searches are done with s_rp
    for (int k = threadIdx.x; k <= rows; k += kBlock) s_rp[k] = rp[r0 + k];
    __syncthreads();
    const int k0 = s_rp[0], k1 = s_rp[rows];
    for (int k = k0 + (int)threadIdx.x; k < k1; k += kBlock) {
      // the row holding nonzero k: the last r with s_rp[r] <= k
      int lo = 0, hi = rows - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_rp[mid] <= k) lo = mid;
        else hi = mid - 1;
      }
      w = max(w, abs(ci[k] - (r0 + lo)));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) w = max(w, __shfl_xor(w, off, 64));
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int m = max(max(s_w[0], s_w[1]), max(s_w[2], s_w[3]));
    if (m > 0) atomicMax(out, m);
  }
}
}  // namespace

hipError_t launch_check_csr(int n, int nnz, const int32_t *rp, const int32_t *ci, int32_t *bad,
                            hipStream_t stream) {
  hipLaunchKernelGGL(k_check_csr, dim3(tiles_of(n)), dim3(kBlock), 0, stream, n, nnz, rp, ci, bad);
  return hipGetLastError();
}

hipError_t launch_bandwidth(int n, const int32_t *rp, const int32_t *ci, int32_t *out,
                            hipStream_t stream) {
  const unsigned g = (unsigned)std::min<int64_t>(tiles_of(n), 1024);
  hipLaunchKernelGGL(k_bandwidth, dim3(g), dim3(kBlock), 0, stream, n, rp, ci, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_residual(const SpMat<T> &A, const T *b, const T *x, T *out, double *partial,
                           int *ntiles, hipStream_t stream) {
  *ntiles = tiles_of(A.n);
  if (A.sdesc)
    hipLaunchKernelGGL((k_residual<T, true>), dim3(*ntiles), dim3(kBlock), 0, stream, A, b, x,
                       out, partial);
  else
    hipLaunchKernelGGL((k_residual<T, false>), dim3(*ntiles), dim3(kBlock), 0, stream, A, b, x,
                       out, partial);
  return hipGetLastError();
}

int orth_grid(int n, int rpt) {
  const int64_t per = (int64_t)kBlock * rpt;
  return (int)((n + per - 1) / per);
}

// Column-count buckets of the CGS2 kernels: steps of 4 columns, so a sweep loads
// at most 3 columns beyond its nc (those re-read column nc - 1 and are multiplied
// by a zero coefficient) and holds no more registers than its bucket needs.
#define PP_NCB_CASE(B, CALL) \
  case (B) / 4:              \
    CALL(B);                 \
    break
#define PP_NCB_SWITCH(nc, CALL)   \
  do {                            \
    switch (((nc) + 3) / 4) {     \
      PP_NCB_CASE(4, CALL);       \
      PP_NCB_CASE(8, CALL);       \
      PP_NCB_CASE(12, CALL);      \
      PP_NCB_CASE(16, CALL);      \
      PP_NCB_CASE(20, CALL);      \
      PP_NCB_CASE(24, CALL);      \
      PP_NCB_CASE(28, CALL);      \
      PP_NCB_CASE(32, CALL);      \
      PP_NCB_CASE(36, CALL);      \
      PP_NCB_CASE(40, CALL);      \
      PP_NCB_CASE(44, CALL);      \
      PP_NCB_CASE(48, CALL);      \
      PP_NCB_CASE(52, CALL);      \
      PP_NCB_CASE(56, CALL);      \
      PP_NCB_CASE(60, CALL);      \
      default:                    \
        CALL(64);                 \
        break;                    \
    }                             \
  } while (0)

template <typename T>
hipError_t launch_dots(int n, int rpt, const T *V, int64_t ldv, int c0, int nc, const T *w,
                       double *partial, hipStream_t stream, const FoldOut *fold, bool cached) {
  if (nc < 1 || nc > kMaxCols || rpt < 1) return hipErrorInvalidValue;
  const int G = orth_grid(n, rpt);
  if (fold && (G > kFoldMaxG || !fold->counter || !fold->h)) return hipErrorInvalidValue;
  const FoldOut f = fold ? *fold : FoldOut{};
  // a folded sweep always runs with ordinary loads (it only serves small sweeps)
#define PP_DOTS_CALL(NCB)                                                                      \
  do {                                                                                         \
    if (fold)                                                                                  \
      hipLaunchKernelGGL((k_dots<T, NCB, true, true>), dim3(G), dim3(kBlock), 0, stream, n,    \
                         rpt, V, ldv, c0, nc, w, partial, f);                                  \
    else if (cached)                                                                           \
      hipLaunchKernelGGL((k_dots<T, NCB, false, true>), dim3(G), dim3(kBlock), 0, stream, n,   \
                         rpt, V, ldv, c0, nc, w, partial, f);                                  \
    else                                                                                       \
      hipLaunchKernelGGL((k_dots<T, NCB, false, false>), dim3(G), dim3(kBlock), 0, stream, n,  \
                         rpt, V, ldv, c0, nc, w, partial, f);                                  \
  } while (0)
  PP_NCB_SWITCH(nc, PP_DOTS_CALL);
#undef PP_DOTS_CALL
  return hipGetLastError();
}

template <typename T, bool DOTS, bool NORM, bool FOLD, bool KEEP>
static void update_dispatch(int n, int rpt, const T *V, int64_t ldv, int nc, const double *ca,
                            const double *cb, double sign, const T *w_in, T *out, double *partial,
                            hipStream_t stream, const FoldOut &f) {
  const int G = orth_grid(n, rpt);
#define PP_UPD_CALL(NCB)                                                                        \
  hipLaunchKernelGGL((k_update<T, NCB, DOTS, NORM, FOLD, KEEP>), dim3(G), dim3(kBlock), 0,        \
                     stream, n, rpt, V, ldv, nc, ca, cb, sign, w_in, out, partial, f)
  PP_NCB_SWITCH(nc, PP_UPD_CALL);
#undef PP_UPD_CALL
}

// The sweep kind's instance: folded (always with ordinary loads and stores), or
// separate with ordinary (cached) or non-temporal ones.
template <typename T, bool DOTS, bool NORM>
static void update_mode(int n, int rpt, const T *V, int64_t ldv, int nc, const double *ca,
                        const double *cb, double sign, const T *w_in, T *out, double *partial,
                        hipStream_t stream, const FoldOut *fold, bool cached) {
  const FoldOut f = fold ? *fold : FoldOut{};
  if constexpr (DOTS || NORM) {
    if (fold) {
      update_dispatch<T, DOTS, NORM, true, true>(n, rpt, V, ldv, nc, ca, cb, sign, w_in, out,
                                                 partial, stream, f);
      return;
    }
  }
  if (cached)
    update_dispatch<T, DOTS, NORM, false, true>(n, rpt, V, ldv, nc, ca, cb, sign, w_in, out,
                                                partial, stream, f);
  else
    update_dispatch<T, DOTS, NORM, false, false>(n, rpt, V, ldv, nc, ca, cb, sign, w_in, out,
                                                 partial, stream, f);
}

template <typename T>
hipError_t launch_update(int n, int rpt, const T *V, int64_t ldv, int nc, const double *coef_a,
                         const double *coef_b, double sign, const T *w_in, T *out, bool dots,
                         bool norm, double *partial, hipStream_t stream, const FoldOut *fold,
                         bool cached) {
  if (nc < 1 || nc > kMaxCols || (dots && norm) || rpt < 1) return hipErrorInvalidValue;
  if (fold && (!(dots || norm) || orth_grid(n, rpt) > kFoldMaxG || !fold->counter ||
               (dots ? !fold->h : !fold->nrm)))
    return hipErrorInvalidValue;
  if (dots)
    update_mode<T, true, false>(n, rpt, V, ldv, nc, coef_a, coef_b, sign, w_in, out, partial,
                                stream, fold, cached);
  else if (norm)
    update_mode<T, false, true>(n, rpt, V, ldv, nc, coef_a, coef_b, sign, w_in, out, partial,
                                stream, fold, cached);
  else
    update_mode<T, false, false>(n, rpt, V, ldv, nc, coef_a, coef_b, sign, w_in, out, partial,
                                 stream, fold, cached);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_norm2(int n, int rpt, const T *x, const double *scale, float *out32,
                        double *partial, hipStream_t stream) {
  if (rpt < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_norm2<T>), dim3(orth_grid(n, rpt)), dim3(kBlock), 0, stream, n, rpt, x,
                     scale, out32, partial);
  return hipGetLastError();
}

hipError_t launch_reduce_cols(const double *partial, int G, int c0, int nc, const double *colscale,
                              double *h, double *coef, hipStream_t stream) {
  hipLaunchKernelGGL(k_reduce_cols, dim3(nc), dim3(kBlock), 0, stream, partial, G, c0, colscale, h,
                     coef);
  return hipGetLastError();
}

hipError_t launch_reduce_norm(const double *partial, int G, double *nrm, double *inv,
                              hipStream_t stream, const double *copy_src, double *copy_dst,
                              int copy_n, int nrm_at) {
  if (copy_dst && (!copy_src || nrm_at < 0 || nrm_at >= copy_n)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_norm, dim3(1), dim3(kBlock), 0, stream, partial, G, nrm, inv,
                     copy_src, copy_dst, copy_n, nrm_at);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(int64_t n, T value, T *x, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_fill<T>), dim3(blocks_of(n)), dim3(kBlock), 0, stream, n, value, x);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_axpy_f64(int n, const double *alpha_dev, const T *d, double *x,
                           hipStream_t stream) {
  hipLaunchKernelGGL((k_axpy_f64<T>), dim3(blocks_of(n)), dim3(kBlock), 0, stream, n, alpha_dev,
                     d, x);
  return hipGetLastError();
}

hipError_t launch_cast_f32(int64_t n, const double *in, float *out, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast_f32, dim3(blocks_of(n)), dim3(kBlock), 0, stream, n, in, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy_from_f64(int n, const double *in, T *out, hipStream_t stream) {
  hipLaunchKernelGGL((k_copy_from_f64<T>), dim3(blocks_of(n)), dim3(kBlock), 0, stream, n, in,
                     out);
  return hipGetLastError();
}

hipError_t launch_count_cols(int nnz, const int32_t *ci, int32_t *cnt, hipStream_t stream) {
  if (nnz <= 0) return hipSuccess;
  unsigned g = blocks_of(nnz);
  if (g > 65536u) g = 65536u;
  hipLaunchKernelGGL(k_count_cols, dim3(g), dim3(kBlock), 0, stream, nnz, ci, cnt);
  return hipGetLastError();
}

int64_t scan_tmp_size(int n) { return (n + kScanPerBlock - 1) / kScanPerBlock + 1; }

hipError_t launch_exclusive_scan(int n, const int32_t *in, int32_t *out, int32_t *tmp,
                                 hipStream_t stream) {
  const int nch = (n + kScanPerBlock - 1) / kScanPerBlock;
  if (nch > 0) {
    hipLaunchKernelGGL(k_scan_chunks, dim3(nch), dim3(kBlock), 0, stream, n, in, out, tmp);
    hipLaunchKernelGGL(k_scan_tops, dim3(1), dim3(kBlock), 0, stream, nch, tmp);
  }
  hipLaunchKernelGGL(k_scan_add, dim3(n > 0 ? blocks_of(n) : 1), dim3(kBlock), 0, stream, n, out,
                     tmp);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scatter_transpose(int n, const int32_t *rp, const int32_t *ci, const T *va,
                                    const int32_t *rp_t, int32_t *cursor, int32_t *ci_t, T *va_t,
                                    int32_t *src_t, hipStream_t stream) {
  hipLaunchKernelGGL((k_scatter_transpose<T>), dim3(blocks_of(n)), dim3(kBlock), 0, stream, n, rp,
                     ci, va, rp_t, cursor, ci_t, va_t, src_t);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sort_rows(int n, const int32_t *rp, int32_t *ci, T *va, int32_t *src,
                            hipStream_t stream) {
  hipLaunchKernelGGL((k_sort_rows<T>), dim3(blocks_of(n)), dim3(kBlock), 0, stream, n, rp, ci, va,
                     src);
  return hipGetLastError();
}

hipError_t launch_csr_grad(int n, const int32_t *rp, const int32_t *ci, const double *lam,
                           const double *x, double *g, hipStream_t stream) {
  hipLaunchKernelGGL(k_csr_grad, dim3(blocks_of(n)), dim3(kBlock), 0, stream, n, rp, ci, lam, x,
                     g);
  return hipGetLastError();
}

hipError_t launch_slice_plan(int n, int ns, const int32_t *rp, const int32_t *ci, int32_t *wlen,
                             int32_t *flag, int32_t *wrow, int32_t *stat, hipStream_t stream) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slice_plan, dim3(blocks_of((int64_t)ns * kSlice)), dim3(kBlock), 0, stream,
                     n, ns, rp, ci, wlen, flag, wrow);
  hipLaunchKernelGGL(k_slice_stats, dim3(1), dim3(1024), 0, stream, ns, wlen, flag, wrow, stat);
  return hipGetLastError();
}

hipError_t launch_slice_fill_idx(int n, int ns, int dmax, const int32_t *rp, const int32_t *ci,
                                 const int32_t *sp, const int32_t *flag, int32_t *sdesc,
                                 int32_t *soff, int32_t *sci, hipStream_t stream) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slice_fill_idx, dim3(blocks_of((int64_t)ns * kSlice)), dim3(kBlock), 0,
                     stream, n, ns, dmax, rp, ci, sp, flag, sdesc, soff, sci);
  return hipGetLastError();
}

template <typename S, typename D>
hipError_t launch_slice_fill_vals(int n, int ns, const int32_t *rp, const int32_t *ci, const S *va,
                                  const int32_t *sp, const int32_t *flag, D *sva,
                                  hipStream_t stream) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_slice_fill_vals<S, D>), dim3(blocks_of((int64_t)ns * kSlice)),
                     dim3(kBlock), 0, stream, n, ns, rp, ci, va, sp, flag, sva);
  return hipGetLastError();
}

template hipError_t launch_slice_fill_vals<double, double>(int, int, const int32_t *,
                                                           const int32_t *, const double *,
                                                           const int32_t *, const int32_t *,
                                                           double *, hipStream_t);
template hipError_t launch_slice_fill_vals<double, float>(int, int, const int32_t *,
                                                          const int32_t *, const double *,
                                                          const int32_t *, const int32_t *,
                                                          float *, hipStream_t);
template hipError_t launch_slice_fill_vals<float, float>(int, int, const int32_t *,
                                                         const int32_t *, const float *,
                                                         const int32_t *, const int32_t *, float *,
                                                         hipStream_t);

// ------------------------------------------------- seeded start vector
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): ten rounds over a 256-bit counter with a 128-bit
// key; each round multiplies words 0 and 2 by fixed constants, swaps the
// products' halves into place XORed with words 1, 3 and the key, and the key
// advances by two Weyl increments between rounds.  Entry i of the vector is
// word i mod 4 of the block at counter floor(i/4) + 1, key (seed, 0), mapped to
// 2 (w >> 11) 2^-53 - 1 (exact in FP64, in [-1, 1)).  One thread per block.
namespace {
__global__ __launch_bounds__(kBlock) void k_uniform_pm1(int64_t n, uint64_t seed,
                                                        double *__restrict__ out) {
  const int64_t blk = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (blk * 4 >= n) return;
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = (uint64_t)blk + 1, x1 = 0, x2 = 0, x3 = 0;
  uint64_t k0 = seed, k1 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(kM0, x0), lo0 = kM0 * x0;
    const uint64_t hi1 = __umul64hi(kM1, x2), lo1 = kM1 * x2;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
    k0 += kW0;
    k1 += kW1;
  }
  const uint64_t w[4] = {x0, x1, x2, x3};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t i = blk * 4 + q;
    if (i < n) out[i] = 2.0 * ((double)(w[q] >> 11) * 0x1.0p-53) - 1.0;
  }
}
}  // namespace

hipError_t launch_uniform_pm1(int64_t n, uint64_t seed, double *out, hipStream_t stream) {
  const int64_t blocks = (n + 4 * kBlock - 1) / (4 * kBlock);
  hipLaunchKernelGGL(k_uniform_pm1, dim3((unsigned)blocks), dim3(kBlock), 0, stream, n, seed, out);
  return hipGetLastError();
}

hipError_t launch_jacobi_scale(int n, const int32_t *rp, const int32_t *ci, const double *va,
                               const double *b, double *va_out, double *b_out, int32_t *bad,
                               hipStream_t stream) {
  hipLaunchKernelGGL(k_jacobi_scale, dim3(blocks_of(n)), dim3(kBlock), 0, stream, n, rp, ci, va, b,
                     va_out, b_out, bad);
  return hipGetLastError();
}

// explicit instantiations
#define PP_INST(T)                                                                              \
  template hipError_t launch_chain<T>(const SpMat<T> &, int, bool, bool, const ChainArgs<T> &,    \
                                      hipStream_t);                                             \
  template hipError_t launch_axpy<T>(int, double, const T *, const double *, const T *, T *,    \
                                     hipStream_t);                                              \
  template hipError_t launch_spmv<T>(const SpMat<T> &, const T *, const double *, T *,           \
                                     hipStream_t, int, int, bool);                              \
  template hipError_t launch_residual<T>(const SpMat<T> &, const T *, const T *, T *, double *,  \
                                         int *, hipStream_t);                                   \
  template hipError_t launch_dots<T>(int, int, const T *, int64_t, int, int, const T *, double *, \
                                     hipStream_t, const FoldOut *, bool);                       \
  template hipError_t launch_update<T>(int, int, const T *, int64_t, int, const double *,       \
                                       const double *, double, const T *, T *, bool, bool,      \
                                       double *, hipStream_t, const FoldOut *, bool);           \
  template hipError_t launch_norm2<T>(int, int, const T *, const double *, float *, double *,   \
                                      hipStream_t);                                             \
  template hipError_t launch_fill<T>(int64_t, T, T *, hipStream_t);                             \
  template hipError_t launch_axpy_f64<T>(int, const double *, const T *, double *,              \
                                         hipStream_t);                                          \
  template hipError_t launch_copy_from_f64<T>(int, const double *, T *, hipStream_t);           \
  template hipError_t launch_scatter_transpose<T>(int, const int32_t *, const int32_t *,        \
                                                  const T *, const int32_t *, int32_t *,        \
                                                  int32_t *, T *, int32_t *, hipStream_t);      \
  template hipError_t launch_sort_rows<T>(int, const int32_t *, int32_t *, T *, int32_t *,      \
                                          hipStream_t);

PP_INST(double)
PP_INST(float)
template hipError_t launch_fill<int32_t>(int64_t, int32_t, int32_t *, hipStream_t);

}  // namespace ppk
