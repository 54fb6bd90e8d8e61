// ILU(0) kernels for gfx950: pattern check, level schedules by frontier
// expansion, the level-scheduled factorisation and triangular sweeps, and the
// elementwise pieces of the composed operator M^-1 A (a chain step with the
// product given, the residual with its norm partials).
//
// The sweeps are bound by the chain of dependent levels, not by bandwidth: each
// level needs the solved values of earlier levels.  Narrow levels therefore run
// back to back inside one workgroup (a barrier between levels, no launch between
// them); a level wider than kRunRows gets its own launch with one thread per row.
// Three run kernels, fastest first: k_sweep_ring (solved values passed through an
// LDS ring, LDS-only barriers, a level's loads issued 4 to 10 levels ahead),
// k_sweep_pipe (two levels ahead, on global memory), and k_forward_run /
// k_backward_run (level-ordered CSR, any row length).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "ilu.h"

namespace ppk {
namespace {

constexpr int kB = 256;

inline unsigned blocks(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

// ------------------------------------------------------------- pattern check
__global__ __launch_bounds__(kB) void k_ilu_check(int n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci,
                                                  int32_t *__restrict__ dpos,
                                                  int32_t *__restrict__ indeg_l,
                                                  int32_t *__restrict__ indeg_u, int32_t *flag) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const int b = rp[i], e = rp[i + 1];
  int d = -1, prev = -1, bad = 0;
  for (int p = b; p < e; ++p) {
    const int c = ci[p];
    if (c <= prev || c >= n) bad |= 1;  // c <= prev also catches c < 0
    if (c == i) d = p;
    prev = c;
  }
  if (d < 0) bad |= 2;
  dpos[i] = d;
  indeg_l[i] = d < 0 ? 0 : d - b;
  indeg_u[i] = d < 0 ? 0 : e - 1 - d;
  if (bad) atomicOr(flag, bad);
}

__global__ __launch_bounds__(kB) void k_scatter_pattern(int n, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci,
                                                        const int32_t *__restrict__ rp_t,
                                                        int32_t *cursor,
                                                        int32_t *__restrict__ rows_t) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    const int j = ci[p];
    rows_t[rp_t[j] + atomicAdd(&cursor[j], 1)] = i;
  }
}

// ------------------------------------------------------------- levels
__global__ __launch_bounds__(kB) void k_level_seed(int n, const int32_t *__restrict__ indeg,
                                                   int32_t *__restrict__ perm, int32_t *lsz) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i < n && indeg[i] == 0) perm[atomicAdd(&lsz[0], 1)] = i;
}

__global__ __launch_bounds__(kB) void k_level_pass(int level, const int32_t *__restrict__ rp_t,
                                                   const int32_t *__restrict__ rows_t, int upper,
                                                   int32_t *indeg, int32_t *perm, int32_t *lbeg,
                                                   int32_t *lsz) {
  const int beg = lbeg[level], cnt = lsz[level];
  const int next = beg + cnt;
  if (blockIdx.x == 0 && threadIdx.x == 0) lbeg[level + 1] = next;
  for (int t = blockIdx.x * kB + threadIdx.x; t < cnt; t += gridDim.x * kB) {
    const int k = perm[beg + t];
    for (int p = rp_t[k]; p < rp_t[k + 1]; ++p) {
      const int i = rows_t[p];
      if (upper ? (i < k) : (i > k)) {
        if (atomicSub(&indeg[i], 1) == 1) perm[next + atomicAdd(&lsz[level + 1], 1)] = i;
      }
    }
  }
}

// ------------------------------------------------------------- factorisation
// Row i of ILU(0), IKJ order: for each stored l_ik (k ascending) divide by the
// pivot u_kk, then subtract l_ik * u_kj from the stored a_ij with j > k (a merge
// of the two sorted rows).  Rows k < i it reads are final (earlier levels).
__device__ __forceinline__ void ilu0_row(int i, const int32_t *__restrict__ rp,
                                         const int32_t *__restrict__ ci,
                                         const int32_t *__restrict__ dpos, double *lu) {
  const int b = rp[i], d = dpos[i], e = rp[i + 1];
  for (int p = b; p < d; ++p) {
    const int k = ci[p];
    const double lik = lu[p] / lu[dpos[k]];
    lu[p] = lik;
    int q = dpos[k] + 1;
    const int qe = rp[k + 1];
    int r = p + 1;
    while (q < qe && r < e) {
      const int cq = ci[q], cr = ci[r];
      if (cq == cr) {
        lu[r] -= lik * lu[q];
        ++q;
        ++r;
      } else if (cq < cr) {
        ++q;
      } else {
        ++r;
      }
    }
  }
}

__global__ __launch_bounds__(kB) void k_factor_level(const int32_t *__restrict__ row, int q0,
                                                     int cnt, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     const int32_t *__restrict__ dpos,
                                                     double *lu) {
  const int t = blockIdx.x * kB + threadIdx.x;
  if (t < cnt) ilu0_row(row[q0 + t], rp, ci, dpos, lu);
}

__global__ __launch_bounds__(kRunThreads) void k_factor_run(const int32_t *__restrict__ row,
                                                            const int32_t *__restrict__ lbeg,
                                                            int l0, int l1,
                                                            const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ ci,
                                                            const int32_t *__restrict__ dpos,
                                                            double *lu) {
  for (int l = l0; l < l1; ++l) {
    const int q1 = lbeg[l + 1];
    for (int q = lbeg[l] + (int)threadIdx.x; q < q1; q += kRunThreads)
      ilu0_row(row[q], rp, ci, dpos, lu);
    __syncthreads();  // this level's rows are final before the next level reads them
  }
}

__global__ __launch_bounds__(kB) void k_ilu_pivots(int n, int64_t nnz,
                                                   const int32_t *__restrict__ dpos,
                                                   const double *__restrict__ lu, int32_t *flag) {
  int bad = 0;
  const int64_t stride = (int64_t)gridDim.x * kB;
  for (int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x; p < nnz; p += stride)
    if (!isfinite(lu[p])) bad |= 2;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += stride)
    if (lu[dpos[i]] == 0.0) bad |= 1;
  if (bad) atomicOr(flag, bad);
}

// ------------------------------------------------------------- level-ordered factors
__global__ __launch_bounds__(kB) void k_sweep_counts(int n, const int32_t *__restrict__ row,
                                                     const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ dpos, int upper,
                                                     int32_t *__restrict__ cnt, int32_t *wmax) {
  const int q = blockIdx.x * kB + threadIdx.x;
  if (q >= n) return;
  const int i = row[q];
  const int c = upper ? rp[i + 1] - dpos[i] - 1 : dpos[i] - rp[i];
  cnt[q] = c;
  atomicMax(wmax, c);
}

__global__ __launch_bounds__(kB) void k_sweep_ell(int n, int width,
                                                  const int32_t *__restrict__ ptr,
                                                  const int32_t *__restrict__ col,
                                                  const double *__restrict__ val,
                                                  int32_t *__restrict__ ecol,
                                                  double *__restrict__ eval) {
  const int q = blockIdx.x * kB + threadIdx.x;
  if (q >= n) return;
  const int b = ptr[q], e = ptr[q + 1];
  for (int s = 0; s < width; ++s) {
    const bool have = b + s < e;
    ecol[(int64_t)s * n + q] = have ? col[b + s] : -1;
    eval[(int64_t)s * n + q] = have ? val[b + s] : 0.0;
  }
}

__global__ __launch_bounds__(kB) void k_sweep_fill(int n, const int32_t *__restrict__ row,
                                                   const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci,
                                                   const int32_t *__restrict__ dpos,
                                                   const double *__restrict__ lu, int upper,
                                                   const int32_t *__restrict__ ptr,
                                                   int32_t *__restrict__ col,
                                                   double *__restrict__ val,
                                                   double *__restrict__ diag) {
  const int q = blockIdx.x * kB + threadIdx.x;
  if (q >= n) return;
  const int i = row[q];
  const int lo = upper ? dpos[i] + 1 : rp[i];
  const int hi = upper ? rp[i + 1] : dpos[i];
  int e = ptr[q];
  for (int p = lo; p < hi; ++p, ++e) {
    col[e] = ci[p];
    val[e] = lu[p];
  }
  if (upper) diag[q] = lu[dpos[i]];
}

// ------------------------------------------------------------- sweeps
// r and z (z and x) may be the same array: a row reads its own right-hand side
// before writing its solution, and the solutions it reads belong to earlier levels.
__device__ __forceinline__ void forward_row(int q, const int32_t *__restrict__ row,
                                            const int32_t *__restrict__ ptr,
                                            const int32_t *__restrict__ col,
                                            const double *__restrict__ val, const double *r,
                                            double *z) {
  const int i = row[q];
  double acc = r[i];
  const int e1 = ptr[q + 1];
  for (int e = ptr[q]; e < e1; ++e) acc -= val[e] * z[col[e]];
  z[i] = acc;
}

__device__ __forceinline__ void backward_row(int q, const int32_t *__restrict__ row,
                                             const int32_t *__restrict__ ptr,
                                             const int32_t *__restrict__ col,
                                             const double *__restrict__ val,
                                             const double *__restrict__ diag, const double *z,
                                             double *x) {
  const int i = row[q];
  double acc = z[i];
  const int e1 = ptr[q + 1];
  for (int e = ptr[q]; e < e1; ++e) acc -= val[e] * x[col[e]];
  x[i] = acc / diag[q];
}

__global__ __launch_bounds__(kB) void k_forward_level(int q0, int cnt,
                                                      const int32_t *__restrict__ row,
                                                      const int32_t *__restrict__ ptr,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ val,
                                                      const double *r, double *z) {
  const int t = blockIdx.x * kB + threadIdx.x;
  if (t < cnt) forward_row(q0 + t, row, ptr, col, val, r, z);
}

__global__ __launch_bounds__(kRunThreads) void k_forward_run(
    int l0, int l1, const int32_t *__restrict__ lbeg, const int32_t *__restrict__ row,
    const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *r, double *z) {
  for (int l = l0; l < l1; ++l) {
    const int q1 = lbeg[l + 1];
    for (int q = lbeg[l] + (int)threadIdx.x; q < q1; q += kRunThreads)
      forward_row(q, row, ptr, col, val, r, z);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kB) void k_backward_level(int q0, int cnt,
                                                       const int32_t *__restrict__ row,
                                                       const int32_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ col,
                                                       const double *__restrict__ val,
                                                       const double *__restrict__ diag,
                                                       const double *z, double *x) {
  const int t = blockIdx.x * kB + threadIdx.x;
  if (t < cnt) backward_row(q0 + t, row, ptr, col, val, diag, z, x);
}

__global__ __launch_bounds__(kRunThreads) void k_backward_run(
    int l0, int l1, const int32_t *__restrict__ lbeg, const int32_t *__restrict__ row,
    const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ diag, const double *z,
    double *x) {
  for (int l = l0; l < l1; ++l) {
    const int q1 = lbeg[l + 1];
    for (int q = lbeg[l] + (int)threadIdx.x; q < q1; q += kRunThreads)
      backward_row(q, row, ptr, col, val, diag, z, x);
    __syncthreads();
  }
}

// Pipelined run over narrow levels (at most one row per thread per level), on the
// slot-major copy of W slots.  In the iteration of level l a thread issues the
// gathers of level l's solved values, then the right-hand side of its level-(l+1)
// row and the entries of its level-(l+2) row (neither depends on the solve), then
// finishes level l: each level costs one round of memory latency instead of the
// chain row -> entries -> gathers.  BACK: the backward sweep (divides by the
// pivot).  rhs may equal out: a row's right-hand side is read before the row is
// solved, at the level before its own.
constexpr int kLbegChunk = 1024;  // level offsets staged in LDS at a time
static_assert(kRunRows <= kRunThreads, "a run level must fit one row per thread");

template <int W, bool BACK>
__device__ __forceinline__ void load_slots(int q, int n, const int32_t *__restrict__ row,
                                           const int32_t *__restrict__ ecol,
                                           const double *__restrict__ eval,
                                           const double *__restrict__ diag, int &i, int (&c)[W],
                                           double (&v)[W], double &d) {
  i = -1;
  d = 1.0;
#pragma unroll
  for (int s = 0; s < W; ++s) {
    c[s] = -1;
    v[s] = 0.0;
  }
  if (q >= 0) {
    i = row[q];
#pragma unroll
    for (int s = 0; s < W; ++s) {
      c[s] = ecol[(int64_t)s * n + q];
      v[s] = eval[(int64_t)s * n + q];
    }
    if constexpr (BACK) d = diag[q];
  }
}

template <int W, bool BACK>
__global__ __launch_bounds__(kRunThreads) void k_sweep_pipe(
    int l0, int l1, int n, const int32_t *__restrict__ lbeg, const int32_t *__restrict__ row,
    const int32_t *__restrict__ ecol, const double *__restrict__ eval,
    const double *__restrict__ diag, const double *rhs, double *out) {
  __shared__ int32_t s_lb[kLbegChunk + 4];
  const int t = threadIdx.x;
  int base = l0;
  // lbeg[base + k] for k < kLbegChunk + 4 (clamped to the run's last offset)
  auto stage = [&]() {
    for (int k = t; k < kLbegChunk + 4; k += kRunThreads) s_lb[k] = lbeg[min(base + k, l1)];
    __syncthreads();
  };
  auto pos = [&](int l) -> int {  // this thread's position at level l, or -1
    if (l >= l1) return -1;
    const int q = s_lb[l - base] + t;
    return q < s_lb[l - base + 1] ? q : -1;
  };
  stage();
  int i0, i1, c0[W], c1[W];
  double v0[W], v1[W], d0, d1;
  load_slots<W, BACK>(pos(l0), n, row, ecol, eval, diag, i0, c0, v0, d0);
  double r0 = i0 >= 0 ? rhs[i0] : 0.0;
  load_slots<W, BACK>(pos(l0 + 1), n, row, ecol, eval, diag, i1, c1, v1, d1);
  for (int l = l0; l < l1; ++l) {
    if (l - base > kLbegChunk) {  // uniform: every thread restages
      base = l;
      stage();
    }
    double g[W];
#pragma unroll
    for (int s = 0; s < W; ++s) g[s] = (i0 >= 0 && c0[s] >= 0) ? out[c0[s]] : 0.0;
    const double r1 = i1 >= 0 ? rhs[i1] : 0.0;
    int i2, c2[W];
    double v2[W], d2;
    load_slots<W, BACK>(pos(l + 2), n, row, ecol, eval, diag, i2, c2, v2, d2);
    if (i0 >= 0) {
      double acc = r0;
#pragma unroll
      for (int s = 0; s < W; ++s) acc -= v0[s] * g[s];
      out[i0] = BACK ? acc / d0 : acc;
    }
    __syncthreads();  // level l is solved before level l + 1 gathers it
    i0 = i1;
    r0 = r1;
    d0 = d1;
    i1 = i2;
    d1 = d2;
#pragma unroll
    for (int s = 0; s < W; ++s) {
      c0[s] = c1[s];
      v0[s] = v1[s];
      c1[s] = c2[s];
      v1[s] = v2[s];
    }
  }
}

// Level of position q: the last l with lbeg[l] <= q.
__device__ __forceinline__ int level_of(int q, int nlev, const int32_t *__restrict__ lbeg) {
  int lo = 0, hi = nlev - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (lbeg[mid] <= q) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kB) void k_sweep_inverse(int n, const int32_t *__restrict__ row,
                                                      int32_t *__restrict__ qpos) {
  const int q = blockIdx.x * kB + threadIdx.x;
  if (q < n) qpos[row[q]] = q;
}

__global__ __launch_bounds__(kB) void k_sweep_sources(int n, int width, int nlev,
                                                      const int32_t *__restrict__ lbeg,
                                                      const int32_t *__restrict__ ecol,
                                                      const int32_t *__restrict__ qpos,
                                                      const int32_t *__restrict__ runstart,
                                                      int32_t *__restrict__ esrc,
                                                      int32_t *__restrict__ lglob, int32_t *flag) {
  const int q = blockIdx.x * kB + threadIdx.x;
  if (q >= n) return;
  const int lq = level_of(q, nlev, lbeg);
  const int rs = runstart[lq];
  int far = 0, glob = 0;
  for (int s = 0; s < width; ++s) {
    const int64_t e = (int64_t)s * n + q;
    const int c = ecol[e];
    int src = -1;
    if (c >= 0 && rs >= 0) {
      const int qc = qpos[c];
      const int lc = level_of(qc, nlev, lbeg);
      if (lc >= rs) {  // solved inside this run
        if (lq - lc < kRing) src = (lc % kRing) * kRunRows + (qc - lbeg[lc]);
        else far = 1;
      } else {
        glob = 1;  // solved by an earlier launch
      }
    }
    esrc[e] = src;
  }
  if (glob) lglob[lq] = 1;
  if (far) atomicOr(flag, 1);
}

// Registers of one row of a run level (see k_sweep_ring).
template <int W>
struct RingRow {
  bool ok;                          // this thread has a row at the level
  int q;                            // its position
  uint32_t xs[ring_swords(W)];    // packed ring slots
  double v[ring_vstride(W)];      // entries (the last ones padding when W = 3)
  double r;                         // right-hand side in level order
};

template <int W>
__device__ __forceinline__ int ring_slot(const RingRow<W> &R, int s) {
  return (int)(int16_t)(R.xs[s >> 1] >> (16 * (s & 1)));
}

// Values solved by earlier launches, taken out of a run's right-hand side before
// the run starts: rq[q] -= sum of v * out[c] over the entries of position q in
// [q0, q1) whose column was solved before the run (esrc -1 on a real column); v
// is the run's stored entry (divided by the pivot in the backward sweep, like
// rq).  The run kernel then reads solved values from its LDS ring alone.
template <int W>
__global__ __launch_bounds__(kB) void k_ring_glob(int q0, int q1, int n,
                                                  const int32_t *__restrict__ ecol,
                                                  const int32_t *__restrict__ esrc,
                                                  const double *__restrict__ rval,
                                                  const double *__restrict__ out,
                                                  double *__restrict__ rq) {
  const int q = q0 + (int)(blockIdx.x * kB + threadIdx.x);
  if (q >= q1) return;
  double acc = rq[q];
#pragma unroll
  for (int s = 0; s < W; ++s) {
    const int64_t e = (int64_t)s * n + q;
    const int c = ecol[e];
    if (c >= 0 && esrc[e] < 0) acc -= rval[(int64_t)q * ring_vstride(W) + s] * out[c];
  }
  rq[q] = acc;
}

// The pipelined run with the solved values of the last kRing levels in an LDS ring
// (each entry's slot says where its value is; values solved by earlier launches
// are already in the right-hand side, see k_ring_glob).  Everything runs in level
// order: position q's right-hand side rq[q] is replaced by its solution (the
// caller scatters the run's positions to rows afterwards), so every load and
// store of a level is contiguous.  The backward sweep comes here with its rows
// divided by the pivots (entries at set-up, the right-hand side at its gather),
// so both sweeps run the same unit-diagonal step.
// Only LDS is exchanged between the run's waves, so the barrier between levels
// fences LDS alone and the global loads issued ahead stay in flight across it.
// Everything a level needs is loaded D levels ahead into one of D + 1 register
// sets (the loop is unrolled by D + 1, so a prefetched value lands in the register
// that later uses it); no load in the loop is conditional (clamped indices,
// results selected at use), so the wait before a level's arithmetic covers that
// level's loads and no later ones.  The level offsets a load needs are read from
// LDS one level early, in the shadow of the barrier.
template <int W, int D>
__global__ __launch_bounds__(kRunThreads) void k_sweep_ring(
    int l0, int l1, const int32_t *__restrict__ lbeg, const uint32_t *__restrict__ rslot,
    const double *__restrict__ rval, double *rq) {
  constexpr int VS = ring_vstride(W), SW = ring_swords(W);
  // the last slot is never written: the target of ring loads a row does not need
  __shared__ double ring[kRing * kRunRows + 1];
  constexpr int kNoSlot = kRing * kRunRows;
  constexpr int kLbExtra = 2 * D + 4;  // offsets read past the run's last level
  // the run's level offsets, lbeg[l0 + k] (clamped to lbeg[l1]); l1 - l0 <= kRunLevels
  __shared__ int32_t s_lb[kRunLevels + kLbExtra];
  const int t = threadIdx.x;
  // position of this thread at level l from the level's first and next offsets
  auto pos = [&](int l, int b0, int b1) -> int {
    const int q = b0 + t;
    return (l < l1 && q < b1) ? q : -1;
  };
  auto load = [&](int q, RingRow<W> &R) {
    R.ok = q >= 0;
    R.q = R.ok ? q : 0;
    R.r = rq[R.q];
    if constexpr (SW == 1) {
      R.xs[0] = rslot[R.q];
    } else {
      const uint2 w = reinterpret_cast<const uint2 *>(rslot)[R.q];
      R.xs[0] = w.x;
      R.xs[1] = w.y;
    }
    const double *vp = rval + (int64_t)R.q * VS;
    if constexpr (VS == 1) {
      R.v[0] = vp[0];
    } else {
#pragma unroll
      for (int k = 0; k < VS; k += 2) {
        const double2 w = reinterpret_cast<const double2 *>(vp)[k / 2];
        R.v[k] = w.x;
        R.v[k + 1] = w.y;
      }
    }
  };
  // offsets of the level whose loads the next step issues: lbeg[l + D], lbeg[l + D + 1]
  int nb0, nb1;
  // level l: solve S0, fetch level l + D into SD
  auto step = [&](int l, RingRow<W> &S0, RingRow<W> &SD) {
    double g[W];
#pragma unroll
    for (int s = 0; s < W; ++s) {
      const int x = ring_slot(S0, s);
      g[s] = ring[x >= 0 ? x : kNoSlot];
    }
    load(pos(l + D, nb0, nb1), SD);
    double acc = S0.r;
#pragma unroll
    for (int s = 0; s < W; ++s) acc -= S0.v[s] * (ring_slot(S0, s) >= 0 ? g[s] : 0.0);
    // a thread with no row at level l owns no reader of this slot
    ring[(l % kRing) * kRunRows + t] = acc;
    if (S0.ok) rq[S0.q] = acc;
    nb0 = nb1;
    nb1 = s_lb[l + D + 2 - l0];
    // level l's ring slots are written before level l + 1 reads them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  };
  // staged once: no global load in the level loop but the prefetches, whose
  // waits then stay D levels behind
  for (int k = t; k < l1 - l0 + kLbExtra; k += (int)blockDim.x) s_lb[k] = lbeg[min(l0 + k, l1)];
  __syncthreads();
  RingRow<W> R[D + 1];
  // the first D levels' loads are issued level after level, in the loop's order,
  // so the loop's waits (fixed in the code, shared with later iterations) count
  // the loads of D - 1 levels as still in flight
#pragma unroll
  for (int k = 0; k < D; ++k) {
    load(pos(l0 + k, s_lb[k], s_lb[k + 1]), R[k]);
    __builtin_amdgcn_sched_barrier(0);
  }
  nb0 = s_lb[D];
  nb1 = s_lb[D + 1];
  // levels past l1 are empty (no row), so the loop may run up to D of them; a run
  // has a level (l0 < l1), and the loop is entered without a test, which keeps the
  // loads above in the order written
  int l = l0;
  do {
#pragma unroll
    for (int k = 0; k <= D; ++k) step(l + k, R[k], R[(k + D) % (D + 1)]);
    l += D + 1;
  } while (l < l1);
}

// Ring-run data from the slot-major copy: slots packed as 16-bit integers, entries
// per position (divided by the pivot when diag is given: the backward sweep).
template <int W>
__global__ __launch_bounds__(kB) void k_ring_pack(int n, const int32_t *__restrict__ esrc,
                                                  const double *__restrict__ eval,
                                                  const double *__restrict__ diag,
                                                  uint32_t *__restrict__ rslot,
                                                  double *__restrict__ rval) {
  const int q = blockIdx.x * kB + threadIdx.x;
  if (q >= n) return;
  constexpr int VS = ring_vstride(W), SW = ring_swords(W);
  uint32_t w[2] = {0u, 0u};
  const double d = diag ? diag[q] : 1.0;
#pragma unroll
  for (int s = 0; s < VS; ++s) {
    int x = -1;
    double v = 0.0;
    if (s < W) {
      x = esrc[(int64_t)s * n + q];
      v = eval[(int64_t)s * n + q];
      if (x < 0) x = -1;
    }
    if (s < 2 * SW) w[s >> 1] |= (uint32_t)(uint16_t)(int16_t)x << (16 * (s & 1));
    rval[(int64_t)q * VS + s] = diag ? v / d : v;
  }
#pragma unroll
  for (int k = 0; k < SW; ++k) rslot[(int64_t)q * SW + k] = w[k];
}

// Right-hand side of a ring sweep in level order: dst[q] = src[row[q]] (divided by
// the pivot when diag is given).
__global__ __launch_bounds__(kB) void k_gather_ring(int n, const int32_t *__restrict__ row,
                                                    const double *__restrict__ diag,
                                                    const double *__restrict__ src,
                                                    double *__restrict__ dst) {
  const int q = blockIdx.x * kB + threadIdx.x;
  if (q < n) dst[q] = diag ? src[row[q]] / diag[q] : src[row[q]];
}

// A finished run's solutions to their rows: dst[row[q]] = src[q], q in [q0, q1).
__global__ __launch_bounds__(kB) void k_scatter_run(int q0, int q1,
                                                    const int32_t *__restrict__ row,
                                                    const double *__restrict__ src,
                                                    double *__restrict__ dst) {
  const int q = q0 + (int)(blockIdx.x * kB + threadIdx.x);
  if (q < q1) dst[row[q]] = src[q];
}


// ------------------------------------------------------------- composed operator
// The chain step kinds of ChainArgs with (A g)(i) replaced by the given prod(i).
template <int KIND, bool FOLD, bool LAST>
__global__ __launch_bounds__(kB) void k_chain_given(int n, const double *__restrict__ prod,
                                                    ChainArgs<double> a) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  constexpr bool kReadY = (KIND == 0) || (KIND == 1) || (KIND == 2 && (FOLD || LAST)) ||
                          (KIND == 3 && LAST);
  constexpr bool kReadSelf = (KIND == 2) || (KIND == 4);
  const double gs = a.gscale ? *a.gscale : 1.0;
  const double own = a.g[i];
  const double yv = (kReadY && a.y_in) ? a.y_in[i] : 0.0;
  const double sf = kReadSelf ? a.self[i] : 0.0;
  const double acc = prod[i];
  const double c1 = a.c1, c2 = a.c2, cf = a.cf;
  if constexpr (KIND == 0) {
    const double p = gs * own;
    double y = yv + c1 * p;
    const double pn = p - c1 * (gs * acc);
    if constexpr (FOLD) {
      y += cf * pn;
    } else {
      a.out[i] = pn;
    }
    a.y_out[i] = y;
  } else if constexpr (KIND == 1) {
    const double tt = gs * acc;
    a.y_out[i] = yv + c1 * (gs * own) - c2 * tt;
    if constexpr (!LAST) a.out[i] = tt;
  } else if constexpr (KIND == 2) {
    const double ss = a.sscale ? *a.sscale : 1.0;
    const double pn = ss * sf - c1 * (gs * own) + c2 * (gs * acc);
    if constexpr (FOLD) {
      a.y_out[i] = yv + cf * pn;
    } else if constexpr (LAST) {
      const double ys = a.yscale ? *a.yscale : 1.0;
      a.out[i] = ys * yv - pn;
    } else {
      a.out[i] = pn;
    }
  } else if constexpr (KIND == 4) {
    const double ss = a.sscale ? *a.sscale : 1.0;
    a.out[i] = c2 * (gs * acc) + c1 * (ss * sf);
  } else {
    const double pn = gs * own - c1 * (gs * acc);
    if constexpr (LAST) {
      const double ys = a.yscale ? *a.yscale : 1.0;
      a.out[i] = ys * yv - pn;
    } else {
      a.out[i] = pn;
    }
  }
}

__global__ __launch_bounds__(kB) void k_sub_norm(int n, const double *__restrict__ b,
                                                 const double *__restrict__ y,
                                                 double *__restrict__ out,
                                                 double *__restrict__ partial) {
  __shared__ double red[kB / 64];
  const int i = blockIdx.x * kB + threadIdx.x;
  double sq = 0.0;
  if (i < n) {
    const double r = b[i] - y[i];
    out[i] = r;
    sq = r * r;
  }
  for (int off = 32; off > 0; off >>= 1) sq += __shfl_down(sq, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kB / 64; ++w) s += red[w];
    partial[blockIdx.x] = s;
  }
}

}  // namespace

// ------------------------------------------------------------- wrappers
hipError_t launch_ilu_check(int n, const int32_t *rp, const int32_t *ci, int32_t *dpos,
                            int32_t *indeg_l, int32_t *indeg_u, int32_t *flag,
                            hipStream_t stream) {
  hipLaunchKernelGGL(k_ilu_check, dim3(blocks(n)), dim3(kB), 0, stream, n, rp, ci, dpos, indeg_l,
                     indeg_u, flag);
  return hipGetLastError();
}

hipError_t launch_scatter_pattern(int n, const int32_t *rp, const int32_t *ci,
                                  const int32_t *rp_t, int32_t *cursor, int32_t *rows_t,
                                  hipStream_t stream) {
  hipLaunchKernelGGL(k_scatter_pattern, dim3(blocks(n)), dim3(kB), 0, stream, n, rp, ci, rp_t,
                     cursor, rows_t);
  return hipGetLastError();
}

hipError_t launch_level_seed(int n, const int32_t *indeg, int32_t *perm, int32_t *lsz,
                             hipStream_t stream) {
  hipLaunchKernelGGL(k_level_seed, dim3(blocks(n)), dim3(kB), 0, stream, n, indeg, perm, lsz);
  return hipGetLastError();
}

hipError_t launch_level_pass(int level, const int32_t *rp_t, const int32_t *rows_t, bool upper,
                             int32_t *indeg, int32_t *perm, int32_t *lbeg, int32_t *lsz,
                             hipStream_t stream) {
  // a fixed grid that strides over the frontier, whose size only the device knows
  hipLaunchKernelGGL(k_level_pass, dim3(512), dim3(kB), 0, stream, level, rp_t, rows_t,
                     upper ? 1 : 0, indeg, perm, lbeg, lsz);
  return hipGetLastError();
}

hipError_t launch_ilu_factor(const Sweep &L, const int32_t *rp, const int32_t *ci,
                             const int32_t *dpos, double *lu, hipStream_t stream) {
  for (const LevelSpan &sp : L.spans) {
    if (sp.run) {
      hipLaunchKernelGGL(k_factor_run, dim3(1), dim3(kRunThreads), 0, stream, L.row, L.lbeg,
                         sp.l0, sp.l1, rp, ci, dpos, lu);
    } else {
      const int q0 = L.lbeg_host[sp.l0], cnt = L.lbeg_host[sp.l0 + 1] - q0;
      hipLaunchKernelGGL(k_factor_level, dim3(blocks(cnt)), dim3(kB), 0, stream, L.row, q0, cnt,
                         rp, ci, dpos, lu);
    }
  }
  return hipGetLastError();
}

hipError_t launch_ilu_pivots(int n, int64_t nnz, const int32_t *dpos, const double *lu,
                             int32_t *flag, hipStream_t stream) {
  const unsigned g = (unsigned)std::min<int64_t>(blocks(std::max<int64_t>(n, nnz)), 4096);
  hipLaunchKernelGGL(k_ilu_pivots, dim3(g), dim3(kB), 0, stream, n, nnz, dpos, lu, flag);
  return hipGetLastError();
}

hipError_t launch_sweep_counts(int n, const int32_t *row, const int32_t *rp,
                               const int32_t *dpos, bool upper, int32_t *cnt, int32_t *wmax,
                               hipStream_t stream) {
  hipLaunchKernelGGL(k_sweep_counts, dim3(blocks(n)), dim3(kB), 0, stream, n, row, rp, dpos,
                     upper ? 1 : 0, cnt, wmax);
  return hipGetLastError();
}

hipError_t launch_sweep_ell(int n, int width, const int32_t *ptr, const int32_t *col,
                            const double *val, int32_t *ecol, double *eval, hipStream_t stream) {
  hipLaunchKernelGGL(k_sweep_ell, dim3(blocks(n)), dim3(kB), 0, stream, n, width, ptr, col, val,
                     ecol, eval);
  return hipGetLastError();
}

hipError_t launch_sweep_inverse(int n, const int32_t *row, int32_t *qpos, hipStream_t stream) {
  hipLaunchKernelGGL(k_sweep_inverse, dim3(blocks(n)), dim3(kB), 0, stream, n, row, qpos);
  return hipGetLastError();
}

hipError_t launch_sweep_sources(int n, int width, int nlev, const int32_t *lbeg,
                                const int32_t *ecol, const int32_t *qpos,
                                const int32_t *runstart, int32_t *esrc, int32_t *lglob,
                                int32_t *flag, hipStream_t stream) {
  hipLaunchKernelGGL(k_sweep_sources, dim3(blocks(n)), dim3(kB), 0, stream, n, width, nlev,
                     lbeg, ecol, qpos, runstart, esrc, lglob, flag);
  return hipGetLastError();
}

// Levels a ring run loads ahead of the one it solves: a level takes a fraction of
// the latency of a load that misses the L2, so as many as the registers allow
// (D + 1 register sets, 4 wavefronts a SIMD at 1024 threads: 128 VGPRs).
template <int W>
constexpr int ring_ahead() {
  return W <= 1 ? 10 : W == 2 ? 7 : W == 3 ? 5 : 4;
}

// One LDS-ring run: the values it waits for from earlier launches out of its
// right-hand side, the run in level order on work, its solutions to their rows.
template <int W>
static void launch_ring(const Sweep &S, const LevelSpan &sp, int n, double *work, double *out,
                        hipStream_t stream) {
  const int q0 = S.lbeg_host[sp.l0], q1 = S.lbeg_host[sp.l1];
  if (sp.glob)
    hipLaunchKernelGGL((k_ring_glob<W>), dim3(blocks(q1 - q0)), dim3(kB), 0, stream, q0, q1, n,
                       S.ecol, S.esrc, S.rval, out, work);
  hipLaunchKernelGGL((k_sweep_ring<W, ring_ahead<W>()>), dim3(1),
                     dim3((sp.width + 63) / 64 * 64), 0, stream, sp.l0, sp.l1, S.lbeg, S.rslot,
                     S.rval, work);
  hipLaunchKernelGGL(k_scatter_run, dim3(blocks(q1 - q0)), dim3(kB), 0, stream, q0, q1, S.row,
                     work, out);
}

// A run of a sweep with a slot-major copy: LDS-ring runs when the sweep has their
// data (work: the right-hand side in level order), else the pipelined run on
// global memory for the sweep's slot count (1..kPipeSlots).
template <bool BACK>
static void launch_slot_run(const Sweep &S, const LevelSpan &sp, int n, const double *rhs,
                            double *work, double *out, hipStream_t stream) {
  if (S.rslot && sp.l1 - sp.l0 <= kRunLevels) {  // (make_spans keeps every run that short)
    switch (S.width) {
      case 1: launch_ring<1>(S, sp, n, work, out, stream); break;
      case 2: launch_ring<2>(S, sp, n, work, out, stream); break;
      case 3: launch_ring<3>(S, sp, n, work, out, stream); break;
      default: launch_ring<4>(S, sp, n, work, out, stream); break;
    }
    return;
  }
#define PP_PIPE(W)                                                                               \
  hipLaunchKernelGGL((k_sweep_pipe<W, BACK>), dim3(1), dim3(kRunThreads), 0, stream, sp.l0,      \
                     sp.l1, n, S.lbeg, S.row, S.ecol, S.eval, S.diag, rhs, out)
  switch (S.width) {
    case 1: PP_PIPE(1); break;
    case 2: PP_PIPE(2); break;
    case 3: PP_PIPE(3); break;
    case 4: PP_PIPE(4); break;
    case 5: PP_PIPE(5); break;
    case 6: PP_PIPE(6); break;
    case 7: PP_PIPE(7); break;
    default: PP_PIPE(8); break;
  }
#undef PP_PIPE
}

hipError_t launch_ring_pack(int n, int width, const int32_t *esrc, const double *eval,
                            const double *diag, uint32_t *rslot, double *rval,
                            hipStream_t stream) {
#define PP_PACK(W)                                                                           \
  hipLaunchKernelGGL((k_ring_pack<W>), dim3(blocks(n)), dim3(kB), 0, stream, n, esrc, eval, \
                     diag, rslot, rval)
  switch (width) {
    case 1: PP_PACK(1); break;
    case 2: PP_PACK(2); break;
    case 3: PP_PACK(3); break;
    case 4: PP_PACK(4); break;
    default: return hipErrorInvalidValue;
  }
#undef PP_PACK
  return hipGetLastError();
}

hipError_t launch_sweep_fill(int n, const int32_t *row, const int32_t *rp, const int32_t *ci,
                             const int32_t *dpos, const double *lu, bool upper,
                             const int32_t *ptr, int32_t *col, double *val, double *diag,
                             hipStream_t stream) {
  hipLaunchKernelGGL(k_sweep_fill, dim3(blocks(n)), dim3(kB), 0, stream, n, row, rp, ci, dpos,
                     lu, upper ? 1 : 0, ptr, col, val, diag);
  return hipGetLastError();
}

hipError_t launch_ilu_forward(int n, const Sweep &L, const double *r, double *z, double *work,
                              hipStream_t stream) {
  if (L.rslot)
    hipLaunchKernelGGL(k_gather_ring, dim3(blocks(n)), dim3(kB), 0, stream, n, L.row, nullptr, r,
                       work);
  for (const LevelSpan &sp : L.spans) {
    if (sp.run && L.ecol) {
      launch_slot_run<false>(L, sp, n, r, work, z, stream);
    } else if (sp.run) {
      hipLaunchKernelGGL(k_forward_run, dim3(1), dim3(kRunThreads), 0, stream, sp.l0, sp.l1,
                         L.lbeg, L.row, L.ptr, L.col, L.val, r, z);
    } else {
      const int q0 = L.lbeg_host[sp.l0], cnt = L.lbeg_host[sp.l0 + 1] - q0;
      hipLaunchKernelGGL(k_forward_level, dim3(blocks(cnt)), dim3(kB), 0, stream, q0, cnt, L.row,
                         L.ptr, L.col, L.val, r, z);
    }
  }
  return hipGetLastError();
}

hipError_t launch_ilu_backward(int n, const Sweep &U, const double *z, double *x, double *work,
                               hipStream_t stream) {
  if (U.rslot)  // the right-hand side in level order, divided by the pivots
    hipLaunchKernelGGL(k_gather_ring, dim3(blocks(n)), dim3(kB), 0, stream, n, U.row, U.diag, z,
                       work);
  for (const LevelSpan &sp : U.spans) {
    if (sp.run && U.ecol) {
      launch_slot_run<true>(U, sp, n, z, work, x, stream);
    } else if (sp.run) {
      hipLaunchKernelGGL(k_backward_run, dim3(1), dim3(kRunThreads), 0, stream, sp.l0, sp.l1,
                         U.lbeg, U.row, U.ptr, U.col, U.val, U.diag, z, x);
    } else {
      const int q0 = U.lbeg_host[sp.l0], cnt = U.lbeg_host[sp.l0 + 1] - q0;
      hipLaunchKernelGGL(k_backward_level, dim3(blocks(cnt)), dim3(kB), 0, stream, q0, cnt,
                         U.row, U.ptr, U.col, U.val, U.diag, z, x);
    }
  }
  return hipGetLastError();
}

hipError_t launch_chain_given(int n, int kind, bool fold, bool last, const double *prod,
                              const ChainArgs<double> &a, hipStream_t stream) {
  const dim3 grid(blocks(n)), block(kB);
#define PP_GIVEN(K, F, L) \
  hipLaunchKernelGGL((k_chain_given<K, F, L>), grid, block, 0, stream, n, prod, a)
  switch (kind) {
    case 0:
      if (fold) PP_GIVEN(0, true, false); else PP_GIVEN(0, false, false);
      break;
    case 1:
      if (last) PP_GIVEN(1, false, true); else PP_GIVEN(1, false, false);
      break;
    case 2:
      if (fold) PP_GIVEN(2, true, false);
      else if (last) PP_GIVEN(2, false, true);
      else PP_GIVEN(2, false, false);
      break;
    case 3:
      if (last) PP_GIVEN(3, false, true); else PP_GIVEN(3, false, false);
      break;
    case 4:
      PP_GIVEN(4, false, false);
      break;
    default:
      return hipErrorInvalidValue;
  }
#undef PP_GIVEN
  return hipGetLastError();
}

hipError_t launch_sub_norm(int n, const double *b, const double *y, double *out,
                           double *partial, int *ntiles, hipStream_t stream) {
  *ntiles = (int)blocks(n);
  hipLaunchKernelGGL(k_sub_norm, dim3(*ntiles), dim3(kB), 0, stream, n, b, y, out, partial);
  return hipGetLastError();
}

}  // namespace ppk
