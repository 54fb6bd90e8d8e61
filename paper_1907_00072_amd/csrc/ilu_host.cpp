// ILU(0) factor object: the device factorisation, its level schedules, the
// level-ordered copies of L and U, and the pp_ilu0_* entry points of include/pp.h.
//
// Every O(nnz) step runs on the device (ilu.hip); the host only steps the level
// loop (reading the frontier sizes back every kLevelBatch levels) and turns the
// level offsets into launch spans.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <new>
#include <vector>

#include "../../include/pp.h"
#include "diag.h"
#include "ilu.h"
#include "kernels.h"

namespace {

using ppk::LevelSpan;
using ppk::Sweep;

// Frontier passes launched between two reads of the level sizes.
constexpr int kLevelBatch = 32;

#define ILU_TRY_HIP(expr) PPD_TRY_HIP(expr, PP_ERR_HIP)
#define ILU_TRY(expr)            \
  do {                           \
    int r_ = (expr);             \
    if (r_ < 0) return r_;       \
  } while (0)

// Device allocations released together (the factor's own, or a call's temporaries).
struct Allocs {
  std::vector<void *> ptrs;
  template <typename T>
  int take(T **p, int64_t count) {
    void *q = nullptr;
    const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    if (hipMalloc(&q, bytes) != hipSuccess) return PP_ERR_NOMEM;
    ptrs.push_back(q);
    *p = static_cast<T *>(q);
    return PP_OK;
  }
  void release() {
    for (void *q : ptrs) (void)hipFree(q);
    ptrs.clear();
  }
  ~Allocs() { release(); }
};

void free_ilu(pp_ilu *M) {
  if (!M) return;
  for (void *q : M->owned) (void)hipFree(q);
  delete M;
}

// Launch spans of a level schedule: consecutive levels of at most kRunRows rows
// share one run of at most kRunLevels levels; a wider level is a span of its own.
std::vector<LevelSpan> make_spans(const std::vector<int32_t> &lbeg) {
  std::vector<LevelSpan> spans;
  const int nlev = (int)lbeg.size() - 1;
  for (int l = 0; l < nlev; ++l) {
    const int rows = lbeg[l + 1] - lbeg[l];
    const bool narrow = rows <= ppk::kRunRows;
    if (narrow && !spans.empty() && spans.back().run && spans.back().l1 == l &&
        l - spans.back().l0 < ppk::kRunLevels) {
      spans.back().l1 = l + 1;
      spans.back().width = std::max(spans.back().width, rows);
    } else {
      spans.push_back(LevelSpan{l, l + 1, narrow, rows});
    }
  }
  return spans;
}

// Level schedule of one sweep by frontier expansion; fills S.row, S.lbeg,
// S.lbeg_host, S.spans.  indeg is consumed.
int build_levels(int n, const int32_t *rp_t, const int32_t *rows_t, bool upper, int32_t *indeg,
                 Sweep &S, Allocs &own, Allocs &tmp, hipStream_t s) {
  int32_t *lsz = nullptr, *lbeg = nullptr;
  const int64_t cap = (int64_t)n + kLevelBatch + 2;
  ILU_TRY(tmp.take(&lsz, cap));
  ILU_TRY(tmp.take(&lbeg, cap));
  ILU_TRY(own.take(&S.row, n));
  ILU_TRY_HIP(ppk::launch_fill<int32_t>(cap, 0, lsz, s));
  ILU_TRY_HIP(ppk::launch_fill<int32_t>(cap, 0, lbeg, s));
  ILU_TRY_HIP(ppk::launch_level_seed(n, indeg, S.row, lsz, s));
  std::vector<int32_t> sizes(kLevelBatch);
  int nlev = -1;
  for (int level = 0; nlev < 0; level += kLevelBatch) {
    if (level > n) return PP_ERR_HIP;  // cannot happen for a checked pattern
    for (int b = 0; b < kLevelBatch; ++b)
      ILU_TRY_HIP(ppk::launch_level_pass(level + b, rp_t, rows_t, upper, indeg, S.row, lbeg, lsz,
                                         s));
    ILU_TRY_HIP(hipMemcpyAsync(sizes.data(), lsz + level + 1, kLevelBatch * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
    ILU_TRY_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < kLevelBatch; ++b) {
      if (sizes[b] == 0) {
        nlev = level + 1 + b;
        break;
      }
    }
  }
  S.nlev = nlev;
  S.lbeg_host.assign(nlev + 1, 0);
  ILU_TRY_HIP(hipMemcpyAsync(S.lbeg_host.data(), lbeg, (nlev + 1) * sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
  ILU_TRY_HIP(hipStreamSynchronize(s));
  if (S.lbeg_host[0] != 0 || S.lbeg_host[nlev] != n) return PP_ERR_HIP;
  ILU_TRY(own.take(&S.lbeg, nlev + 1));
  ILU_TRY_HIP(hipMemcpyAsync(S.lbeg, lbeg, (nlev + 1) * sizeof(int32_t),
                             hipMemcpyDeviceToDevice, s));
  S.spans = make_spans(S.lbeg_host);
  return PP_OK;
}

// Level-ordered copy of one triangle of the factors.
int build_sweep(int n, const int32_t *rp, const int32_t *ci, const int32_t *dpos,
                const double *lu, bool upper, Sweep &S, Allocs &own, Allocs &tmp,
                hipStream_t s) {
  int32_t *cnt = nullptr, *scan = nullptr, *wmax = nullptr;
  ILU_TRY(tmp.take(&cnt, n));
  ILU_TRY(tmp.take(&scan, ppk::scan_tmp_size(n)));
  ILU_TRY(tmp.take(&wmax, 64));
  ILU_TRY(own.take(&S.ptr, (int64_t)n + 1));
  ILU_TRY_HIP(ppk::launch_fill<int32_t>(1, 0, wmax, s));
  ILU_TRY_HIP(ppk::launch_sweep_counts(n, S.row, rp, dpos, upper, cnt, wmax, s));
  ILU_TRY_HIP(ppk::launch_exclusive_scan(n, cnt, S.ptr, scan, s));
  int32_t hv[2] = {0, 0};
  ILU_TRY_HIP(hipMemcpyAsync(&hv[0], S.ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  ILU_TRY_HIP(hipMemcpyAsync(&hv[1], wmax, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  ILU_TRY_HIP(hipStreamSynchronize(s));
  const int32_t entries = hv[0];
  S.entries = entries;
  S.width = hv[1];
  ILU_TRY(own.take(&S.col, entries));
  ILU_TRY(own.take(&S.val, entries));
  if (upper) ILU_TRY(own.take(&S.diag, n));
  ILU_TRY_HIP(ppk::launch_sweep_fill(n, S.row, rp, ci, dpos, lu, upper, S.ptr, S.col, S.val,
                                     S.diag, s));
  if (S.width <= ppk::kPipeSlots) {  // slot-major copy for the pipelined runs (>= 1 slot)
    const int w = std::max(S.width, 1);
    S.width = w;
    ILU_TRY(own.take(&S.ecol, (int64_t)w * n));
    ILU_TRY(own.take(&S.eval, (int64_t)w * n));
    ILU_TRY_HIP(ppk::launch_sweep_ell(n, w, S.ptr, S.col, S.val, S.ecol, S.eval, s));
    // where the run kernel finds each entry's solved value (LDS ring or global)
    std::vector<int32_t> runstart(S.nlev, -1);
    for (const ppk::LevelSpan &sp : S.spans)
      if (sp.run)
        for (int l = sp.l0; l < sp.l1; ++l) runstart[l] = sp.l0;
    int32_t *qpos = nullptr, *rs = nullptr, *flag = nullptr;
    ILU_TRY(tmp.take(&qpos, n));
    ILU_TRY(tmp.take(&rs, S.nlev));
    ILU_TRY(tmp.take(&flag, 64));
    ILU_TRY(own.take(&S.esrc, (int64_t)w * n));
    int32_t *lglob = nullptr;
    ILU_TRY(tmp.take(&lglob, S.nlev));
    ILU_TRY_HIP(ppk::launch_fill<int32_t>(S.nlev, 0, lglob, s));
    ILU_TRY_HIP(hipMemcpyAsync(rs, runstart.data(), S.nlev * sizeof(int32_t),
                               hipMemcpyHostToDevice, s));
    ILU_TRY_HIP(ppk::launch_fill<int32_t>(1, 0, flag, s));
    ILU_TRY_HIP(ppk::launch_sweep_inverse(n, S.row, qpos, s));
    ILU_TRY_HIP(ppk::launch_sweep_sources(n, w, S.nlev, S.lbeg, S.ecol, qpos, rs, S.esrc,
                                          lglob, flag, s));
    int32_t far = 0;
    std::vector<int32_t> hglob(S.nlev);
    ILU_TRY_HIP(hipMemcpyAsync(&far, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    ILU_TRY_HIP(hipMemcpyAsync(hglob.data(), lglob, S.nlev * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
    ILU_TRY_HIP(hipStreamSynchronize(s));
    if (far) {
      S.esrc = nullptr;  // (its buffer stays owned and is freed with the factor)
    } else {
      for (ppk::LevelSpan &sp : S.spans)
        if (sp.run)
          for (int l = sp.l0; l < sp.l1; ++l) sp.glob = sp.glob || hglob[l] != 0;
      if (w <= ppk::kRingSlots) {  // LDS-ring runs: their per-position data
        uint32_t *rslot = nullptr;
        ILU_TRY(own.take(&rslot, (int64_t)ppk::ring_swords(w) * n));
        ILU_TRY(own.take(&S.rval, (int64_t)ppk::ring_vstride(w) * n));
        ILU_TRY_HIP(ppk::launch_ring_pack(n, w, S.esrc, S.eval, upper ? S.diag : nullptr, rslot,
                                          S.rval, s));
        S.rslot = rslot;
      }
    }
  }
  return PP_OK;
}

int factor_steps(const pp_csr *A, hipStream_t s, pp_ilu *M, Allocs &own, Allocs &tmp) {
  const int n = (int)A->n;
  const int64_t nnz = A->nnz;
  M->n = n;
  M->nnz = nnz;
  int32_t *dpos, *indeg_l, *indeg_u, *flag, *cnt, *rp_t, *cursor, *rows_t, *scan;
  ILU_TRY(tmp.take(&dpos, n));
  ILU_TRY(tmp.take(&indeg_l, n));
  ILU_TRY(tmp.take(&indeg_u, n));
  ILU_TRY(tmp.take(&flag, 64));
  ILU_TRY(tmp.take(&cnt, n));
  ILU_TRY(tmp.take(&rp_t, (int64_t)n + 1));
  ILU_TRY(tmp.take(&cursor, n));
  ILU_TRY(tmp.take(&rows_t, nnz));
  ILU_TRY(tmp.take(&scan, ppk::scan_tmp_size(n)));
  // the pattern: sorted unique columns in range and a stored diagonal in every row
  ILU_TRY_HIP(ppk::launch_fill<int32_t>(1, 0, flag, s));
  ILU_TRY_HIP(ppk::launch_ilu_check(n, A->row_ptr, A->col_ind, dpos, indeg_l, indeg_u, flag, s));
  int32_t hflag = 0;
  ILU_TRY_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  ILU_TRY_HIP(hipStreamSynchronize(s));
  if (hflag) return PP_ERR_ARG;
  // rows of each column, for the frontier passes
  ILU_TRY_HIP(ppk::launch_fill<int32_t>(n, 0, cnt, s));
  ILU_TRY_HIP(ppk::launch_fill<int32_t>(n, 0, cursor, s));
  ILU_TRY_HIP(ppk::launch_count_cols((int)nnz, A->col_ind, cnt, s));
  ILU_TRY_HIP(ppk::launch_exclusive_scan(n, cnt, rp_t, scan, s));
  ILU_TRY_HIP(ppk::launch_scatter_pattern(n, A->row_ptr, A->col_ind, rp_t, cursor, rows_t, s));
  ILU_TRY(build_levels(n, rp_t, rows_t, false, indeg_l, M->fwd, own, tmp, s));
  ILU_TRY(build_levels(n, rp_t, rows_t, true, indeg_u, M->bwd, own, tmp, s));
  // the factorisation, in place on a copy of A's values, in forward level order
  ILU_TRY(own.take(&M->lu, nnz));
  ILU_TRY_HIP(hipMemcpyAsync(M->lu, A->vals, nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
  ILU_TRY_HIP(ppk::launch_ilu_factor(M->fwd, A->row_ptr, A->col_ind, dpos, M->lu, s));
  ILU_TRY_HIP(ppk::launch_fill<int32_t>(1, 0, flag, s));
  ILU_TRY_HIP(ppk::launch_ilu_pivots(n, nnz, dpos, M->lu, flag, s));
  ILU_TRY_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  ILU_TRY_HIP(hipStreamSynchronize(s));
  if (hflag) return PP_ERR_SINGULAR;
  ILU_TRY(build_sweep(n, A->row_ptr, A->col_ind, dpos, M->lu, false, M->fwd, own, tmp, s));
  ILU_TRY(build_sweep(n, A->row_ptr, A->col_ind, dpos, M->lu, true, M->bwd, own, tmp, s));
  ILU_TRY(own.take(&M->work, n));
  return PP_OK;
}

// The factorisation; on any error the stream is drained before the buffers go.
int factor(const pp_csr *A, hipStream_t s, pp_ilu *M) {
  Allocs own, tmp;
  int rc = factor_steps(A, s, M, own, tmp);
  if (hipStreamSynchronize(s) != hipSuccess && rc >= 0) rc = PP_ERR_HIP;
  if (rc < 0) return rc;
  M->owned = own.ptrs;
  own.ptrs.clear();
  return PP_OK;
}

}  // namespace

namespace ppi {

hipError_t ilu_solve(const pp_ilu &M, const double *r, double *z, hipStream_t s) {
  const hipError_t e = ppk::launch_ilu_forward((int)M.n, M.fwd, r, z, M.work, s);
  if (e != hipSuccess) return e;
  return ppk::launch_ilu_backward((int)M.n, M.bwd, z, z, M.work, s);
}

bool on_device(const pp_ilu &M) {
  int dev = -1;
  return hipGetDevice(&dev) == hipSuccess && dev == M.device;
}

double ilu_solve_bytes(const pp_ilu &M) {
  // per sweep: the level order and row pointers (8 n), the waited-for entries
  // (12 per entry), the right-hand side read, the solution written and gathered
  // (24 n); the backward sweep also reads the pivots (8 n)
  const double n = (double)M.n;
  return 2.0 * (8.0 * n + 24.0 * n) + 8.0 * n + 12.0 * (double)(M.fwd.entries + M.bwd.entries);
}

}  // namespace ppi

extern "C" {

int pp_ilu0_factor(const pp_csr *A, void *stream, pp_ilu **out) {
  ppd::enter("pp_ilu0_factor");
  if (!out) return PP_ERR_ARG;
  *out = nullptr;
  if (!A || A->n <= 0 || A->n >= ((int64_t)1 << 31) || A->nnz < A->n ||
      A->nnz >= ((int64_t)1 << 31) || !A->row_ptr || !A->col_ind || !A->vals ||
      A->dtype != PP_F64)
    return PP_ERR_ARG;
  pp_ilu *M = new (std::nothrow) pp_ilu;
  if (!M) return PP_ERR_NOMEM;
  if (hipGetDevice(&M->device) != hipSuccess) {
    delete M;
    return PP_ERR_HIP;
  }
  const int rc = factor(A, static_cast<hipStream_t>(stream), M);
  if (rc < 0) {
    free_ilu(M);
    return rc;
  }
  if (const char *v = std::getenv("PP_LOG"); v && std::atoi(v) >= 1)
    std::fprintf(stderr, "[pp] ilu0: n %lld, levels %d forward / %d backward, %zu + %zu spans\n",
                 (long long)M->n, M->fwd.nlev, M->bwd.nlev, M->fwd.spans.size(),
                 M->bwd.spans.size());
  *out = M;
  return PP_OK;
}

int pp_ilu0_apply(const pp_ilu *M, const double *r, double *z, void *stream) {
  ppd::enter("pp_ilu0_apply");
  if (!M || !r || !z || !ppi::on_device(*M)) return PP_ERR_ARG;
  std::lock_guard<std::mutex> lk(M->lock);  // M->work, until the sweeps are done
  hipStream_t s = static_cast<hipStream_t>(stream);
  ILU_TRY_HIP(ppi::ilu_solve(*M, r, z, s));
  ILU_TRY_HIP(hipStreamSynchronize(s));
  return PP_OK;
}

int pp_ilu0_values(const pp_ilu *M, double *lu, void *stream) {
  ppd::enter("pp_ilu0_values");
  if (!M || !lu || !ppi::on_device(*M)) return PP_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ILU_TRY_HIP(hipMemcpyAsync(lu, M->lu, M->nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
  ILU_TRY_HIP(hipStreamSynchronize(s));
  return PP_OK;
}

int pp_ilu0_levels(const pp_ilu *M, int32_t *nlev_forward, int32_t *nlev_backward,
                   int32_t *launches) {
  if (!M) return PP_ERR_ARG;
  if (nlev_forward) *nlev_forward = M->fwd.nlev;
  if (nlev_backward) *nlev_backward = M->bwd.nlev;
  // the sweeps' spans; a sweep with LDS-ring runs adds its level-order gather and,
  // per run, the scatter of its solutions and (when the run waits for values solved
  // by earlier launches) the right-hand-side update before it
  auto extra = [](const Sweep &S) {
    if (!S.rslot) return 0;
    int k = 1;
    for (const ppk::LevelSpan &sp : S.spans) k += sp.run ? (sp.glob ? 2 : 1) : 0;
    return k;
  };
  if (launches)
    *launches = (int32_t)(M->fwd.spans.size() + M->bwd.spans.size() + extra(M->fwd) +
                          extra(M->bwd));
  return PP_OK;
}

void pp_ilu0_free(pp_ilu *M) {
  if (M) (void)hipDeviceSynchronize();
  free_ilu(M);
}

}  // extern "C"
