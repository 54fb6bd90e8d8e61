// ILU(0) on the device (internal to libpp): the kernels' launch wrappers and the
// host-side factor object behind the opaque pp_ilu of include/pp.h.
//
// ILU(0) (Saad, Iterative Methods for Sparse Linear Systems, Section 10.3) keeps
// A's pattern: L unit lower and U upper triangular with (L U)_ij = a_ij on every
// stored (i, j).  It is the left preconditioner of Section VI's second example.
//
// Both the factorisation and the triangular solves run level by level: the
// level of a row is one more than the highest level among the rows it waits
// for (k < i stored in row i for the forward solve and the factorisation,
// k > i for the backward solve), so the rows of one level are independent.
// Levels are found on the device by frontier expansion over the transposed
// pattern.  A run of consecutive narrow levels (at most kRunRows rows each, at
// most kRunLevels levels) goes to one workgroup that steps through them with a barrier between levels; a
// wide level gets a launch of its own.  Inside a run the solved values of the
// last kRing levels travel through LDS when every dependency allows it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "kernels.h"

namespace ppk {

constexpr int kRunThreads = 1024;  // threads of the one workgroup that steps through a run
constexpr int kRunRows = 1024;     // widest level handled inside a run
constexpr int kPipeSlots = 8;      // most waited-for entries per row of the pipelined run
constexpr int kRing = 4;           // levels of solved values a run keeps in LDS
constexpr int kRingSlots = 4;      // most entries per row of the LDS-ring run kernel
constexpr int kRunLevels = 4096;   // most levels in one run (a longer chain of narrow levels
                                   // is split into several runs)

// Per-position layout of the LDS-ring run data (see Sweep): doubles of entries and
// 32-bit words of packed slots for rows of w <= kRingSlots entries.
constexpr int ring_vstride(int w) { return w == 1 ? 1 : w == 2 ? 2 : 4; }
constexpr int ring_swords(int w) { return w <= 2 ? 1 : 2; }
static_assert(kRing * kRunRows < 32768, "ring slots are 16-bit integers");

// A span of consecutive levels [l0, l1): a run (narrow levels, one workgroup) or
// a single wide level.
struct LevelSpan {
  int l0, l1;
  bool run;
  int width;          // rows of the span's widest level
  bool glob = false;  // a run some of whose rows wait for values solved by earlier launches
};

// Level schedule of one triangular sweep and its level-ordered copy of the factor.
// Position q (0..n-1) is the q-th row of the sweep in level order: row[q]; the
// off-diagonal entries the row waits for are ptr[q]..ptr[q+1] in col/val; diag[q]
// is U's pivot of the row (backward sweep only).  When no row waits for more than
// kPipeSlots entries the same entries are also kept slot-major (width slots per
// position, slot s of position q at s * n + q, padding column -1 / value 0) for
// the pipelined run kernel.
struct Sweep {
  int nlev = 0;
  int32_t *row = nullptr;   // [n]
  int32_t *lbeg = nullptr;  // [nlev + 1] device: first position of each level
  int32_t *ptr = nullptr;   // [n + 1]
  int32_t *col = nullptr;   // [entries]
  double *val = nullptr;    // [entries]
  double *diag = nullptr;   // [n] (backward sweep)
  int64_t entries = 0;
  int width = 0;            // most entries one row waits for
  int32_t *ecol = nullptr;  // [width * n] slot-major copy (nullptr: width > kPipeSlots)
  double *eval = nullptr;   // [width * n]
  // [width * n] where the run kernel finds each entry's solved value: its slot in the
  // run's LDS ring ((level % kRing) * kRunRows + position in the level) when the
  // column was solved in the same run at most kRing - 1 levels earlier, -1 when it
  // was solved by an earlier launch; nullptr when some entry is neither (then the
  // run kernel reads every solved value from global memory)
  int32_t *esrc = nullptr;
  // LDS-ring run data (nullptr unless esrc is set and width <= kRingSlots), per
  // position q: ring_swords(width) 32-bit words of ring slots at rslot[q * words],
  // each slot a 16-bit integer (-1: the value is not in the ring), and the entries at
  // rval[q * ring_vstride(width) + s] (zero past width), divided by the pivot in the
  // backward sweep
  uint32_t *rslot = nullptr;
  double *rval = nullptr;
  std::vector<int32_t> lbeg_host;
  std::vector<LevelSpan> spans;
};

// z = L^-1 r (z may equal r): the forward sweep of the level-ordered L.  work
// (n doubles) receives r in level order when the sweep has LDS-ring runs.
hipError_t launch_ilu_forward(int n, const Sweep &L, const double *r, double *z, double *work,
                              hipStream_t stream);
// x = U^-1 z, in place allowed (x == z); work as above.
hipError_t launch_ilu_backward(int n, const Sweep &U, const double *z, double *x, double *work,
                               hipStream_t stream);

// Pattern check: dpos[i] = position of row i's diagonal (-1 if absent);
// indeg_l[i] / indeg_u[i] = entries left / right of it; *flag |= 1 when a row's
// columns are not strictly increasing or out of [0, n), |= 2 when a row has no
// diagonal.
hipError_t launch_ilu_check(int n, const int32_t *rp, const int32_t *ci, int32_t *dpos,
                            int32_t *indeg_l, int32_t *indeg_u, int32_t *flag,
                            hipStream_t stream);
// Rows of each column: rows_t[rp_t[j] + ...] = i for every stored (i, j) (any order
// inside a column); cursor[n] zeroed by the caller.
hipError_t launch_scatter_pattern(int n, const int32_t *rp, const int32_t *ci,
                                  const int32_t *rp_t, int32_t *cursor, int32_t *rows_t,
                                  hipStream_t stream);
// Level 0: rows with indeg 0 are appended to perm (lsz[0] counts them).
hipError_t launch_level_seed(int n, const int32_t *indeg, int32_t *perm, int32_t *lsz,
                             hipStream_t stream);
// Frontier expansion of `level`: its rows perm[lbeg[level] + 0..lsz[level]) release
// the rows that wait for them (rows i > k of column k, or i < k when `upper`);
// a row released for the last time is appended as level + 1.  Writes
// lbeg[level + 1].
hipError_t launch_level_pass(int level, const int32_t *rp_t, const int32_t *rows_t, bool upper,
                             int32_t *indeg, int32_t *perm, int32_t *lbeg, int32_t *lsz,
                             hipStream_t stream);
// The factorisation, level by level of the forward schedule, in place on lu
// (A's values on entry, in A's CSR order).
hipError_t launch_ilu_factor(const Sweep &L, const int32_t *rp, const int32_t *ci,
                             const int32_t *dpos, double *lu, hipStream_t stream);
// *flag |= 1 for a zero pivot, |= 2 for a non-finite factor entry.
hipError_t launch_ilu_pivots(int n, int64_t nnz, const int32_t *dpos, const double *lu,
                             int32_t *flag, hipStream_t stream);
// cnt[q] = entries row[q] waits for (left of the diagonal, or right when `upper`);
// *wmax = max of them (atomic max; zeroed by the caller).
hipError_t launch_sweep_counts(int n, const int32_t *row, const int32_t *rp,
                               const int32_t *dpos, bool upper, int32_t *cnt, int32_t *wmax,
                               hipStream_t stream);
// Slot-major copy of a level-ordered sweep (width >= every row's entry count).
hipError_t launch_sweep_ell(int n, int width, const int32_t *ptr, const int32_t *col,
                            const double *val, int32_t *ecol, double *eval, hipStream_t stream);
// Level-ordered copy of one triangle of lu: col/val at ptr[q].., diag[q] when upper.
hipError_t launch_sweep_fill(int n, const int32_t *row, const int32_t *rp, const int32_t *ci,
                             const int32_t *dpos, const double *lu, bool upper,
                             const int32_t *ptr, int32_t *col, double *val, double *diag,
                             hipStream_t stream);

// qpos[row[q]] = q.
hipError_t launch_sweep_inverse(int n, const int32_t *row, int32_t *qpos, hipStream_t stream);
// esrc of a slot-major sweep (see Sweep); runstart[l] = first level of the run that
// holds level l, or -1 for a level launched on its own; lglob[l] = 1 (zeroed by the
// caller) when a row of run level l reads a value solved by an earlier launch;
// *flag = 1 when an entry's column was solved in the same run but kRing or more
// levels earlier.
hipError_t launch_sweep_sources(int n, int width, int nlev, const int32_t *lbeg,
                                const int32_t *ecol, const int32_t *qpos,
                                const int32_t *runstart, int32_t *esrc, int32_t *lglob,
                                int32_t *flag, hipStream_t stream);

// LDS-ring run data (Sweep::rslot, Sweep::rval) from the slot-major copy and esrc
// (width 1..kRingSlots); diag: the backward sweep's pivots (entries divided by
// them), nullptr for the forward sweep.
hipError_t launch_ring_pack(int n, int width, const int32_t *esrc, const double *eval,
                            const double *diag, uint32_t *rslot, double *rval,
                            hipStream_t stream);

// Elementwise chain step with the operator's product given (prod = Op g, unscaled):
// the kinds of ChainArgs with (A g)(i) replaced by prod(i).
hipError_t launch_chain_given(int n, int kind, bool fold, bool last, const double *prod,
                              const ChainArgs<double> &a, hipStream_t stream);
// out = b - y and partial[g] = sum of out^2 over workgroup g; *ntiles = workgroups.
hipError_t launch_sub_norm(int n, const double *b, const double *y, double *out,
                           double *partial, int *ntiles, hipStream_t stream);

}  // namespace ppk

// The factor object behind pp_ilu: device arrays owned by it.
struct pp_ilu {
  int64_t n = 0, nnz = 0;
  int device = -1;                       // the device its arrays live on
  double *lu = nullptr;                  // factors in A's CSR order
  ppk::Sweep fwd, bwd;
  double *work = nullptr;                // [n] right-hand side in level order
  std::vector<void *> owned;             // every device allocation above
  mutable std::mutex lock;               // held by every call that uses work, until it completes
};

namespace ppi {
// z = M^-1 r = U^-1 L^-1 r (z may equal r).
hipError_t ilu_solve(const pp_ilu &M, const double *r, double *z, hipStream_t s);
// Algorithmic HBM bytes of one ilu_solve.
double ilu_solve_bytes(const pp_ilu &M);
// Whether the current device is the one the factor lives on.
bool on_device(const pp_ilu &M);
}  // namespace ppi
