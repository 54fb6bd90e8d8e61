// libpp host driver: the C ABI of include/pp.h.
//
// The device does every O(n) step (kernels.hip); the host keeps only the
// small dense state of the method: the (m+1) x m Hessenberg matrix, its Givens
// rotations and least-squares solution, and the d x d harmonic Ritz
// eigenproblem (host_numerics.cpp).  Each Arnoldi step ends with one
// device-to-host copy of the new Hessenberg column (the two CGS passes'
// coefficients and the norm) and one stream synchronisation.
//
// Basis storage: column c of the Krylov basis is kept unnormalised in V and
// scaled on the fly by colscale[c] (a device array written by the norm
// reduction), so no separate normalisation pass is needed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/pp.h"
#include "diag.h"
#include "host_numerics.h"
#include "ilu.h"
#include "kernels.h"
#include "noalloc.h"

struct pp_poly {
  int64_t n;
  int dtype;
  int kind = 0;                 // 0: Leja-ordered roots; 1: power-basis coefficients
  std::vector<double> re, im;   // kind 0
  std::vector<ppn::Step> steps; // kind 0
  std::vector<double> coeffs;   // kind 1: p(A) = sum_k coeffs[k] A^k
  int info = 0;                 // kind 1: POTRF status of the Gram matrix
};

namespace {

using ppk::SpMat;

constexpr int kMaxM = 256;
constexpr int kMaxD = 256;
constexpr double kBreakdownRtol = 1e-12;
// Attainable accuracy: below kStagnationBand * tol, kStagnationCycles consecutive
// restart cycles that each end on the implicit estimate (it reached tol) and leave
// the true residual above kStagnationFactor times
// its previous value end the solve (PP_WARN_NOT_CONVERGED).
constexpr double kStagnationBand = 100.0;
constexpr double kStagnationFactor = 0.9;
constexpr int kStagnationCycles = 3;
// Working set of one chain launch (its matrix rows and two vectors) that MI355X's
// 256 MiB Infinity Cache still returns to the next launch: 27/32 of it.  Measured
// on the 256^3 stencil: the slab-skewed schedule gains up to 3.0M rows per slab in
// FP64 (73 B a row, 219 MiB) and 6.3M in FP32 (37 B, 222 MiB), and loses it all
// at 3.5M rows in FP64 (255 MiB).
constexpr double kCacheBudget = 216.0 * 1024 * 1024;
// the slab-skewed schedule is chosen only when the bandwidth is at most this
// fraction of a slab (the rest of a slab is re-read from cache)
constexpr int kSlabPerBandwidth = 8;
// group size standing for "all of a step's launches"
constexpr int kAllLaunches = 1 << 20;
// seed of the start vector drawn when pp_build_poly / pp_build_poly_power get none
constexpr uint64_t kDefaultSeed = 0;
// FP32 refinement: default inner relative reduction, and the margin of the
// automatic looser one on a step close to tol (see solve_f32_ir)
constexpr double kInnerTolDefault = 1e-5;
constexpr double kInnerMargin = 0.5;

#define PP_TRY_HIP(expr) PPD_TRY_HIP(expr, PP_ERR_HIP)
#define PP_TRY(expr)                                  \
  do {                                                \
    int r_ = (expr);                                  \
    if (r_ < 0) return r_;                            \
  } while (0)

std::mutex g_lock;

// Tracing to stderr, from the environment variable PP_LOG (read once): 0 (default)
// silent; 1 one line per restart cycle / refinement step; 2 also every Arnoldi
// step's implicit residual.
int log_level() { return ppd::log_level(); }

struct Arena {
  char *dev = nullptr;
  size_t dev_cap = 0;
  char *aux = nullptr;  // composed operator (scaled copy of A, scaled b); outlives `dev` carving
  size_t aux_cap = 0;
  char *mat = nullptr;  // sliced copy of the call's matrix; outlives `dev` carving
  size_t mat_cap = 0;
  double *host = nullptr;  // pinned
  size_t host_cap = 0;     // in doubles
  hipEvent_t step_ev[2] = {nullptr, nullptr};  // completion of an Arnoldi step, per host slot
};
std::vector<Arena> g_arena;

int current_arena(Arena **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PP_ERR_HIP;
  if ((int)g_arena.size() <= dev) g_arena.resize(dev + 1);
  *out = &g_arena[dev];
  return PP_OK;
}

int ensure_arena(Arena *a, size_t dev_bytes, size_t host_doubles) {
  if (dev_bytes > a->dev_cap) {
    if (a->dev) {
      if (hipDeviceSynchronize() != hipSuccess) return PP_ERR_HIP;
      (void)hipFree(a->dev);
      a->dev = nullptr;
      a->dev_cap = 0;
    }
    if (hipMalloc((void **)&a->dev, dev_bytes) != hipSuccess) {
      a->dev = nullptr;
      return PP_ERR_NOMEM;
    }
    a->dev_cap = dev_bytes;
  }
  if (host_doubles > a->host_cap) {
    if (a->host) {
      // kernels write step results into it: nothing may still be in flight
      if (hipDeviceSynchronize() != hipSuccess) return PP_ERR_HIP;
      (void)hipHostFree(a->host);
    }
    a->host = nullptr;
    a->host_cap = 0;
    // coherent: kernels write small results straight into it (the Arnoldi step's
    // Hessenberg column), visible to the host once the stream is synchronised
    if (hipHostMalloc((void **)&a->host, host_doubles * sizeof(double), hipHostMallocCoherent) !=
        hipSuccess) {
      a->host = nullptr;
      return PP_ERR_NOMEM;
    }
    a->host_cap = host_doubles;
  }
  for (hipEvent_t &e : a->step_ev)
    if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      e = nullptr;
      return PP_ERR_HIP;
    }
  return PP_OK;
}

// Grow one of the arena's side buffers (aux, mat) to at least `bytes`.
int ensure_side(char **buf, size_t *cap, size_t bytes) {
  if (bytes <= *cap) return PP_OK;
  if (*buf) {
    if (hipDeviceSynchronize() != hipSuccess) return PP_ERR_HIP;
    (void)hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
  }
  if (hipMalloc((void **)buf, bytes) != hipSuccess) {
    *buf = nullptr;
    return PP_ERR_NOMEM;
  }
  *cap = bytes;
  return PP_OK;
}

int ensure_aux(Arena *a, size_t bytes) { return ensure_side(&a->aux, &a->aux_cap, bytes); }

// Sequential 256-byte aligned carving of the device arena.  With base == nullptr
// it only measures.
struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(char *b) : base(b) {}
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Leading dimension of the Krylov basis: n rounded up to 64 elements (512 B), plus 64
// more when that is a multiple of 2048 elements, so columns are not a power-of-two
// number of bytes apart (the CGS2 sweeps read one row of every column together).
inline int64_t pad_ld(int64_t n) {
  const int64_t ld = (n + 63) / 64 * 64;
  return ld % 2048 == 0 ? ld + 64 : ld;
}

// ------------------------------------------------------- CGS2 sweep sizing
// Sweep kinds, for the choice of rows per thread.
constexpr int kOrthRead = 0;        // k_dots, k_norm2 without the FP32 copy (read-only)
constexpr int kOrthUpdateDots = 1;  // k_update fused with the next pass's dots
constexpr int kOrthWrite = 2;       // k_update with the norm or alone, k_norm2 with the copy
constexpr int kOrthMinRpt = 1;      // the smallest value orth_rpt returns

// Rows per thread of a CGS2 sweep of n rows over nc <= kMaxCols basis columns (each
// workgroup owns a contiguous block of 256 * rpt rows).  The table was measured on
// gfx950 at n = 16.8M: read-only sweeps run long workgroups; sweeps that write run
// short ones, so the resident workgroups' stores stay within a narrow window of
// HBM, as in a flat copy (FP64 update + norm: 5.2 -> 6.0 TB/s); the update + dots
// sweep sits between.  Smaller n lowers rpt (down to 1) until the sweep keeps a
// floor of workgroups, or one per 256 rows: long blocks on a few hundred thousand
// rows leave most compute units idle (at 512^2 the dot sweep ran 32 workgroups at
// 1.1 TB/s).  Each workgroup of a sweep with dots ends with nc block reductions,
// so that floor falls with nc (2048 workgroups for a few columns, 256 from 32
// columns on); the update and norm sweeps keep 2048.
int orth_rpt_table(int kind, int nc, bool f32) {
  if (kind == kOrthRead) return (f32 && nc <= 24) ? 4 : 32;
  if (kind == kOrthUpdateDots) {
    if (nc <= 8) return f32 ? 4 : 2;
    if (nc <= 24) return 4;
    if (nc <= 40) return 8;
    return 32;
  }
  return (!f32 && nc > 40) ? 8 : 2;
}

int orth_rpt(int kind, int nc, bool f32, int64_t n) {
  const int64_t groups =
      kind == kOrthWrite ? 2048 : std::min<int64_t>(2048, std::max<int64_t>(256, 8192 / nc));
  const int64_t cap = n / ((int64_t)ppk::kBlock * groups);
  const int rpt = orth_rpt_table(kind, nc, f32);
  return (int)std::max<int64_t>(kOrthMinRpt, std::min<int64_t>(rpt, cap));
}

// Environment variable PP_FOLD=1 folds each CGS2 reduction's second stage into its
// sweep where the partials are few (the same bits, three launches fewer per step;
// measured slower on MI355X, so off by default).  Read at each call.
bool fold_enabled() {
  const char *v = std::getenv("PP_FOLD");
  return v && std::atoi(v) != 0;
}

// One-step lookahead of short Arnoldi steps (see StepPipe); PP_LOOKAHEAD=0 turns it off.
bool lookahead_enabled() {
  const char *v = std::getenv("PP_LOOKAHEAD");
  return !(v && std::atoi(v) == 0);
}

// Device workspace of one solve in compute type T.
template <typename T>
struct Work {
  int n = 0, L = 0;  // L = basis columns
  int64_t ldv = 0;
  T *V = nullptr, *P0 = nullptr, *P1 = nullptr, *Tb = nullptr, *Z = nullptr, *W = nullptr,
    *U = nullptr;
  double *partial = nullptr;
  double *colscale = nullptr;  // [L]
  double *hbuf = nullptr;      // [2L + 8]: h1 | h2 | nrm
  double *coef1 = nullptr, *coef2 = nullptr, *ybuf = nullptr;  // [L] each
  double *misc = nullptr;      // [16]
  // pinned: two slots of 2L + 8 (an Arnoldi step's Hessenberg column h1 | h2 | nrm,
  // slot j & 1 for step j), then the staging of y [L] and 16 spare
  double *host = nullptr;
  hipEvent_t step_ev[2] = {nullptr, nullptr};  // step j done: step_ev[j & 1]
  int32_t *fold_counter = nullptr;  // ticket counter of the folded reductions
  bool fold_armed = false;          // fold_counter zeroed on the device
  bool fold_ok = false;             // folded reductions asked for (PP_FOLD=1)
  bool lookahead_ok = true;         // short steps issued one ahead (PP_LOOKAHEAD)

  template <typename C>
  void carve(C &c, int n_, int L_) {
    n = n_;
    L = L_;
    ldv = pad_ld(n_);
    V = c.template take<T>((size_t)ldv * L);
    P0 = c.template take<T>(ldv);
    P1 = c.template take<T>(ldv);
    Tb = c.template take<T>(ldv);
    Z = c.template take<T>(ldv);
    W = c.template take<T>(ldv);
    U = c.template take<T>(ldv);
    const size_t tiles = (size_t)(n_ + ppk::kBlock - 1) / ppk::kBlock;
    // CGS2 partials: up to L columns at the largest workgroup count of any sweep
    const size_t gmax = (size_t)ppk::orth_grid(n_, kOrthMinRpt);
    partial = c.template take<double>(std::max((size_t)L * gmax, tiles) + 64);
    colscale = c.template take<double>(L);
    hbuf = c.template take<double>(2 * (size_t)L + 8);
    coef1 = c.template take<double>(L);
    coef2 = c.template take<double>(L);
    ybuf = c.template take<double>(L);
    misc = c.template take<double>(16);
    fold_counter = c.template take<int32_t>(64);
    fold_armed = false;
    fold_ok = fold_enabled();
    lookahead_ok = lookahead_enabled();
  }
  size_t host_doubles() const { return 2 * hslot_doubles() + (size_t)L + 16; }
  size_t hslot_doubles() const { return 2 * (size_t)L + 8; }
  double *hslot(int j) const { return host + (size_t)(j & 1) * hslot_doubles(); }
  double *ystage() const { return host + 2 * hslot_doubles(); }
  void attach(const Arena &a) {
    host = a.host;
    step_ev[0] = a.step_ev[0];
    step_ev[1] = a.step_ev[1];
  }
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Event-timed phases of the Arnoldi steps: one set of events per host slot (step j
// uses set j & 1), so a step issued ahead does not overwrite the events of the
// step still to be collected.
struct Timers {
  bool on = false;
  hipEvent_t ev[2][4] = {};
  int slot = 0;         // the set mark() records into
  double t_last = 0.0;  // wall clock at the previous step's collection
  int init() {
    for (auto &set : ev)
      for (auto &e : set)
        if (hipEventCreate(&e) != hipSuccess) return PP_ERR_HIP;
    return PP_OK;
  }
  ~Timers() {
    for (auto &set : ev)
      for (auto &e : set)
        if (e) (void)hipEventDestroy(e);
  }
  void mark(int k, hipStream_t s) {
    if (on) (void)hipEventRecord(ev[slot][k], s);
  }
  void start() {
    if (on) t_last = now_s();
  }
  // Accumulate the event-timed phases of the step of set `set`; the rest of the wall
  // time since the previous collection (launch latency, synchronisation, host least
  // squares, whatever the device phases do not cover) is counted as host time.
  void collect(int set) {
    if (!on) return;
    const double now = now_s();
    const double wall = now - t_last;
    t_last = now;
    float a = 0, b = 0, c = 0;
    (void)hipEventElapsedTime(&a, ev[set][0], ev[set][1]);
    (void)hipEventElapsedTime(&b, ev[set][1], ev[set][2]);
    (void)hipEventElapsedTime(&c, ev[set][2], ev[set][3]);
    chain += a * 1e-3;
    spmv += b * 1e-3;
    orth += c * 1e-3;
    host += std::max(0.0, wall - (a + b + c) * 1e-3);
  }
  double chain = 0, spmv = 0, orth = 0, host = 0;
};

struct Counters {
  int64_t spmvs = 0, dots = 0;
  int iters = 0;
  double bytes_chain = 0, bytes_spmv = 0, bytes_orth = 0;
  int64_t launches_chain = 0;
  double *history = nullptr;
  int history_cap = 0, history_len = 0;
  void push(double v) {
    if (history && history_len < history_cap) history[history_len++] = v;
  }
};

inline bool finite(double v) { return std::isfinite(v); }

// The polynomial a solve applies: none, Leja-ordered roots, or power coefficients.
struct PolyRef {
  const std::vector<ppn::Step> *steps = nullptr;
  const std::vector<double> *coeffs = nullptr;
  bool active() const {
    return (steps && !steps->empty()) || (coeffs && !coeffs->empty());
  }
  bool power() const { return coeffs && !coeffs->empty(); }
  static PolyRef of(const pp_poly *p) {
    PolyRef r;
    if (p && p->kind == 1) r.coeffs = &p->coeffs;
    else if (p) r.steps = &p->steps;
    return r;
  }
};

// The operator of a solve: A itself, or M^-1 A with M an ILU(0) factorisation
// applied on the left (Section VI, second example; FP64 only).  prod is the
// composed operator's product buffer (n entries).
template <typename T>
struct Opr : SpMat<T> {
  const pp_ilu *ilu = nullptr;
  T *prod = nullptr;
  // slab-skewed schedule of the Arnoldi step's chain (group >= 2: on)
  int blk_group = 0;
  int blk_slab_rows = 0;
  int blk_bw_rows = 0;  // the matrix bandwidth max |col - row|
  // full-range operator-form launches with cached loads and stores (a launch's
  // matrix and vectors fit the last-level cache)
  bool keep = false;
  Opr(const SpMat<T> &m) : SpMat<T>(m) {}  // NOLINT: a plain matrix is an operator
};

// out = Op (gscale * g).
template <typename T>
int op_product(const Opr<T> &A, const T *g, const double *gscale, T *out, hipStream_t s) {
  PP_TRY_HIP(ppk::launch_spmv<T>(A, g, gscale, out, s, 0, 0, A.keep));
  if constexpr (sizeof(T) == sizeof(double)) {
    if (A.ilu) PP_TRY_HIP(ppi::ilu_solve(*A.ilu, out, out, s));
  }
  return PP_OK;
}

// One chain step (ChainArgs kinds) with the operator's product: fused with the
// sparse product for A, elementwise after the product for M^-1 A.
template <typename T>
int op_chain(const Opr<T> &A, int kind, bool fold, bool last, const ppk::ChainArgs<T> &a,
             hipStream_t s) {
  if constexpr (sizeof(T) == sizeof(double)) {
    if (A.ilu) {
      PP_TRY(op_product<T>(A, a.g, nullptr, A.prod, s));
      PP_TRY_HIP(ppk::launch_chain_given(A.n, kind, fold, last, A.prod, a, s));
      return PP_OK;
    }
  }
  if (A.keep) {
    ppk::ChainArgs<T> c = a;
    c.cached = true;
    PP_TRY_HIP(ppk::launch_chain<T>(A, kind, fold, last, c, s));
  } else {
    PP_TRY_HIP(ppk::launch_chain<T>(A, kind, fold, last, a, s));
  }
  return PP_OK;
}

// ------------------------------------------------------------------ chain
// Algorithmic HBM bytes of one sparse-product launch: the matrix (values,
// column indices, row pointers) and the gathered vector once, plus `vec_rw`
// further vector reads/writes of n entries.
template <typename T>
double product_bytes(const Opr<T> &A, int vec_rw) {
  double vecs = (double)sizeof(T) * A.n * (1 + vec_rw);
  if (A.ilu)  // the two triangular sweeps, and the product written then read back
    vecs += ppi::ilu_solve_bytes(*A.ilu) + 2.0 * sizeof(T) * A.n;
  if (A.sdesc)  // sliced copy: stored values (padding included), explicit columns,
                // diagonal offsets past the descriptors, slice descriptors
    return (double)A.snnz * sizeof(T) + 4.0 * A.snnz_ell + 4.0 * A.soff_extra +
           4.0 * ppk::kDesc * ((A.n + ppk::kSlice - 1) / ppk::kSlice) + vecs;
  return (double)A.nnz * (sizeof(T) + sizeof(int32_t)) + 4.0 * (A.n + 1) + vecs;
}

// One launch of a chain: a plain product (t = A p) or a fused product + update
// (ChainArgs kind, with its fold / last variant).
template <typename T>
struct OpLaunch {
  bool product;
  int kind;
  bool last;
  ppk::ChainArgs<T> a;  // for a product: g, gscale and out only
  bool fold = false;
};

// A chain's launches in slab-skewed order (ppn::slab_order, a matrix-powers style
// schedule, Section VII): the launches taken `group` at a time, and inside a group
// slab b of the group's k-th launch covers the tiles [b S - k w, (b+1) S - k w)
// (S tiles per slab, w = the bandwidth rounded up to whole tiles), for b = 0, 1, ...
// with the group's launches in order inside each slab.  Launch k reads launch k-1's
// output only within the bandwidth of its own rows, all of which is written by
// then; a buffer read by launch k (gathered or elementwise) is next overwritten by
// launch k + 2 or later, only at rows every later reader of its old contents has
// passed; and accumulators read and written elementwise see each row's launches
// in chain order.  So each slab's matrix and vectors are read group times while
// they may still sit in cache, with results bit-identical to the full-range
// launches.  The launches use ordinary (cached) loads and stores: with the
// non-temporal ones of the full-range chain, a slab's second pass came back from
// HBM.  *launched counts the kernel launches issued.
template <typename T>
int run_op_launches_blocked(const Opr<T> &A, const std::vector<OpLaunch<T>> &L, hipStream_t s,
                            int64_t *launched) {
  const int tr = ppk::chain_tile_rows(A);
  const int ntile = (A.n + tr - 1) / tr;
  const int S = std::max(1, A.blk_slab_rows / tr);
  const int w = (A.blk_bw_rows + tr - 1) / tr;
  std::vector<ppn::SlabPart> order;
  ppn::slab_order(ntile, S, w, (int)L.size(), A.blk_group, order);
  for (const ppn::SlabPart &part : order) {
    const OpLaunch<T> &l = L[part.k];
    const int t0 = part.t0, t1 = part.t1;
    if (l.product) {
      PP_TRY_HIP(ppk::launch_spmv<T>(A, l.a.g, l.a.gscale, l.a.out, s, t0, t1 - t0, true));
    } else {
      ppk::ChainArgs<T> a = l.a;
      a.tile0 = t0;
      a.ntiles = t1 - t0;
      a.cached = true;
      PP_TRY_HIP(ppk::launch_chain<T>(A, l.kind, l.fold, l.last, a, s));
    }
    if (launched) ++*launched;
  }
  return PP_OK;
}

// The launches of a chain as they are produced: run at once, or collected for
// the slab-skewed order when the operator asks for it (A.blk_group >= 2, no M^-1).
template <typename T>
struct ChainEmitter {
  const Opr<T> &A;
  hipStream_t s;
  Counters *cnt;
  double *bytes;
  int64_t *launches;
  bool blocked;
  std::vector<OpLaunch<T>> L;
  ChainEmitter(const Opr<T> &A_, hipStream_t s_, Counters *cnt_, double *bytes_,
               int64_t *launches_)
      : A(A_), s(s_), cnt(cnt_), bytes(bytes_), launches(launches_),
        blocked(A_.blk_group >= 2 && !A_.ilu) {}
  // one fused launch; vec_rw as for product_bytes
  int chain(int kind, bool fold, bool last, const ppk::ChainArgs<T> &a, int vec_rw) {
    if (bytes) *bytes += product_bytes(A, vec_rw);
    if (cnt) cnt->spmvs++;
    if (blocked) {
      L.push_back(OpLaunch<T>{false, kind, last, a, fold});
      return PP_OK;
    }
    if (launches) ++*launches;
    return op_chain<T>(A, kind, fold, last, a, s);
  }
  // one plain product out = A (gscale * g); vec_rw as for product_bytes
  int product(const T *g, const double *gscale, T *out, int vec_rw) {
    if (bytes) *bytes += product_bytes(A, vec_rw);
    if (cnt) cnt->spmvs++;
    if (blocked) {
      L.push_back(OpLaunch<T>{true, 0, false,
                              ppk::ChainArgs<T>{g, gscale, nullptr, nullptr, out, nullptr,
                                                nullptr, 0.0, 0.0, 0.0, nullptr}});
      return PP_OK;
    }
    if (launches) ++*launches;
    return op_product<T>(A, g, gscale, out, s);
  }
  // the collected launches, if any
  int finish() {
    if (!blocked || L.empty()) return PP_OK;
    return run_op_launches_blocked<T>(A, L, s, launches);
  }
};

// y_out = y_in + p(A) (gscale * g) for the step table; y_in may be nullptr
// (zero) or equal y_out.  Uses P0, P1, Tb as chain temporaries.  Adds the
// launches and their algorithmic bytes to *bytes / *launches when given.
template <typename T>
int run_chain(const Opr<T> &A, const std::vector<ppn::Step> &steps, const T *g,
              const double *gscale, const T *y_in, T *y_out, T *P0, T *P1, T *Tb,
              hipStream_t s, Counters *cnt, double *bytes = nullptr,
              int64_t *launches = nullptr) {
  ChainEmitter<T> em(A, s, cnt, bytes, launches);
  const int K = (int)steps.size();
  const T *cur = g;
  const double *cs = gscale;
  const T *yi = y_in;
  T *bufs[2] = {P0, P1};
  int pb = 0;
  for (int k = 0; k < K; ++k) {
    const ppn::Step &st = steps[k];
    const bool last = (k == K - 1);
    const bool fold = (k + 2 == K) && steps[k + 1].kind == 0;
    const double cf = fold ? steps[k + 1].c1 : 0.0;
    if (st.kind == 0) {
      if (last) {  // only for a single real root
        PP_TRY_HIP(ppk::launch_axpy<T>(A.n, st.c1, cur, cs, yi, y_out, s));
        break;
      }
      ppk::ChainArgs<T> a{cur, cs, nullptr, nullptr, fold ? nullptr : bufs[pb], yi, y_out,
                          st.c1, 0.0, cf};
      PP_TRY(em.chain(0, fold, false, a, (yi ? 1 : 0) + 1 + (fold ? 0 : 1)));
      yi = y_out;
      if (fold) break;
      cur = bufs[pb];
      cs = nullptr;
      pb ^= 1;
    } else {
      ppk::ChainArgs<T> a{cur, cs, nullptr, nullptr, last ? nullptr : Tb, yi, y_out,
                          st.c1, st.c2, 0.0};
      PP_TRY(em.chain(1, false, last, a, (yi ? 1 : 0) + 1 + (last ? 0 : 1)));
      yi = y_out;
      if (last) break;
      ppk::ChainArgs<T> b{Tb, nullptr, cur, cs, fold ? nullptr : bufs[pb], yi, y_out,
                          st.c1, st.c2, cf};
      PP_TRY(em.chain(2, fold, false, b, 1 + (fold ? 2 : 1)));
      if (fold) break;
      cur = bufs[pb];
      cs = nullptr;
      pb ^= 1;
    }
  }
  return em.finish();
}

// out = p(A) (gscale * g) for p(A) = sum_k c[k] A^k by Horner's rule,
// z <- A z + c[k] v from the top coefficient down: deg fused product + axpy
// launches (one axpy launch for a constant polynomial).
template <typename T>
int run_horner(const Opr<T> &A, const std::vector<double> &c, const T *g, const double *gscale,
               T *out, T *P0, T *P1, hipStream_t s, Counters *cnt, double *bytes = nullptr,
               int64_t *launches = nullptr) {
  const int deg = (int)c.size() - 1;
  if (deg < 0) return PP_ERR_ARG;
  if (deg == 0) {
    PP_TRY_HIP(ppk::launch_axpy<T>(A.n, c[0], g, gscale, nullptr, out, s));
    return PP_OK;
  }
  ChainEmitter<T> em(A, s, cnt, bytes, launches);
  T *bufs[2] = {P0, P1};
  int pb = 0;
  const T *z = g;
  const double *zs = gscale;
  for (int k = deg - 1; k >= 0; --k) {
    T *dst = (k == 0) ? out : bufs[pb];
    ppk::ChainArgs<T> a{z, zs, g, gscale, dst, nullptr, nullptr, c[k],
                        k == deg - 1 ? c[deg] : 1.0, 0.0, nullptr};
    PP_TRY(em.chain(4, false, false, a, 2));
    z = dst;
    zs = nullptr;
    pb ^= 1;
  }
  return em.finish();
}

// w_out = A p(A) (gscale * g), evaluated as v - pi(A) v with v = gscale * g:
// one fused root-update launch per real root (p' = p - A p / theta) and two per
// conjugate pair (t = A p, then p' = p - c1 t + c2 A t), the last launch writing
// v - p' instead of p'.  d products, no accumulator vector.
template <typename T>
int run_op_chain(const Opr<T> &A, const std::vector<ppn::Step> &steps, const T *g,
                 const double *gscale, T *w_out, T *P0, T *P1, T *Tb, hipStream_t s,
                 Counters *cnt, double *bytes = nullptr, int64_t *launches = nullptr) {
  ChainEmitter<T> em(A, s, cnt, bytes, launches);
  const int K = (int)steps.size();
  const T *cur = g;
  const double *cs = gscale;
  T *bufs[2] = {P0, P1};
  int pb = 0;
  for (int k = 0; k < K; ++k) {
    const ppn::Step &st = steps[k];
    const bool last = (k == K - 1);
    T *dst = last ? w_out : bufs[pb];
    if (st.kind == 0) {
      ppk::ChainArgs<T> a{cur, cs, nullptr, nullptr, dst, last ? g : nullptr, nullptr,
                          st.c1, 0.0, 0.0, last ? gscale : nullptr};
      PP_TRY(em.chain(3, false, last, a, 1 + (last ? 1 : 0)));
    } else {
      PP_TRY(em.product(cur, cs, Tb, 1));
      ppk::ChainArgs<T> b{Tb, nullptr, cur, cs, dst, last ? g : nullptr, nullptr,
                          st.c1, st.c2, 0.0, last ? gscale : nullptr};
      PP_TRY(em.chain(2, false, last, b, 2 + (last ? 1 : 0)));
    }
    cur = dst;
    cs = nullptr;
    pb ^= 1;
  }
  return em.finish();
}

template <typename T>
constexpr bool is_f32() {
  return sizeof(T) == sizeof(float);
}

// out = w_in - V(:, 0..nc) coef (chunks of kMaxCols columns); optional norm of out,
// whose partials' workgroup count is returned in *G.
template <typename T>
int update_any(Work<T> &w, int nc, const double *coef, const T *w_in, T *out, bool norm,
               hipStream_t s, int *G, bool cached = false) {
  const int rpt =
      orth_rpt(kOrthWrite, std::min(nc, ppk::kMaxCols), is_f32<T>(), w.n);
  for (int c0 = 0; c0 < nc; c0 += ppk::kMaxCols) {
    const int cc = std::min(ppk::kMaxCols, nc - c0);
    const bool lastc = (c0 + cc >= nc);
    PP_TRY_HIP(ppk::launch_update<T>(w.n, rpt, w.V + (int64_t)c0 * w.ldv, w.ldv, cc, coef + c0,
                                     nullptr, 1.0, c0 == 0 ? w_in : out, out, false,
                                     norm && lastc, w.partial, s, nullptr, cached));
  }
  if (G) *G = ppk::orth_grid(w.n, rpt);
  return PP_OK;
}

// partial dots of vec with V(:, 0..nc); *G receives the partials' workgroup count.
template <typename T>
int dots_any(Work<T> &w, int nc, const T *vec, hipStream_t s, int *G, bool cached = false) {
  const int rpt =
      orth_rpt(kOrthRead, std::min(nc, ppk::kMaxCols), is_f32<T>(), w.n);
  for (int c0 = 0; c0 < nc; c0 += ppk::kMaxCols) {
    const int cc = std::min(ppk::kMaxCols, nc - c0);
    PP_TRY_HIP(ppk::launch_dots<T>(w.n, rpt, w.V, w.ldv, c0, cc, vec, w.partial, s, nullptr,
                                   cached));
  }
  *G = ppk::orth_grid(w.n, rpt);
  return PP_OK;
}

// The device part of Arnoldi step j: w = Op(V_j), two CGS passes, V_{j+1} =
// w / ||w||, column j of Hbar (h1 | h2 | nrm) written to the pinned host slot
// w.hslot(j) and the slot's event recorded.  Nothing waits on the host, so step
// j + 1 can be issued before step j is collected: its input V_{j+1} is made on the
// device, and it writes the other slot.
template <typename T>
int arnoldi_issue(const Opr<T> &A, const PolyRef &pr, int op_form, Work<T> &w, int j,
                  hipStream_t s, Timers &tm, Counters &cnt) {
  const T *vj = w.V + (int64_t)j * w.ldv;
  const double *sj = w.colscale + j;
  tm.slot = j & 1;
  tm.mark(0, s);
  if (pr.active() && !pr.power() && op_form == PP_OP_RESIDUAL_POLY) {
    PP_TRY(run_op_chain<T>(A, *pr.steps, vj, sj, w.W, w.P0, w.P1, w.Tb, s, &cnt,
                           &cnt.bytes_chain, &cnt.launches_chain));
    tm.mark(1, s);
  } else {
    if (pr.active()) {
      if (pr.power())
        PP_TRY(run_horner<T>(A, *pr.coeffs, vj, sj, w.Z, w.P0, w.P1, s, &cnt, &cnt.bytes_chain,
                             &cnt.launches_chain));
      else
        PP_TRY(run_chain<T>(A, *pr.steps, vj, sj, nullptr, w.Z, w.P0, w.P1, w.Tb, s, &cnt,
                            &cnt.bytes_chain, &cnt.launches_chain));
      tm.mark(1, s);
      PP_TRY(op_product<T>(A, w.Z, nullptr, w.W, s));
    } else {
      tm.mark(1, s);
      PP_TRY(op_product<T>(A, vj, sj, w.W, s));
    }
    cnt.spmvs++;
    cnt.bytes_spmv += product_bytes(A, 1);
  }
  tm.mark(2, s);
  const int nc = j + 1;
  const int L = w.L;
  double *h1 = w.hbuf, *h2 = w.hbuf + L, *nrm = w.hbuf + 2 * L;
  T *vnext = w.V + (int64_t)(j + 1) * w.ldv;
  // With few partials (small n) each sweep's last workgroup also does the second
  // reduction stage, bitwise as the separate launch would (ppk::FoldOut).
  const bool one_chunk = nc <= ppk::kMaxCols;
  const bool may_fold = one_chunk && w.fold_ok;
  // the step's three sweeps re-read the same nc basis columns: ordinary loads when
  // they (and w) fit the cache budget, so the second and third sweeps find them there
  const bool keep = (double)(nc + 2) * (double)w.ldv * sizeof(T) <= kCacheBudget;
  const int rpt1 =
      orth_rpt(kOrthRead, std::min(nc, ppk::kMaxCols), is_f32<T>(), w.n);
  const int rpt2 = orth_rpt(kOrthUpdateDots, nc, is_f32<T>(), w.n);
  const int rpt3 =
      orth_rpt(kOrthWrite, std::min(nc, ppk::kMaxCols), is_f32<T>(), w.n);
  const bool fold1 = may_fold && ppk::orth_grid(w.n, rpt1) <= ppk::kFoldMaxG;
  const bool fold2 = may_fold && ppk::orth_grid(w.n, rpt2) <= ppk::kFoldMaxG;
  const bool fold3 = may_fold && ppk::orth_grid(w.n, rpt3) <= ppk::kFoldMaxG;
  if ((fold1 || fold2 || fold3) && !w.fold_armed) {
    PP_TRY_HIP(ppk::launch_fill<int32_t>(1, 0, w.fold_counter, s));
    w.fold_armed = true;
  }
  // pass 1: h1 = V^T w
  int G1 = 0, G2 = 0, G3 = 0;
  if (fold1) {
    const ppk::FoldOut f{w.fold_counter, w.colscale, h1, w.coef1};
    PP_TRY_HIP(ppk::launch_dots<T>(w.n, rpt1, w.V, w.ldv, 0, nc, w.W, w.partial, s, &f));
  } else {
    PP_TRY(dots_any<T>(w, nc, w.W, s, &G1, keep));
    PP_TRY_HIP(ppk::launch_reduce_cols(w.partial, G1, 0, nc, w.colscale, h1, w.coef1, s));
  }
  if (one_chunk) {
    // w -= V h1, fused with pass 2's dots
    const ppk::FoldOut f{w.fold_counter, w.colscale, h2, w.coef2};
    PP_TRY_HIP(ppk::launch_update<T>(w.n, rpt2, w.V, w.ldv, nc, w.coef1, nullptr, 1.0, w.W, w.W,
                                     true, false, w.partial, s, fold2 ? &f : nullptr, keep));
    G2 = ppk::orth_grid(w.n, rpt2);
  } else {
    PP_TRY(update_any<T>(w, nc, w.coef1, w.W, w.W, false, s, nullptr));
    PP_TRY(dots_any<T>(w, nc, w.W, s, &G2));
  }
  if (!fold2)
    PP_TRY_HIP(ppk::launch_reduce_cols(w.partial, G2, 0, nc, w.colscale, h2, w.coef2, s));
  // pass 2 update, norm, store as column j+1
  // the norm's second stage also hands the column (h1 | h2 | nrm) to the pinned host
  // buffer, so the step needs no separate device-to-host copy
  const int hcount = 2 * L + 1;
  if (fold3) {
    ppk::FoldOut f;
    f.counter = w.fold_counter;
    f.nrm = nrm;
    f.inv = w.colscale + j + 1;
    f.copy_src = w.hbuf;
    f.copy_dst = w.hslot(j);
    f.copy_n = hcount;
    f.nrm_at = 2 * L;
    PP_TRY_HIP(ppk::launch_update<T>(w.n, rpt3, w.V, w.ldv, nc, w.coef2, nullptr, 1.0, w.W,
                                     vnext, false, true, w.partial, s, &f));
  } else {
    PP_TRY(update_any<T>(w, nc, w.coef2, w.W, vnext, true, s, &G3, keep));
    PP_TRY_HIP(ppk::launch_reduce_norm(w.partial, G3, nrm, w.colscale + j + 1, s, w.hbuf,
                                       w.hslot(j), hcount, 2 * L));
  }
  cnt.dots += 3;
  // three sweeps over nc basis columns; w read three times and written twice
  cnt.bytes_orth += (double)sizeof(T) * w.n * (3.0 * nc + 5.0);
  tm.mark(3, s);
  PP_TRY_HIP(hipEventRecord(w.step_ev[j & 1], s));
  return PP_OK;
}

// The host part of Arnoldi step j (issued by arnoldi_issue): waits for its slot,
// hcol[0..j+1] receives column j of Hbar and *w0 an estimate of ||Op(V_j)||.
// Returns PP_OK, or PP_WARN_NONFINITE when a coefficient is not finite.
template <typename T>
int arnoldi_collect(Work<T> &w, int j, Timers &tm, double *hcol, double *w0) {
  PP_TRY_HIP(hipEventSynchronize(w.step_ev[j & 1]));
  const int nc = j + 1, L = w.L;
  const double *h = w.hslot(j);
  double a2 = 0.0;
  bool ok = true;
  for (int i = 0; i < nc; ++i) {
    const double x1 = h[i], x2 = h[L + i];
    hcol[i] = x1 + x2;
    a2 += x1 * x1 + x2 * x2;
    ok = ok && finite(x1) && finite(x2);
  }
  const double hn = h[2 * L];
  hcol[j + 1] = hn;
  *w0 = std::sqrt(a2 + hn * hn);
  tm.collect(j & 1);
  return (ok && finite(hn)) ? PP_OK : PP_WARN_NONFINITE;
}

// Device work of the step issued ahead, in the counters, so that it can be taken
// back when the cycle stops before that step.
struct IssueCounts {
  int64_t spmvs = 0, dots = 0, launches_chain = 0;
  double bytes_chain = 0, bytes_spmv = 0, bytes_orth = 0;
  static IssueCounts of(const Counters &c) {
    return IssueCounts{c.spmvs, c.dots, c.launches_chain, c.bytes_chain, c.bytes_spmv,
                       c.bytes_orth};
  }
};

// Lookahead: a step's device work is issued before the previous step is collected
// (the host's wait, least squares and launches then overlap the device), when a
// step is short enough that the host's share matters (at most kLookaheadBytes of
// estimated traffic).  When the cycle stops at step j, a step j + 1 already issued
// is wasted device work (its results are never read; V(:, j + 2) is past the
// cycle's columns), one step per stop.  PP_LOOKAHEAD=0 turns it off.
constexpr double kLookaheadBytes = 512.0 * 1024 * 1024;


template <typename T>
struct StepPipe {
  const Opr<T> &A;
  const PolyRef &pr;
  int op_form;
  Work<T> &w;
  hipStream_t s;
  Timers &tm;
  Counters &cnt;
  int issued = -1;  // highest step issued
  IssueCounts before, after;  // counters around the last issue

  double step_bytes(int j) const {
    int products = 1;
    if (pr.power()) {
      products += (int)pr.coeffs->size() - 1;
    } else if (pr.active()) {
      for (const ppn::Step &st : *pr.steps) products += st.kind == 0 ? 1 : 2;
    }
    return products * product_bytes(A, 1) + (double)sizeof(T) * w.n * (3.0 * (j + 1) + 5.0);
  }
  int issue(int j) {
    before = IssueCounts::of(cnt);
    PP_TRY(arnoldi_issue<T>(A, pr, op_form, w, j, s, tm, cnt));
    after = IssueCounts::of(cnt);
    issued = j;
    return PP_OK;
  }
  // Step j's column, with step j + 1 (< jmax) issued first when lookahead applies.
  int next(int j, int jmax, double *hcol, double *w0) {
    if (issued < j) PP_TRY(issue(j));
    if (j + 1 < jmax && w.lookahead_ok && step_bytes(j + 1) <= kLookaheadBytes)
      PP_TRY(issue(j + 1));
    return arnoldi_collect<T>(w, j, tm, hcol, w0);
  }
  // The caller stops after step j: a step issued past it leaves the counters.
  void stop(int j) {
    if (issued <= j) return;
    cnt.spmvs -= after.spmvs - before.spmvs;
    cnt.dots -= after.dots - before.dots;
    cnt.launches_chain -= after.launches_chain - before.launches_chain;
    cnt.bytes_chain -= after.bytes_chain - before.bytes_chain;
    cnt.bytes_spmv -= after.bytes_spmv - before.bytes_spmv;
    cnt.bytes_orth -= after.bytes_orth - before.bytes_orth;
    issued = j;
  }
};

// Start column: V(:,0) = (T) src (device double), colscale[0] = 1/||.||; returns the norm.
template <typename T>
int start_from_vector(Work<T> &w, const double *src, hipStream_t s, double *beta) {
  PP_TRY_HIP(ppk::launch_copy_from_f64<T>(w.n, src, w.V, s));
  const int rpt = orth_rpt(kOrthRead, 1, is_f32<T>(), w.n);
  PP_TRY_HIP(ppk::launch_norm2<T>(w.n, rpt, w.V, nullptr, nullptr, w.partial, s));
  PP_TRY_HIP(ppk::launch_reduce_norm(w.partial, ppk::orth_grid(w.n, rpt), w.misc, w.colscale,
                                     s));
  PP_TRY_HIP(hipMemcpyAsync(w.host, w.misc, sizeof(double), hipMemcpyDeviceToHost, s));
  PP_TRY_HIP(hipStreamSynchronize(s));
  *beta = w.host[0];
  return PP_OK;
}

// d Arnoldi steps on v0, harmonic Ritz values, Leja order, step table.
template <typename T>
int build_poly_impl(const Opr<T> &A, const double *v0, int d, Work<T> &w, hipStream_t s,
                    Counters &cnt, Timers &tm, pp_poly *out) {
  double beta = 0.0;
  PP_TRY(start_from_vector<T>(w, v0, s, &beta));
  cnt.dots += 1;
  if (!(beta > 0.0) || !finite(beta)) return PP_ERR_SINGULAR;
  const int ldh = d + 1;
  std::vector<double> Hbar((size_t)ldh * d, 0.0), hcol(d + 1);
  int sdim = d;
  const PolyRef none{};
  StepPipe<T> pipe{A, none, 0, w, s, tm, cnt};
  tm.start();
  for (int j = 0; j < d; ++j) {
    double w0 = 0.0;
    int rc = pipe.next(j, d, hcol.data(), &w0);
    if (rc < 0) return rc;
    if (rc == PP_WARN_NONFINITE) return PP_ERR_SINGULAR;
    for (int i = 0; i <= j + 1; ++i) Hbar[i + (size_t)j * ldh] = hcol[i];
    if (hcol[j + 1] <= kBreakdownRtol * w0) {
      sdim = j + 1;
      pipe.stop(j);
      break;
    }
  }
  std::vector<double> wr, wi, lr, li;
  PP_TRY(ppn::harmonic_ritz(Hbar.data(), ldh, sdim, wr, wi));
  PP_TRY(ppn::leja_order(wr, wi, lr, li));
  std::vector<ppn::Step> steps;
  PP_TRY(ppn::step_table(lr, li, steps));
  out->n = A.n;
  out->re = lr;
  out->im = li;
  out->steps = steps;
  return sdim < d ? PP_WARN_DEGREE_REDUCED : PP_OK;
}

// The paper's construction (Section II, eqs. (1)-(2)): V = [v0, A v0, ...,
// A^(deg+1) v0] (deg+1 products, columns left unnormalised as the power basis
// is), the Gram matrix W^T W and right-hand side W^T v0 of W = A V(:, 0..deg)
// from one multi-dot per column, then a host Cholesky.  With auto_degree the
// leading blocks are factored in increasing order and the highest degree
// without a Cholesky failure is kept (Section IV); otherwise a failure at column
// k keeps the solution of the leading (k-1) block, zeros above, and warns.
template <typename T>
int build_power_impl(const Opr<T> &A, const double *v0, int deg, bool auto_deg, Work<T> &w,
                     double *gram, hipStream_t s, Counters &cnt, pp_poly *out, int *info_out) {
  const int L = deg + 2;
  PP_TRY_HIP(ppk::launch_copy_from_f64<T>(w.n, v0, w.V, s));
  for (int k = 1; k < L; ++k) {
    PP_TRY(op_product<T>(A, w.V + (int64_t)(k - 1) * w.ldv, nullptr, w.V + (int64_t)k * w.ldv,
                         s));
    cnt.spmvs++;
  }
  for (int j = 1; j < L; ++j) {
    int G = 0;
    PP_TRY(dots_any<T>(w, j + 1, w.V + (int64_t)j * w.ldv, s, &G));
    PP_TRY_HIP(ppk::launch_reduce_cols(w.partial, G, 0, j + 1, nullptr, gram + (size_t)j * L,
                                       nullptr, s));
  }
  cnt.dots += 2;  // the paper's two block inner products
  std::vector<double> g((size_t)L * L);
  PP_TRY_HIP(hipMemcpyAsync(g.data(), gram, g.size() * sizeof(double), hipMemcpyDeviceToHost,
                            s));
  PP_TRY_HIP(hipStreamSynchronize(s));
  // G(a, b) = V(:, a+1) . V(:, b+1), rhs(a) = V(:, a+1) . V(:, 0), a, b = 0..deg
  const int K = deg + 1;
  std::vector<double> G((size_t)K * K), rhs(K);
  for (int b = 0; b < K; ++b) {
    rhs[b] = g[(size_t)(b + 1) * L];
    for (int a = 0; a <= b; ++a) {
      G[a + (size_t)b * K] = G[b + (size_t)a * K] = g[(a + 1) + (size_t)(b + 1) * L];
    }
  }
  for (double v : G)
    if (!finite(v)) return PP_ERR_SINGULAR;
  std::vector<double> R;
  int keep = K, info = 0;
  if (auto_deg) {
    keep = 0;
    for (int k = 1; k <= K; ++k) {
      const int rc = ppn::cholesky_upper(G.data(), K, k, R);
      if (rc) {
        info = rc;
        break;
      }
      keep = k;
    }
  } else {
    info = ppn::cholesky_upper(G.data(), K, K, R);
    if (info) keep = info - 1;
  }
  if (keep == 0) return PP_ERR_SINGULAR;
  PP_TRY(ppn::cholesky_upper(G.data(), K, keep, R) ? PP_ERR_SINGULAR : PP_OK);
  out->kind = 1;
  out->n = A.n;
  out->coeffs.assign(auto_deg ? keep : K, 0.0);
  ppn::cholesky_solve(R, keep, rhs.data(), out->coeffs.data());
  out->info = info;
  if (info_out) *info_out = info;
  return (!auto_deg && info) ? PP_WARN_CHOLESKY : PP_OK;
}

// Givens least squares state of one cycle.
struct Lsq {
  int m;
  std::vector<double> R, cs, sn, g;
  explicit Lsq(int m_) : m(m_), R((size_t)(m_ + 1) * m_, 0.0), cs(m_), sn(m_), g(m_ + 1, 0.0) {}
  // add column j (length j+2); returns |g_{j+1}|
  double add(int j, double *h) {
    for (int i = 0; i < j; ++i) {
      const double t = cs[i] * h[i] + sn[i] * h[i + 1];
      h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
      h[i] = t;
    }
    const double a = h[j], b = h[j + 1];
    double c = 1.0, sv = 0.0, r = a;
    if (b != 0.0) {
      r = std::hypot(a, b);
      c = a / r;
      sv = b / r;
    }
    cs[j] = c;
    sn[j] = sv;
    h[j] = r;
    h[j + 1] = 0.0;
    for (int i = 0; i <= j; ++i) R[i + (size_t)j * (m + 1)] = h[i];
    g[j + 1] = -sv * g[j];
    g[j] = c * g[j];
    return std::fabs(g[j + 1]);
  }
  void solve(int k, double *y) const {
    for (int i = k - 1; i >= 0; --i) {
      double acc = g[i];
      for (int c = i + 1; c < k; ++c) acc -= R[i + (size_t)c * (m + 1)] * y[c];
      y[i] = acc / R[i + (size_t)i * (m + 1)];
    }
  }
};

// One GMRES(m) cycle from V(:,0) (colscale[0] set) with start residual norm beta.
// Returns steps taken in *k and the solution coefficients in y.
template <typename T>
int gmres_cycle(const Opr<T> &A, const PolyRef &pr, int op_form, Work<T> &w, int m,
                double beta, double tol_abs, double bscale, int max_steps, hipStream_t s,
                Timers &tm, Counters &cnt, std::vector<double> &y, int *k, double *res,
                bool *nonfinite) {
  Lsq ls(m);
  ls.g[0] = beta;
  std::vector<double> hcol(m + 2);
  *k = 0;
  *res = beta;
  *nonfinite = false;
  const int jmax = std::min(m, max_steps);
  StepPipe<T> pipe{A, pr, op_form, w, s, tm, cnt};
  tm.start();
  for (int j = 0; j < jmax; ++j) {
    double w0 = 0.0;
    int rc = pipe.next(j, jmax, hcol.data(), &w0);
    if (rc < 0) return rc;
    cnt.iters++;
    if (rc == PP_WARN_NONFINITE) {
      *nonfinite = true;
      pipe.stop(j);
      break;
    }
    const double hn = hcol[j + 1];
    *res = ls.add(j, hcol.data());
    *k = j + 1;
    cnt.push(*res / bscale);
    if (log_level() >= 2)
      std::fprintf(stderr, "[pp] step %d (cycle step %d): implicit relres %.3e\n", cnt.iters,
                   j + 1, *res / bscale);
    if (!finite(*res)) {
      *nonfinite = true;
      pipe.stop(j);
      break;
    }
    if (hn <= kBreakdownRtol * w0 || *res < tol_abs) {
      pipe.stop(j);
      break;
    }
  }
  y.assign(std::max(*k, 1), 0.0);
  if (*k > 0 && !*nonfinite) {
    ls.solve(*k, y.data());
    for (int i = 0; i < *k; ++i)
      if (!finite(y[i])) *nonfinite = true;
  }
  return PP_OK;
}

// x_out = x_in + p(A) V(:,0..k) (colscale o y)   [x_in may equal x_out, or be nullptr]
template <typename T>
int cycle_update(const Opr<T> &A, const PolyRef &pr, Work<T> &w, int k,
                 const std::vector<double> &y, const T *x_in, T *x_out, hipStream_t s,
                 Counters &cnt) {
  if (k <= 0) return PP_OK;
  std::memcpy(w.ystage(), y.data(), k * sizeof(double));
  PP_TRY_HIP(hipMemcpyAsync(w.ybuf, w.ystage(), k * sizeof(double),
                            hipMemcpyHostToDevice, s));
  const bool poly = pr.active();
  const int rpt =
      orth_rpt(kOrthWrite, std::min(k, ppk::kMaxCols), is_f32<T>(), w.n);
  for (int c0 = 0; c0 < k; c0 += ppk::kMaxCols) {
    const int cc = std::min(ppk::kMaxCols, k - c0);
    T *dst = poly ? w.U : x_out;
    const T *src = poly ? (c0 == 0 ? nullptr : w.U) : (c0 == 0 ? x_in : x_out);
    PP_TRY_HIP(ppk::launch_update<T>(w.n, rpt, w.V + (int64_t)c0 * w.ldv, w.ldv, cc,
                                     w.ybuf + c0, w.colscale + c0, -1.0, src, dst, false, false,
                                     w.partial, s));
  }
  if (poly && pr.power()) {
    PP_TRY(run_horner<T>(A, *pr.coeffs, w.U, nullptr, w.Z, w.P0, w.P1, s, &cnt));
    PP_TRY_HIP(ppk::launch_axpy<T>(A.n, 1.0, w.Z, nullptr, x_in, x_out, s));
  } else if (poly) {
    PP_TRY(run_chain<T>(A, *pr.steps, w.U, nullptr, x_in, x_out, w.P0, w.P1, w.Tb, s, &cnt));
  }
  // the host staging of y must not be reused before the copy has run
  PP_TRY_HIP(hipStreamSynchronize(s));
  return PP_OK;
}

int check_csr(const pp_csr *A) {
  if (!A || A->n <= 0 || A->nnz < 0 || A->n >= (int64_t)1 << 31 || A->nnz >= (int64_t)1 << 31)
    return PP_ERR_ARG;
  if (!A->row_ptr || (A->nnz > 0 && (!A->col_ind || !A->vals))) return PP_ERR_ARG;
  if (A->dtype != PP_F64 && A->dtype != PP_F32) return PP_ERR_ARG;
  if (A->layout != PP_LAYOUT_AUTO && A->layout != PP_LAYOUT_CSR && A->layout != PP_LAYOUT_SELL)
    return PP_ERR_ARG;
  return PP_OK;
}

// The CSR structure checked on the device before any kernel indexes with it
// (row_ptr from 0 to nnz and nondecreasing, every column in [0, n)): a
// malformed matrix is PP_ERR_ARG, never an out-of-bounds access.  One pass over
// row_ptr and col_ind and one synchronisation.  Uses the head of the arena.
// bad: one device int32 (cleared here), h: one host int32.
int check_csr_on_device(const pp_csr *A, int32_t *bad, int32_t *h, hipStream_t s) {
  PP_TRY_HIP(ppk::launch_fill<int32_t>(1, 0, bad, s));
  PP_TRY_HIP(ppk::launch_check_csr((int)A->n, (int)A->nnz, A->row_ptr, A->col_ind, bad, s));
  PP_TRY_HIP(hipMemcpyAsync(h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PP_TRY_HIP(hipStreamSynchronize(s));
  return *h ? PP_ERR_ARG : PP_OK;
}

int validate_csr(const pp_csr *A, hipStream_t s) {
  Arena *ar = nullptr;
  PP_TRY(current_arena(&ar));
  PP_TRY(ensure_arena(ar, 256, 64));
  return check_csr_on_device(A, reinterpret_cast<int32_t *>(ar->dev),
                             reinterpret_cast<int32_t *>(ar->host), s);
}

// The sliced copy of a call's matrix (see SpMat): built on the device from the
// CSR arrays into the arena's matrix buffer.  `use` is false when the caller
// asked for CSR, when the stored slots would not fit int32 offsets, or
// (PP_LAYOUT_AUTO) when one product would stream more than 1.25 times the bytes
// of the CSR product, or when the call's `products` sparse products cannot
// repay the copy: each is credited with the bytes it saves (at least 5% of the
// CSR product, the sliced kernels' better bandwidth), against the bytes the
// conversion moves.
struct SellCopy {
  bool use = false;
  int64_t snnz = 0, ell = 0, extra = 0;
  int dmax = 0;
  int32_t *desc = nullptr, *soff = nullptr, *sci = nullptr;
  double *va64 = nullptr;
  float *va32 = nullptr;
};

// want64 / want32: value arrays to fill (FP64 from A's values; FP32 from src32
// when given, else from A's values).  Uses the main arena as scratch, so call it
// before carving the solve's workspace.
int make_sell(const pp_csr *A, bool want64, bool want32, const float *src32, double products,
              hipStream_t s, SellCopy *out) {
  *out = SellCopy{};
  if (A->layout == PP_LAYOUT_CSR) return PP_OK;
  const int n = (int)A->n;
  const double vb = A->dtype == PP_F64 ? 8.0 : 4.0;
  const double csr = A->nnz * (vb + 4.0) + 4.0 * (n + 1);
  const double idx_pass = 4.0 * A->nnz + 4.0 * (n + 1);  // one read of row_ptr and col_ind
  const int nvals = (want64 ? 1 : 0) + (want32 ? 1 : 0);
  if (A->layout == PP_LAYOUT_AUTO) {
    // best case: every slice diagonal without padding (8 or 4 bytes per entry)
    const double conv_min = 3.0 * idx_pass + nvals * (vb + 4.0) * A->nnz;
    if (products * (csr - vb * A->nnz) < conv_min) return PP_OK;
  }
  Arena *ar = nullptr;
  PP_TRY(current_arena(&ar));
  const int ns = (n + ppk::kSlice - 1) / ppk::kSlice;
  Carver meas(nullptr);
  meas.take<int32_t>(ns);
  meas.take<int32_t>(ns + 1);
  meas.take<int32_t>(ns);
  meas.take<int32_t>(ns);
  meas.take<int32_t>(ppk::scan_tmp_size(ns));
  meas.take<int32_t>(64);
  PP_TRY(ensure_arena(ar, meas.off + 256, 64));
  Carver c(ar->dev);
  int32_t *wlen = c.take<int32_t>(ns);
  int32_t *spt = c.take<int32_t>(ns + 1);
  int32_t *flagt = c.take<int32_t>(ns);
  int32_t *wrow = c.take<int32_t>(ns);
  int32_t *tmp = c.take<int32_t>(ppk::scan_tmp_size(ns));
  // [0] longest row, [1] explicit-column slots, [2] most slots of a diagonal slice,
  // [3] diagonal slots past the descriptors
  int32_t *stats = c.take<int32_t>(64);
  PP_TRY_HIP(ppk::launch_slice_plan(n, ns, A->row_ptr, A->col_ind, wlen, flagt, wrow, stats, s));
  PP_TRY_HIP(ppk::launch_exclusive_scan(ns, wlen, spt, tmp, s));
  int32_t *h = reinterpret_cast<int32_t *>(ar->host);
  PP_TRY_HIP(hipMemcpyAsync(h, spt + ns, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PP_TRY_HIP(hipMemcpyAsync(h + 1, stats, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PP_TRY_HIP(hipStreamSynchronize(s));
  const int64_t longest = h[1];
  if ((int64_t)96 * longest * ns >= ((int64_t)1 << 31)) return PP_OK;
  const int64_t snnz = h[0], ell = h[2], dmax = h[3], extra = h[4];
  if (A->layout == PP_LAYOUT_AUTO) {
    const double sliced = snnz * vb + ell * 4.0 + extra * 4.0 + 4.0 * ppk::kDesc * ns;
    const double conv = 3.0 * idx_pass + nvals * vb * A->nnz +
                        snnz * (nvals * vb + (ell > 0 ? 4.0 : 0.0));
    if (sliced > 1.25 * csr || products * std::max(csr - sliced, 0.05 * csr) < conv) return PP_OK;
  }
  const int64_t cap = std::max<int64_t>(snnz, 1);
  // one batch of slack: the product kernel fetches whole batches of offsets
  const int64_t ocap = (int64_t)ns * dmax + ppk::kSellBatch;
  Carver mm(nullptr);
  mm.take<int32_t>((int64_t)ns * ppk::kDesc);
  mm.take<int32_t>(ocap);
  if (ell > 0) mm.take<int32_t>(cap);
  if (want64) mm.take<double>(cap);
  if (want32) mm.take<float>(cap);
  PP_TRY(ensure_side(&ar->mat, &ar->mat_cap, mm.off + 256));
  Carver m(ar->mat);
  out->desc = m.take<int32_t>((int64_t)ns * ppk::kDesc);
  out->soff = m.take<int32_t>(ocap);
  if (ell > 0) out->sci = m.take<int32_t>(cap);
  if (want64) out->va64 = m.take<double>(cap);
  if (want32) out->va32 = m.take<float>(cap);
  // sp and the kinds stay in the scratch arena: only the fills below read them
  PP_TRY_HIP(ppk::launch_slice_fill_idx(n, ns, (int)dmax, A->row_ptr, A->col_ind, spt, flagt,
                                        out->desc, out->soff, out->sci, s));
  if (want64) {
    if (A->dtype != PP_F64) return PP_ERR_ARG;
    PP_TRY_HIP((ppk::launch_slice_fill_vals<double, double>(
        n, ns, A->row_ptr, A->col_ind, static_cast<const double *>(A->vals), spt, flagt,
        out->va64, s)));
  }
  if (want32) {
    if (src32 || A->dtype == PP_F32) {
      const float *src = src32 ? src32 : static_cast<const float *>(A->vals);
      PP_TRY_HIP((ppk::launch_slice_fill_vals<float, float>(n, ns, A->row_ptr, A->col_ind, src,
                                                            spt, flagt, out->va32, s)));
    } else {
      PP_TRY_HIP((ppk::launch_slice_fill_vals<double, float>(
          n, ns, A->row_ptr, A->col_ind, static_cast<const double *>(A->vals), spt, flagt,
          out->va32, s)));
    }
  }
  out->use = true;
  out->snnz = snnz;
  out->ell = ell;
  out->dmax = (int)dmax;
  out->extra = extra;
  return PP_OK;
}

// Attach the sliced copy (when built) to a view of type T.
template <typename T>
SpMat<T> with_sell(SpMat<T> M, const SellCopy &c) {
  if (!c.use) return M;
  M.sdesc = c.desc;
  M.soff = c.soff;
  M.sci = c.sci;
  if constexpr (sizeof(T) == sizeof(double)) M.sva = c.va64;
  else M.sva = c.va32;
  M.snnz = (int)c.snnz;
  M.snnz_ell = (int)c.ell;
  M.dmax = c.dmax;
  M.soff_extra = (int)c.extra;
  return M;
}

void note_layout(pp_stats *st, const pp_csr *A, const SellCopy &c) {
  if (!st) return;
  st->layout_used = c.use ? PP_LAYOUT_SELL : PP_LAYOUT_CSR;
  st->nnz_stored = c.use ? c.snnz : A->nnz;
}

template <typename T>
SpMat<T> view(const pp_csr *A, const void *vals) {
  return SpMat<T>{(int)A->n, (int)A->nnz, A->row_ptr, A->col_ind, static_cast<const T *>(vals)};
}

// Cache policy and order of an operator's chain launches (Section VII's reuse of
// the matrix across several products): the Arnoldi step's operator, the
// cycle-end update and pp_apply's product form, the power basis' Horner chain.
// One launch streams its matrix rows and two vectors; when all of that fits
// kCacheBudget, group 0 (automatic) runs full-range launches with cached loads and
// stores, so each launch finds the matrix where the previous one left it.  Larger
// matrices get the slab-skewed order over all of a chain's launches with slabs
// that fit the budget, when the bandwidth (one pass over csr's column indices) is
// small beside a slab; otherwise full-range, non-temporal launches.  group 1:
// full-range, non-temporal; >= 2: the slab-skewed order with that group and
// slab_rows (0: budget-sized slabs).  Not for M^-1 A (M^-1 couples all rows).
template <typename T>
int choose_schedule(Opr<T> &A, const pp_csr *csr, int group, int slab_rows, int32_t *scratch,
                    hipStream_t s) {
  if (A.ilu || group == 1) return PP_OK;
  const double per_row = product_bytes(A, 1) / (double)A.n;
  const int64_t tr = ppk::chain_tile_rows(A);
  const int64_t fit = std::max<int64_t>(tr, (int64_t)(kCacheBudget / per_row) / tr * tr);
  if (group == 0 && fit >= A.n) {
    A.keep = true;
    return PP_OK;
  }
  const int slab = slab_rows > 0 ? slab_rows : (int)std::min<int64_t>(fit, 1 << 30);
  PP_TRY_HIP(ppk::launch_fill<int32_t>(1, 0, scratch, s));
  PP_TRY_HIP(ppk::launch_bandwidth(A.n, csr->row_ptr, csr->col_ind, scratch, s));
  int32_t bw = 0;
  PP_TRY_HIP(hipMemcpyAsync(&bw, scratch, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PP_TRY_HIP(hipStreamSynchronize(s));
  if (group == 0) {
    if ((int64_t)bw * kSlabPerBandwidth > slab) return PP_OK;
    A.blk_group = kAllLaunches;
  } else {
    A.blk_group = group;
  }
  A.blk_slab_rows = slab;
  A.blk_bw_rows = bw;
  return PP_OK;
}

// y = p(A) v on operator M with three n-entry temporaries (the chain's or, for a
// power-basis polynomial, Horner's).
template <typename T>
int apply_run(const Opr<T> &M, const pp_poly *p, const T *v, T *y, T *const bufs[3],
              hipStream_t s) {
  if (p->kind == 1) {
    PP_TRY(run_horner<T>(M, p->coeffs, v, nullptr, y, bufs[0], bufs[1], s, nullptr));
  } else if (p->steps.empty()) {
    PP_TRY_HIP(ppk::launch_fill<T>(M.n, T(0), y, s));
  } else {
    PP_TRY(run_chain<T>(M, p->steps, v, nullptr, nullptr, y, bufs[0], bufs[1], bufs[2], s,
                        nullptr));
  }
  return PP_OK;
}

template <typename T>
int apply_impl(const pp_csr *A, const pp_poly *p, const void *v, void *y, hipStream_t s) {
  Arena *ar = nullptr;
  PP_TRY(current_arena(&ar));
  const int n = (int)A->n;
  SellCopy sc;
  const double products = p->kind == 1 ? (double)p->coeffs.size() - 1.0 : (double)p->steps.size();
  if (products > 0) PP_TRY(make_sell(A, sizeof(T) == 8, sizeof(T) == 4, nullptr, products, s, &sc));
  Carver meas(nullptr);
  T *bufs[3];
  for (auto &b : bufs) b = meas.take<T>(pad_ld(n));
  int32_t *isc = meas.take<int32_t>(64);
  PP_TRY(ensure_arena(ar, meas.off + 256, 64));
  Carver c(ar->dev);
  for (auto &b : bufs) b = c.take<T>(pad_ld(n));
  isc = c.take<int32_t>(64);
  Opr<T> M(with_sell(view<T>(A, A->vals), sc));
  if (products > 0) PP_TRY(choose_schedule<T>(M, A, 0, 0, isc, s));
  PP_TRY(apply_run<T>(M, p, static_cast<const T *>(v), static_cast<T *>(y), bufs, s));
  PP_TRY_HIP(hipStreamSynchronize(s));
  return PP_OK;
}

// pp_apply_noalloc: the same chain on A's CSR arrays, with the three temporaries
// and the check's flag carved from the library's fixed per-GPU array.  Full-range
// launches only (the slab-skewed order keeps its launch list in host memory):
// cached when a product's working set fits the cache budget, else non-temporal,
// the choice choose_schedule makes for group 0 without the slab option.
template <typename T>
int apply_noalloc_impl(const pp_csr *A, const pp_poly *p, const void *v, void *y,
                       hipStream_t s) {
  const int n = (int)A->n;
  void *base = nullptr;
  size_t cap = 0;
  PP_TRY_HIP(ppx::noalloc_scratch(&base, &cap));
  Carver meas(nullptr);
  meas.take<int32_t>(64);
  for (int k = 0; k < 3; ++k) meas.take<T>(pad_ld(n));
  // the stated limit (the array holds a little slack beyond it for alignment)
  const int64_t max_rows = ppx::kNoAllocMaxRowsF64 * (int64_t)(sizeof(double) / sizeof(T));
  if (n > max_rows || meas.off + 256 > cap) {
    ppd::note_msg("pp_apply_noalloc: n = %d needs %zu bytes of scratch, the fixed array holds "
                  "%zu (n <= %lld rows in FP64, %lld in FP32)",
                  n, meas.off + 256, cap, (long long)ppx::kNoAllocMaxRowsF64,
                  (long long)(2 * ppx::kNoAllocMaxRowsF64));
    return PP_ERR_ARG;
  }
  Carver c(static_cast<char *>(base));
  int32_t *flag = c.take<int32_t>(64);
  T *bufs[3];
  for (auto &b : bufs) b = c.take<T>(pad_ld(n));
  int32_t hflag = 0;
  PP_TRY(check_csr_on_device(A, flag, &hflag, s));
  Opr<T> M(view<T>(A, A->vals));
  const double per_row = product_bytes(M, 1) / (double)n;
  M.keep = (double)n * per_row <= kCacheBudget;
  PP_TRY(apply_run<T>(M, p, static_cast<const T *>(v), static_cast<T *>(y), bufs, s));
  PP_TRY_HIP(hipStreamSynchronize(s));
  return PP_OK;
}

template <typename T>
int build_impl(const pp_csr *A, const double *v0, int d, hipStream_t s, pp_poly **out) {
  Arena *ar = nullptr;
  PP_TRY(current_arena(&ar));
  const int n = (int)A->n;
  SellCopy sc;
  PP_TRY(make_sell(A, sizeof(T) == 8, sizeof(T) == 4, nullptr, d, s, &sc));
  Work<T> w;
  Carver meas(nullptr);
  w.carve(meas, n, d + 1);
  double *v0gen = v0 ? nullptr : meas.take<double>(n);
  PP_TRY(ensure_arena(ar, meas.off + 256, w.host_doubles()));
  Carver c(ar->dev);
  w.carve(c, n, d + 1);
  w.attach(*ar);
  if (!v0) {
    v0gen = c.take<double>(n);
    PP_TRY_HIP(ppk::launch_uniform_pm1(n, kDefaultSeed, v0gen, s));
    v0 = v0gen;
  }
  Counters cnt;
  Timers tm;
  pp_poly *p = new pp_poly();
  p->dtype = A->dtype;
  int rc = build_poly_impl<T>(with_sell(view<T>(A, A->vals), sc), v0, d, w, s, cnt, tm, p);
  if (rc < 0) {
    delete p;
    return rc;
  }
  *out = p;
  return rc;
}

// Everything a solve needs from the FP64 side.
struct SolveIn {
  const pp_csr *A;
  const double *b;
  double *x;
  int m, d;
  double tol;
  pp_opts o;
  hipStream_t s;
  const pp_ilu *ilu = nullptr;  // left ILU(0): the operator is M^-1 A and b is M^-1 b
};

// Products with A per application of the preconditioned operator A p(A).
int poly_size(const pp_poly *p) {
  return p->kind == 1 ? (int)p->coeffs.size() : (int)p->re.size();
}

// A lower estimate of a solve's sparse products: the build's d, then one
// restart cycle of m preconditioned steps (d products each) and its cycle end.
double solve_products(const SolveIn &in) {
  const int d = in.o.poly ? poly_size(in.o.poly) : in.d;
  return (double)d + (double)in.m * std::max(d, 1) + (double)d + 1.0;
}

int worst(int a, int b) {
  if (a < 0 || b < 0) return std::min(a, b);
  return std::max(a, b);
}

// ||b|| in FP64 (device) -> host.
int norm_f64(Work<double> &w, const double *x, hipStream_t s, double *out) {
  const int rpt = orth_rpt(kOrthRead, 1, false, w.n);
  PP_TRY_HIP(ppk::launch_norm2<double>(w.n, rpt, x, nullptr, nullptr, w.partial, s));
  PP_TRY_HIP(ppk::launch_reduce_norm(w.partial, ppk::orth_grid(w.n, rpt), w.misc + 1, nullptr,
                                     s));
  PP_TRY_HIP(hipMemcpyAsync(w.host, w.misc + 1, sizeof(double), hipMemcpyDeviceToHost, s));
  PP_TRY_HIP(hipStreamSynchronize(s));
  *out = w.host[0];
  return PP_OK;
}

// r = b - A x into V(:,0), colscale[0] = 1/||r||; returns ||r||.
int residual_f64(const Opr<double> &A, Work<double> &w, const double *b, const double *x,
                 hipStream_t s, double *beta) {
  int nt = 0;
  if (A.ilu) {  // M^-1 b - M^-1 A x, with b = M^-1 b given
    PP_TRY(op_product<double>(A, x, nullptr, A.prod, s));
    PP_TRY_HIP(ppk::launch_sub_norm(A.n, b, A.prod, w.V, w.partial, &nt, s));
  } else {
    PP_TRY_HIP(ppk::launch_residual<double>(A, b, x, w.V, w.partial, &nt, s));
  }
  PP_TRY_HIP(ppk::launch_reduce_norm(w.partial, nt, w.misc, w.colscale, s));
  PP_TRY_HIP(hipMemcpyAsync(w.host, w.misc, sizeof(double), hipMemcpyDeviceToHost, s));
  PP_TRY_HIP(hipStreamSynchronize(s));
  *beta = w.host[0];
  return PP_OK;
}

// The solve's choice (pp_opts.chain_group / chain_slab_rows).
template <typename T>
int set_blocking(Opr<T> &A, const SolveIn &in, int32_t *scratch, hipStream_t s) {
  if (in.ilu) return PP_OK;
  return choose_schedule<T>(A, in.A, in.o.chain_group, in.o.chain_slab_rows, scratch, s);
}

// What set_blocking chose, for pp_stats and the PP_LOG trace.
template <typename T>
void note_schedule(pp_stats *st, const Opr<T> &A) {
  const bool blocked = A.blk_group >= 2;
  if (log_level() >= 1) {
    if (blocked)
      std::fprintf(stderr, "[pp] chain: slab-skewed, %d-row slabs, bandwidth %d, cached (%s)\n",
                   A.blk_slab_rows, A.blk_bw_rows, sizeof(T) == 4 ? "FP32" : "FP64");
    else
      std::fprintf(stderr, "[pp] chain: full-range, %s (%s)\n",
                   A.keep ? "cached" : "non-temporal", sizeof(T) == 4 ? "FP32" : "FP64");
  }
  if (!st) return;
  st->chain_slab_rows = blocked ? A.blk_slab_rows : 0;
  st->chain_cached = (blocked || A.keep) ? 1 : 0;
}

int solve_f64(const SolveIn &in, pp_stats *st) {
  const double t_start = now_s();
  Arena *ar = nullptr;
  PP_TRY(current_arena(&ar));
  const int n = (int)in.A->n;
  const int L = std::max(in.m, in.o.poly ? 0 : in.d) + 1;
  SellCopy sc;
  PP_TRY(make_sell(in.A, true, false, nullptr, solve_products(in), in.s, &sc));
  note_layout(st, in.A, sc);
  Work<double> w;
  Carver meas(nullptr);
  w.carve(meas, n, L);
  double *xsave = meas.take<double>(n);
  double *prod = in.ilu ? meas.take<double>(n) : nullptr;
  int32_t *iscratch = meas.take<int32_t>(64);
  const bool draw_v0 = !in.o.v0 && !in.o.poly && in.d > 0;
  double *v0gen = draw_v0 ? meas.take<double>(n) : nullptr;
  PP_TRY(ensure_arena(ar, meas.off + 256, w.host_doubles()));
  Carver c(ar->dev);
  w.carve(c, n, L);
  xsave = c.take<double>(n);
  prod = in.ilu ? c.take<double>(n) : nullptr;
  iscratch = c.take<int32_t>(64);
  v0gen = draw_v0 ? c.take<double>(n) : nullptr;
  w.attach(*ar);
  Opr<double> A(with_sell(view<double>(in.A, in.A->vals), sc));
  A.ilu = in.ilu;
  A.prod = prod;
  PP_TRY(set_blocking<double>(A, in, iscratch, in.s));
  note_schedule(st, A);
  hipStream_t s = in.s;
  Counters cnt;
  cnt.history = in.o.history;
  cnt.history_cap = in.o.history ? in.o.history_cap : 0;
  Timers tm;
  if (in.o.timing) {
    PP_TRY(tm.init());
    tm.on = true;
  }
  int status = PP_OK;
  double bnorm = 0.0;
  PP_TRY(norm_f64(w, in.b, s, &bnorm));
  if (!finite(bnorm)) return PP_ERR_ARG;
  auto finish = [&](double relres_true, double relres_impl, int cycles) {
    if (st) {
      st->iters = cnt.iters;
      st->cycles = cycles;
      st->spmvs = cnt.spmvs;
      st->dots = cnt.dots;
      st->relres_true = relres_true;
      st->relres_implicit = relres_impl;
      st->history_len = cnt.history_len;
      st->t_chain = tm.chain;
      st->t_spmv = tm.spmv;
      st->t_orth = tm.orth;
      st->t_host = tm.host;
      st->bytes_chain = cnt.bytes_chain;
      st->bytes_spmv = cnt.bytes_spmv;
      st->bytes_orth = cnt.bytes_orth;
      st->launches_chain = cnt.launches_chain;
      st->t_total = now_s() - t_start;
    }
  };
  if (bnorm == 0.0) {
    PP_TRY_HIP(ppk::launch_fill<double>(n, 0.0, in.x, s));
    PP_TRY_HIP(hipStreamSynchronize(s));
    finish(0.0, 0.0, 0);
    return PP_OK;
  }
  // the polynomial
  pp_poly built;
  PolyRef steps;
  if (in.o.poly) {
    steps = PolyRef::of(in.o.poly);
  } else if (in.d > 0) {
    const double t0 = now_s();
    if (draw_v0) PP_TRY_HIP(ppk::launch_uniform_pm1(n, in.o.v0_seed, v0gen, s));
    int rc = build_poly_impl<double>(A, draw_v0 ? v0gen : in.o.v0, in.d, w, s, cnt, tm, &built);
    if (rc < 0) return rc;
    status = worst(status, rc);
    steps = PolyRef::of(&built);
    if (st) st->t_poly = now_s() - t0;
  }
  const int nroots = in.o.poly ? poly_size(in.o.poly) : (in.d > 0 ? (int)built.re.size() : 0);
  if (st) st->nroots = nroots;
  const int max_iters = in.o.max_iters > 0 ? in.o.max_iters : 100000;
  double beta = 0.0;
  PP_TRY(residual_f64(A, w, in.b, in.x, s, &beta));
  cnt.spmvs++;
  cnt.dots++;
  double relres = beta / bnorm, relimp = relres;
  int cycles = 0;
  std::vector<double> y;
  if (!finite(relres)) {
    finish(relres, relres, 0);
    return worst(status, PP_WARN_NONFINITE);
  }
  int stagnant = 0;
  while (relres >= in.tol && cnt.iters < max_iters && stagnant < kStagnationCycles) {
    const double prev = relres;
    ++cycles;
    PP_TRY_HIP(hipMemcpyAsync(xsave, in.x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    int k = 0;
    double res = 0.0;
    bool nonfinite = false;
    PP_TRY(gmres_cycle<double>(A, steps, in.o.op_form, w, in.m, beta, in.tol * bnorm, bnorm,
                               max_iters - cnt.iters, s, tm, cnt, y, &k, &res, &nonfinite));
    if (nonfinite) {
      status = worst(status, PP_WARN_NONFINITE);
      break;
    }
    relimp = res / bnorm;
    PP_TRY(cycle_update<double>(A, steps, w, k, y, in.x, in.x, s, cnt));
    double nb = 0.0;
    PP_TRY(residual_f64(A, w, in.b, in.x, s, &nb));
    cnt.spmvs++;
    cnt.dots++;
    if (!finite(nb)) {
      PP_TRY_HIP(hipMemcpyAsync(in.x, xsave, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      PP_TRY_HIP(hipStreamSynchronize(s));
      status = worst(status, PP_WARN_NONFINITE);
      break;
    }
    beta = nb;
    relres = beta / bnorm;
    if (log_level() >= 1)
      std::fprintf(stderr, "[pp] cycle %d: %d steps, true relres %.3e (implicit %.3e)\n",
                   cycles, k, relres, relimp);
    // only a cycle whose estimate reached tol counts: one that ran all m steps is
    // converging slowly, not stuck at the rounding floor
    stagnant = (res < in.tol * bnorm && relres < kStagnationBand * in.tol &&
                relres > kStagnationFactor * prev)
                   ? stagnant + 1
                   : 0;
  }
  if (status != PP_WARN_NONFINITE && relres >= in.tol) status = worst(status, PP_WARN_NOT_CONVERGED);
  finish(relres, relimp, cycles);
  return status;
}

int solve_f32_ir(const SolveIn &in, pp_stats *st) {
  const double t_start = now_s();
  Arena *ar = nullptr;
  PP_TRY(current_arena(&ar));
  const int n = (int)in.A->n;
  const int64_t nnz = in.A->nnz;
  const int L = std::max(in.m, in.o.poly ? 0 : in.d) + 1;
  SellCopy sc;
  PP_TRY(make_sell(in.A, true, true, in.o.vals_f32, solve_products(in), in.s, &sc));
  note_layout(st, in.A, sc);
  // the FP32 CSR values are needed only when the products run on CSR
  const bool cast32 = !in.o.vals_f32 && !sc.use;
  Work<float> w;
  Work<double> w64;  // only the residual / norm pieces are used
  Carver meas(nullptr);
  w.carve(meas, n, L);
  w64.carve(meas, n, 1);
  float *vals32 = cast32 ? meas.take<float>(nnz > 0 ? nnz : 1) : nullptr;
  double *xsave = meas.take<double>(n);
  int32_t *iscratch = meas.take<int32_t>(64);
  const bool draw_v0 = !in.o.v0 && !in.o.poly && in.d > 0;
  double *v0gen = draw_v0 ? meas.take<double>(n) : nullptr;
  PP_TRY(ensure_arena(ar, meas.off + 256, w.host_doubles() + 16));
  Carver c(ar->dev);
  w.carve(c, n, L);
  w64.carve(c, n, 1);
  vals32 = cast32 ? c.take<float>(nnz > 0 ? nnz : 1) : nullptr;
  xsave = c.take<double>(n);
  iscratch = c.take<int32_t>(64);
  v0gen = draw_v0 ? c.take<double>(n) : nullptr;
  w.attach(*ar);
  w64.attach(*ar);
  hipStream_t s = in.s;
  const SpMat<double> A64 = with_sell(view<double>(in.A, in.A->vals), sc);
  if (cast32) PP_TRY_HIP(ppk::launch_cast_f32(nnz, (const double *)in.A->vals, vals32, s));
  Opr<float> A32(with_sell(
      view<float>(in.A, in.o.vals_f32 ? (const void *)in.o.vals_f32 : (const void *)vals32), sc));
  PP_TRY(set_blocking<float>(A32, in, iscratch, s));
  note_schedule(st, A32);
  Counters cnt;
  cnt.history = in.o.history;
  cnt.history_cap = in.o.history ? in.o.history_cap : 0;
  Timers tm;
  if (in.o.timing) {
    PP_TRY(tm.init());
    tm.on = true;
  }
  int status = PP_OK;
  double bnorm = 0.0;
  PP_TRY(norm_f64(w64, in.b, s, &bnorm));
  if (!finite(bnorm)) return PP_ERR_ARG;
  int outer = 0;
  auto finish = [&](double relres_true, double relres_impl) {
    if (st) {
      st->iters = cnt.iters;
      st->cycles = outer;
      st->outer = outer;
      st->spmvs = cnt.spmvs;
      st->dots = cnt.dots;
      st->relres_true = relres_true;
      st->relres_implicit = relres_impl;
      st->history_len = cnt.history_len;
      st->t_chain = tm.chain;
      st->t_spmv = tm.spmv;
      st->t_orth = tm.orth;
      st->t_host = tm.host;
      st->bytes_chain = cnt.bytes_chain;
      st->bytes_spmv = cnt.bytes_spmv;
      st->bytes_orth = cnt.bytes_orth;
      st->launches_chain = cnt.launches_chain;
      st->t_total = now_s() - t_start;
    }
  };
  if (bnorm == 0.0) {
    PP_TRY_HIP(ppk::launch_fill<double>(n, 0.0, in.x, s));
    PP_TRY_HIP(hipStreamSynchronize(s));
    finish(0.0, 0.0);
    return PP_OK;
  }
  pp_poly built;
  PolyRef steps;
  if (in.o.poly) {
    steps = PolyRef::of(in.o.poly);
  } else if (in.d > 0) {
    const double t0 = now_s();
    if (draw_v0) PP_TRY_HIP(ppk::launch_uniform_pm1(n, in.o.v0_seed, v0gen, s));
    int rc = build_poly_impl<float>(A32, draw_v0 ? v0gen : in.o.v0, in.d, w, s, cnt, tm, &built);
    if (rc < 0) return rc;
    status = worst(status, rc);
    steps = PolyRef::of(&built);
    if (st) st->t_poly = now_s() - t0;
  }
  if (st) st->nroots = in.o.poly ? poly_size(in.o.poly) : (in.d > 0 ? (int)built.re.size() : 0);
  const int max_iters = in.o.max_iters > 0 ? in.o.max_iters : 100000;
  const int max_outer = in.o.max_outer > 0 ? in.o.max_outer : 100;
  // inner stop: a given inner_tol as it is; by default 1e-5, loosened on a
  // refinement step that needs less to kInnerMargin * tol / relres, the reduction
  // still missing with a margin, so the last inner cycle does not overshoot
  const bool inner_auto = !(in.o.inner_tol > 0);
  const double inner_floor = inner_auto ? kInnerTolDefault : in.o.inner_tol;
  double relres = 0.0, relimp = 0.0;
  std::vector<double> y;
  double *r64 = w64.V;  // FP64 residual
  for (;;) {
    double beta = 0.0;
    PP_TRY(residual_f64(A64, w64, in.b, in.x, s, &beta));
    cnt.spmvs++;
    cnt.dots++;
    relres = beta / bnorm;
    if (log_level() >= 1)
      std::fprintf(stderr, "[pp] refinement step %d: true relres %.3e, %d inner steps so far\n",
                   outer, relres, cnt.iters);
    if (!finite(relres)) {
      if (outer > 0) {
        PP_TRY_HIP(hipMemcpyAsync(in.x, xsave, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        PP_TRY_HIP(hipStreamSynchronize(s));
      }
      status = worst(status, PP_WARN_NONFINITE);
      break;
    }
    if (relres < in.tol) break;
    if (outer >= max_outer || cnt.iters >= max_iters) {
      status = worst(status, PP_WARN_NOT_CONVERGED);
      break;
    }
    // V32(:,0) = (float)(r / beta), with its FP32 norm
    const int rpt = orth_rpt(kOrthWrite, 1, true, n);
    PP_TRY_HIP(ppk::launch_norm2<double>(n, rpt, r64, w64.colscale, w.V, w.partial, s));
    PP_TRY_HIP(ppk::launch_reduce_norm(w.partial, ppk::orth_grid(n, rpt), w.misc, w.colscale,
                                       s));
    PP_TRY_HIP(hipMemcpyAsync(w.host, w.misc, sizeof(double), hipMemcpyDeviceToHost, s));
    PP_TRY_HIP(hipMemcpyAsync(w64.misc + 2, &beta, sizeof(double), hipMemcpyHostToDevice, s));
    PP_TRY_HIP(hipStreamSynchronize(s));
    const double beta_in = w.host[0];
    cnt.dots++;
    PP_TRY_HIP(hipMemcpyAsync(xsave, in.x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    int k = 0;
    double res = 0.0;
    bool nonfinite = false;
    const double inner_tol =
        inner_auto ? std::max(inner_floor, kInnerMargin * in.tol / relres) : inner_floor;
    PP_TRY(gmres_cycle<float>(A32, steps, in.o.op_form, w, in.m, beta_in, inner_tol * beta_in,
                              beta_in,
                              max_iters - cnt.iters, s, tm, cnt, y, &k, &res, &nonfinite));
    ++outer;
    if (nonfinite) {
      status = worst(status, PP_WARN_NONFINITE);
      break;
    }
    relimp = relres * res / beta_in;
    // d32 = p(A32) V32 (colscale o y), then x += beta * d32 in FP64
    if (k > 0) {
      PP_TRY(cycle_update<float>(A32, steps, w, k, y, nullptr, w.Z, s, cnt));
      PP_TRY_HIP(ppk::launch_axpy_f64<float>(n, w64.misc + 2, w.Z, in.x, s));
    }
  }
  finish(relres, relimp);
  return status;
}

}  // namespace

// ====================================================================== C ABI
namespace ppd {

namespace {
thread_local char t_detail[320] = "";
}

int log_level() {
  static const int level = [] {
    const char *v = std::getenv("PP_LOG");
    return v ? std::atoi(v) : 0;
  }();
  return level;
}

hipError_t note(hipError_t e, const char *expr, const char *file, int line) {
  const char *base = std::strrchr(file, '/');
  std::snprintf(t_detail, sizeof(t_detail), "%s:%d: %s -> %s", base ? base + 1 : file, line,
                expr, hipGetErrorName(e));
  if (log_level() >= 1) std::fprintf(stderr, "[pp] HIP failure at %s\n", t_detail);
  return e;
}

const char *last_detail() { return t_detail; }

void note_msg(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(t_detail, sizeof(t_detail), fmt, ap);
  va_end(ap);
  if (log_level() >= 1) std::fprintf(stderr, "[pp] %s\n", t_detail);
}

void enter(const char *entry) {
  t_detail[0] = '\0';
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess && log_level() >= 1)
    std::fprintf(stderr, "[pp] %s: cleared a HIP error pending from before the call (%s)\n",
                 entry, hipGetErrorName(e));
}

}  // namespace ppd

// An error can end a call with work of its own still queued (a step issued one
// ahead of the one that failed): wait for it, so that nothing the call launched
// outlives it.
static int settle(int rc, hipStream_t s) {
  if (rc < 0) (void)hipStreamSynchronize(s);
  return rc;
}

extern "C" {

int pp_build_poly(const pp_csr *A, const double *v0, int d, void *stream, pp_poly **out) {
  ppd::enter("pp_build_poly");
  if (!out) return PP_ERR_ARG;
  *out = nullptr;
  PP_TRY(check_csr(A));
  if (d < 1 || d > kMaxD || d > A->n) return PP_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_lock);
  hipStream_t s = static_cast<hipStream_t>(stream);
  PP_TRY(validate_csr(A, s));
  const int rc = A->dtype == PP_F64 ? build_impl<double>(A, v0, d, s, out)
                                    : build_impl<float>(A, v0, d, s, out);
  return settle(rc, s);
}

int pp_apply(const pp_csr *A, const pp_poly *p, const void *v, void *y, void *stream) {
  ppd::enter("pp_apply");
  PP_TRY(check_csr(A));
  if (!p || !v || !y || v == y || p->n != A->n) return PP_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_lock);
  hipStream_t s = static_cast<hipStream_t>(stream);
  PP_TRY(validate_csr(A, s));
  return A->dtype == PP_F64 ? apply_impl<double>(A, p, v, y, s)
                            : apply_impl<float>(A, p, v, y, s);
}

int pp_apply_noalloc(const pp_csr *A, const pp_poly *p, const void *v, void *y,
                     void *stream) {
  ppd::enter("pp_apply_noalloc");
  PP_TRY(check_csr(A));
  if (!p || !v || !y || v == y || p->n != A->n) return PP_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_lock);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return A->dtype == PP_F64 ? apply_noalloc_impl<double>(A, p, v, y, s)
                            : apply_noalloc_impl<float>(A, p, v, y, s);
}

int pp_gmres_solve(const pp_csr *A, const double *b, double *x, int m, int d, double tol,
                   const pp_opts *opt, void *stream, pp_stats *st) {
  ppd::enter("pp_gmres_solve");
  if (st) std::memset(st, 0, sizeof(*st));
  PP_TRY(check_csr(A));
  if (!b || !x || m < 1 || m > kMaxM || !(tol > 0) || d < 0 || d > kMaxD || A->dtype != PP_F64)
    return PP_ERR_ARG;
  SolveIn in{A, b, x, m, d, tol, pp_opts{}, static_cast<hipStream_t>(stream)};
  pp_csr scaled;
  if (opt) in.o = *opt;
  if (in.o.precision != PP_PREC_F64 && in.o.precision != PP_PREC_F32_IR) return PP_ERR_ARG;
  if (in.o.op_form != PP_OP_RESIDUAL_POLY && in.o.op_form != PP_OP_PRODUCT) return PP_ERR_ARG;
  if (in.o.chain_group < 0 || in.o.chain_slab_rows < 0) return PP_ERR_ARG;
  if (in.o.poly) {
    if (in.o.poly->n != A->n) return PP_ERR_ARG;
  } else if (d > A->n) {
    return PP_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(g_lock);
  PP_TRY(validate_csr(A, in.s));
  Arena *ar = nullptr;
  std::unique_lock<std::mutex> ilu_lock;
  if (in.o.left_ilu) {
    // Section VI, second example: ILU(0) on the left, the polynomial of M^-1 A on
    // the right; the solve runs on (M^-1 A, M^-1 b)
    const pp_ilu *M = in.o.left_ilu;
    if (in.o.left_jacobi || in.o.precision != PP_PREC_F64 || in.o.vals_f32 || M->n != A->n ||
        M->nnz != A->nnz || !ppi::on_device(*M))
      return PP_ERR_ARG;
    PP_TRY(current_arena(&ar));
    PP_TRY(ensure_aux(ar, (size_t)A->n * sizeof(double) + 256));
    double *bs = reinterpret_cast<double *>(ar->aux);
    ilu_lock = std::unique_lock<std::mutex>(M->lock);  // M->work, for the whole solve
    PP_TRY_HIP(ppi::ilu_solve(*M, b, bs, in.s));
    in.b = bs;
    in.ilu = M;
  }
  if (in.o.left_jacobi) {
    // Section II composition: run the unchanged solver on (D^-1 A, D^-1 b).
    if (in.o.vals_f32) return PP_ERR_ARG;
    PP_TRY(current_arena(&ar));
    const int64_t n = A->n, nnz = A->nnz;
    Carver meas(nullptr);
    meas.take<double>(nnz > 0 ? nnz : 1);
    meas.take<double>(n);
    meas.take<int32_t>(64);
    PP_TRY(ensure_aux(ar, meas.off + 256));
    Carver c(ar->aux);
    double *va = c.take<double>(nnz > 0 ? nnz : 1);
    double *bs = c.take<double>(n);
    int32_t *bad = c.take<int32_t>(64);
    hipStream_t s = in.s;
    PP_TRY_HIP(ppk::launch_fill<int32_t>(1, 0, bad, s));
    PP_TRY_HIP(ppk::launch_jacobi_scale((int)n, A->row_ptr, A->col_ind,
                                        static_cast<const double *>(A->vals), b, va, bs, bad, s));
    int32_t hbad = 0;
    PP_TRY_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PP_TRY_HIP(hipStreamSynchronize(s));
    if (hbad) return PP_ERR_SINGULAR;
    scaled = *A;
    scaled.vals = va;
    in.A = &scaled;
    in.b = bs;
  }
  int rc = in.o.precision == PP_PREC_F64 ? solve_f64(in, st) : solve_f32_ir(in, st);
  rc = settle(rc, in.s);
  if (st) {
    st->status = rc;
    st->relres_original = st->relres_true;
  }
  if ((in.o.left_jacobi || in.o.left_ilu) && rc >= 0 && st) {
    // ||b - A x|| / ||b|| of the original system, in the (re-carved) main arena
    const int n = (int)A->n;
    Work<double> w;
    Carver meas(nullptr);
    w.carve(meas, n, 1);
    PP_TRY(ensure_arena(ar, meas.off + 256, w.host_doubles()));
    Carver c(ar->dev);
    w.carve(c, n, 1);
    w.attach(*ar);
    double bn = 0.0, rn = 0.0;
    PP_TRY(norm_f64(w, b, in.s, &bn));
    PP_TRY(residual_f64(view<double>(A, A->vals), w, b, x, in.s, &rn));
    st->relres_original = bn > 0 ? rn / bn : 0.0;
  }
  return rc;
}

int pp_build_poly_power(const pp_csr *A, const double *v0, int deg, int auto_degree,
                        void *stream, pp_poly **out, int *info_out) {
  ppd::enter("pp_build_poly_power");
  if (!out) return PP_ERR_ARG;
  *out = nullptr;
  if (info_out) *info_out = 0;
  PP_TRY(check_csr(A));
  if (deg < 0 || deg > ppk::kMaxCols - 2 || deg + 1 > A->n) return PP_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_lock);
  hipStream_t s = static_cast<hipStream_t>(stream);
  PP_TRY(validate_csr(A, s));
  Arena *ar = nullptr;
  PP_TRY(current_arena(&ar));
  const int n = (int)A->n, L = deg + 2;
  auto go = [&](auto tag) -> int {
    using T = decltype(tag);
    SellCopy sc;
    PP_TRY(make_sell(A, sizeof(T) == 8, sizeof(T) == 4, nullptr, deg + 1.0, s, &sc));
    Work<T> w;
    Carver meas(nullptr);
    w.carve(meas, n, L);
    meas.take<double>((size_t)L * L);
    if (!v0) meas.take<double>(n);
    PP_TRY(ensure_arena(ar, meas.off + 256, w.host_doubles()));
    Carver c(ar->dev);
    w.carve(c, n, L);
    double *gram = c.take<double>((size_t)L * L);
    w.attach(*ar);
    const double *start = v0;
    if (!v0) {
      double *v0gen = c.take<double>(n);
      PP_TRY_HIP(ppk::launch_uniform_pm1(n, kDefaultSeed, v0gen, s));
      start = v0gen;
    }
    Counters cnt;
    pp_poly *p = new pp_poly();
    p->dtype = A->dtype;
    int rc = build_power_impl<T>(with_sell(view<T>(A, A->vals), sc), start, deg, auto_degree != 0,
                                 w, gram, s, cnt, p, info_out);
    if (rc < 0) {
      delete p;
      return rc;
    }
    *out = p;
    return rc;
  };
  return settle(A->dtype == PP_F64 ? go(double{}) : go(float{}), s);
}

int pp_poly_coeffs(const pp_poly *p, double *c, int cap, int *n_out) {
  if (!p || !n_out || p->kind != 1) return PP_ERR_ARG;
  const int k = (int)p->coeffs.size();
  *n_out = k;
  if (!c || cap < k) return PP_ERR_ARG;
  for (int i = 0; i < k; ++i) c[i] = p->coeffs[i];
  return PP_OK;
}

int pp_poly_roots(const pp_poly *p, double *re, double *im, int cap, int *d_out) {
  if (!p || !d_out || p->kind != 0) return PP_ERR_ARG;
  const int d = (int)p->re.size();
  *d_out = d;
  if (d > 0 && (!re || !im || cap < d)) return PP_ERR_ARG;
  for (int i = 0; i < d; ++i) {
    re[i] = p->re[i];
    im[i] = p->im[i];
  }
  return PP_OK;
}

int pp_poly_from_roots(int64_t n, const double *re, const double *im, int d, int dtype,
                       pp_poly **out) {
  if (!out || n <= 0 || d < 0 || d > kMaxD || (d > 0 && (!re || !im)) ||
      (dtype != PP_F64 && dtype != PP_F32))
    return PP_ERR_ARG;
  *out = nullptr;
  std::vector<double> r(re, re + d), i(im, im + d);
  std::vector<ppn::Step> steps;
  PP_TRY(ppn::step_table(r, i, steps));
  pp_poly *p = new pp_poly();
  p->n = n;
  p->dtype = dtype;
  p->re = r;
  p->im = i;
  p->steps = steps;
  *out = p;
  return PP_OK;
}

void pp_poly_free(pp_poly *p) { delete p; }

int pp_roots_from_hessenberg(const double *Hbar, int ldh, int s, double *re, double *im) {
  if (!Hbar || !re || !im || s < 1 || s > 4096 || ldh < s + 1) return PP_ERR_ARG;
  std::vector<double> wr, wi, lr, li;
  PP_TRY(ppn::harmonic_ritz(Hbar, ldh, s, wr, wi));
  PP_TRY(ppn::leja_order(wr, wi, lr, li));
  for (int k = 0; k < s; ++k) {
    re[k] = lr[k];
    im[k] = li[k];
  }
  return PP_OK;
}

int pp_csr_transpose(const pp_csr *A, int32_t *rp_t, int32_t *ci_t, void *vals_t, void *stream) {
  ppd::enter("pp_csr_transpose");
  PP_TRY(check_csr(A));
  if (!rp_t || (A->nnz > 0 && (!ci_t || !vals_t))) return PP_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_lock);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = (int)A->n, nnz = (int)A->nnz;
  Arena *ar = nullptr;
  PP_TRY(current_arena(&ar));
  PP_TRY(validate_csr(A, s));
  Carver meas(nullptr);
  meas.take<int32_t>(n);
  meas.take<int32_t>(n);
  meas.take<int32_t>(ppk::scan_tmp_size(n));
  meas.take<int32_t>(nnz > 0 ? nnz : 1);
  PP_TRY(ensure_arena(ar, meas.off + 256, 64));
  Carver c(ar->dev);
  int32_t *cnt = c.take<int32_t>(n);
  int32_t *cursor = c.take<int32_t>(n);
  int32_t *tmp = c.take<int32_t>(ppk::scan_tmp_size(n));
  int32_t *src = c.take<int32_t>(nnz > 0 ? nnz : 1);
  PP_TRY_HIP(ppk::launch_fill<int32_t>(n, 0, cnt, s));
  PP_TRY_HIP(ppk::launch_fill<int32_t>(n, 0, cursor, s));
  PP_TRY_HIP(ppk::launch_count_cols(nnz, A->col_ind, cnt, s));
  PP_TRY_HIP(ppk::launch_exclusive_scan(n, cnt, rp_t, tmp, s));
  if (nnz > 0) {
    if (A->dtype == PP_F64) {
      PP_TRY_HIP(ppk::launch_scatter_transpose<double>(n, A->row_ptr, A->col_ind,
                                                       (const double *)A->vals, rp_t, cursor,
                                                       ci_t, (double *)vals_t, src, s));
      PP_TRY_HIP(ppk::launch_sort_rows<double>(n, rp_t, ci_t, (double *)vals_t, src, s));
    } else {
      PP_TRY_HIP(ppk::launch_scatter_transpose<float>(n, A->row_ptr, A->col_ind,
                                                      (const float *)A->vals, rp_t, cursor, ci_t,
                                                      (float *)vals_t, src, s));
      PP_TRY_HIP(ppk::launch_sort_rows<float>(n, rp_t, ci_t, (float *)vals_t, src, s));
    }
  }
  PP_TRY_HIP(hipStreamSynchronize(s));
  return PP_OK;
}

int pp_csr_grad(const pp_csr *A, const double *lam, const double *x, double *g_vals,
                void *stream) {
  ppd::enter("pp_csr_grad");
  if (!A || A->n <= 0 || A->nnz < 0 || A->n >= (int64_t)1 << 31 || A->nnz >= (int64_t)1 << 31 ||
      !A->row_ptr || !lam || !x || (A->nnz > 0 && (!A->col_ind || !g_vals)))
    return PP_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_lock);
  hipStream_t s = static_cast<hipStream_t>(stream);
  PP_TRY(validate_csr(A, s));
  PP_TRY_HIP(ppk::launch_csr_grad((int)A->n, A->row_ptr, A->col_ind, lam, x, g_vals, s));
  PP_TRY_HIP(hipStreamSynchronize(s));
  return PP_OK;
}

int pp_uniform_vector(int64_t n, uint64_t seed, double *out, void *stream) {
  ppd::enter("pp_uniform_vector");
  if (!out || n <= 0 || n >= ((int64_t)1 << 40)) return PP_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PP_TRY_HIP(ppk::launch_uniform_pm1(n, seed, out, s));
  PP_TRY_HIP(hipStreamSynchronize(s));
  return PP_OK;
}

void pp_release_workspace(void) {
  std::lock_guard<std::mutex> lk(g_lock);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (size_t dev = 0; dev < g_arena.size(); ++dev) {
    Arena &a = g_arena[dev];
    if (!a.dev && !a.host && !a.aux && !a.mat) continue;
    (void)hipSetDevice((int)dev);
    (void)hipDeviceSynchronize();
    if (a.dev) (void)hipFree(a.dev);
    if (a.aux) (void)hipFree(a.aux);
    if (a.mat) (void)hipFree(a.mat);
    if (a.host) (void)hipHostFree(a.host);
    for (hipEvent_t e : a.step_ev)
      if (e) (void)hipEventDestroy(e);
    a = Arena{};
  }
  (void)hipSetDevice(cur);
}

const char *pp_status_string(int code) {
  switch (code) {
    case PP_OK: return "ok";
    case PP_ERR_ARG: return "invalid argument";
    case PP_ERR_HIP: return "HIP runtime error";
    case PP_ERR_NOMEM: return "out of memory";
    case PP_ERR_EIG: return "Hessenberg QR did not converge";
    case PP_ERR_SINGULAR: return "singular Hessenberg, zero start vector, or zero/non-finite root";
    case PP_WARN_DEGREE_REDUCED: return "warning: Arnoldi breakdown, polynomial has fewer roots";
    case PP_WARN_NOT_CONVERGED:
      return "warning: not converged (iteration cap, or stagnation at attainable accuracy)";
    case PP_WARN_NONFINITE: return "warning: non-finite value met, last finite iterate returned";
    case PP_WARN_CHOLESKY:
      return "warning: power-basis Gram matrix not positive definite (POTRF info > 0)";
    default: return "unknown status";
  }
}

const char *pp_last_error(void) { return ppd::last_detail(); }

const char *pp_version(void) { return "libpp 0.4.0 gfx950"; }

}  // extern "C"
