// Host side of the C ABI declared in include/sfk.h: validation, workspace
// layout, initialisation and the per-iteration stage sequence.  A context holds
// one instance (sfk_init), a batch of independent instances (sfk_init_batch),
// or R right-hand sides sharing one operator pair (sfk_init_multi).  They
// advance in lockstep: every stage kernel serves all instances of the context
// in one launch, through a block -> (instance, workgroup) map for a batch, or
// over interleaved vectors for shared operators.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "sfk.h"
#include "sfk_dev.h"
#include "sfk_units.h"
#include "sfk_adjoint_layout.h"
#include "sfk_lowrank.h"

namespace sfk {
void launch_stage_A(const Launch &L, int k, hipStream_t st);
void launch_stage_B(const Launch &L, int k, hipStream_t st);
void launch_stage_C(const Launch &L, int k, hipStream_t st);
void launch_stage_D(const Launch &L, int k, hipStream_t st);
void launch_sketch(const Launch &L, int k, hipStream_t st);
void launch_ls(const Launch &L, int k, hipStream_t st);
int spmv_blocks_per_cu();
void launch_backsub(const Dev &D, int j, double *yout, hipStream_t st);
void launch_init_b(const Dev &D, double eta, double noise, double tol_user, int use_disc,
                   hipStream_t st);
void launch_init_rhs(const Dev &D, hipStream_t st);
void launch_csr_check(const int *rp, const int *ci, int rows, int cols, long long nnz, int *err,
                      hipStream_t st);
void launch_partition(const int *rp, int rows, long long nnz, int nw, int *part, hipStream_t st);
void launch_transpose(const int *rp, const int *ci, const double *va, int rows, int cols, int *brp,
                      int *bci, double *bva, int *cursor, int *err, hipStream_t st);
void launch_sketch_build(const Dev &D, uint64_t key0, uint64_t key1, uint64_t key1_rows,
                         int *scratch, int *err, hipStream_t st);
void launch_perm_check(const int *perm, int n, int *cnt, int *pinv, int *err, hipStream_t st);
void launch_relabel_cols(const int *rp, const int *ci, const double *va, int rows, int nnz,
                         const int *perm, int *oci, double *ova, int *err, hipStream_t st);
void launch_perm_rows(const int *rp, const int *ci, const double *va, int rows, const int *perm,
                      int *orp, int *oci, double *ova, hipStream_t st);
void launch_solution(const Dev &D, int kk, const double *yv, double *x, hipStream_t st);
void launch_true_residual(const Dev &D, const double *x, double *out, hipStream_t st);
void launch_true_iter(const Dev &D, int k, hipStream_t st);
void launch_zero_bytes(void *p, size_t n, hipStream_t st);
void launch_beam_rays(const Dev &D, hipStream_t st);
void launch_uniform_part(int rows, int nw, int *part, hipStream_t st);
size_t full_scratch_doubles(int maxit);
void launch_full_init(const Dev &D, int vwB, hipStream_t st);
void launch_full_iteration(const Dev &D, int k, int vwA, int vwB, hipStream_t st,
                           void (*mark)(void *, int, int), void *ctx);
void launch_full_backsub(const Dev &D, int j, double *yout, hipStream_t st);
void launch_checkpoint_w(const Dev &D, int k, double *ck, hipStream_t st);
size_t adjoint_checkpoint_doubles(int maxit, int tape, int ell, int m);

void launch_iota_map(int2 *map, int count, hipStream_t st);
void launch_export_vec(const double *src, int vs, int len, const double *scale, const int *pinv,
                       double *out, hipStream_t st);
void launch_group_stage(const Grp &G, int stage, int k, hipStream_t st);
int gspmm_blocks_per_cu(int RS);
int gspmm_x_blocks_per_cu(int RS);
int gspmm_x_units_per_block(int RS);
int gspmm_l_blocks_per_cu(int RS);
void launch_scan(int *a, int len, hipStream_t st);
void launch_sell_len(const int *rp, int rows, int nsl, int *slen, hipStream_t st);
void launch_to_u16(const int *in, uint16_t *out, long long n, hipStream_t st);
void launch_spmv_core(const Dev &D, bool isa, int vw, const double *x, double *y, hipStream_t st);
void launch_sell_fill(const int *rp, const int *ci, const double *va, int rows, const int *soff,
                      const int *slen, int *scol, double *sval, hipStream_t st);
void launch_collect_halt(const Launch &L, int k, int *out, hipStream_t st);
void launch_xs_count(const int *rp, const int *ci, int rows, int NS, const int *cb, int *touch,
                     int *rowcnt, int *err, hipStream_t st);
void launch_xs_fill1(const int *rp, const int *ci, int rows, int NS, const int *cb,
                     const int *touch, const int *crp, int *slot, int *seglen, int *segsrc,
                     int *segrow, int *segcnt, hipStream_t st);
void launch_xs_fill2(const int *ci, const double *va, int nseg, const int *pos, const int *segsrc,
                     const int *segrow, const int *segcnt, const int *slot, int RS, int4 *seg,
                     XNz *xnz, hipStream_t st);
void launch_xs_part(const int *touch, int rows, int NS, int nseg, const int *pos, int nbs,
                    int *spart, hipStream_t st);
}  // namespace sfk

using namespace sfk;

struct Plan;

struct Inst {
  sfk_params p{};
  Dev D{};                        // host copy of the instance descriptor
  void *ws = nullptr;
  size_t ws_bytes = 0;
  bool owns_ws = false;
  int *d_err = nullptr;
  double *d_scalar = nullptr;     // one double of scratch (true residual)
  double *d_ytmp = nullptr;       // maxit
  int *chunk_scratch = nullptr;   // sparse-sign build scratch
  const int *user_aci = nullptr;  // the caller's A columns/values when the products
  const double *user_ava = nullptr;  // run on a renumbered copy (true residual)
  int k_done = 0, stopped = 0, breakdown = 0, halted = 0;
  double rhsnorm = 0.0;
  bool lowrank = false;           // tau LOWRANK / LOWRANK_RND: z = tau_r(p) stage
  LrBufs lr{};
};

struct sfk_ctx {
  std::vector<Inst> inst;
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;       // sketch + least-squares stream (default priority)
  static constexpr int kRing = kRawSlots;   // iterations of synchronisation events kept
  hipEvent_t ev_main[kRing] = {}, ev_sk[kRing] = {}, ev_ls[kRing] = {};
  void *hdr = nullptr;              // device: instance descriptors and block maps
  size_t hdr_bytes = 0, gws_bytes = 0;
  Launch L{};
  Scal *h_scal = nullptr;           // pinned copies of the device scalars
  // early exit of long iterate() calls: the run state of every instance is
  // copied back after each batch of iterations (side stream, pinned memory)
  static constexpr int kChkSlots = 2;
  int *d_halt = nullptr;            // device, kChkSlots * ninst
  int *h_halt = nullptr;            // pinned, kChkSlots * ninst
  hipEvent_t ev_chk[kChkSlots] = {};
  int k_iter = 0;                   // lockstep iterations launched
  // events of iterations below ev_from were recorded inside a graph capture
  // (or belong to a finished graph): no stream waits on them
  int ev_from = 0;
  bool graph = false;               // driver GRAPH
  hipGraphExec_t gexec = nullptr;   // executable graph of the last batch (updated per batch)
  hipEvent_t ev_join = nullptr;     // joins the side stream into a captured batch
  hipStream_t gstream = nullptr;    // capture stream (the caller's may be the legacy
  hipEvent_t ev_fork = nullptr;     // default stream, which cannot be captured), ordered
  hipEvent_t ev_done = nullptr;     // after and before the caller's by these events
  int maxitmax = 0;
  bool sketch_after_C = false;      // an sFLSMR instance sketches B w_{k+1}
  bool any_rew = false;
  int resid = 0;                    // per-iteration true residual (single instance)
  bool full = false;                // FLSQR / FLSMR (full orthogonalisation)
  int tape = 0;                     // derivative tape: checkpoint interval (0: none)
  int open_stage[SFK_NUM_STAGES] = {-1, -1, -1, -1, -1, -1, -1};
  size_t lib_bytes = 0;             // device memory allocated besides the workspaces
  int pending_side[2] = {-1, -1};   // iterations whose sketch/LS wait for the next flush point
  bool multi = false;               // right-hand sides sharing A and B (stages via grp)
  Grp grp{};
  void *gws = nullptr;              // workspace of the shared arrays
  std::vector<std::pair<void *, size_t>> xmem;  // sliced / SELL / renumbered copies of A and B
  const int *gperm = nullptr;       // shared operators: the group's order of the
  const int *gpinv = nullptr;       // unknowns and its inverse (NULL: identity)
  char err[512] = {};               // last error (fixed storage: reporting allocates nothing)
  // optional per-stage timing with HIP events
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_used;   // (stage, index of the start event)
  double stage_ms[SFK_NUM_STAGES] = {};
  int stage_count[SFK_NUM_STAGES] = {};
};

// Device memory owned by the context besides the workspaces (released in
// order by lib_pop, all at sfk_destroy).
static hipError_t lib_malloc(sfk_ctx *c, void **q, size_t bytes) {
  hipError_t e = hipMalloc(q, bytes);
  if (e == hipSuccess) c->xmem.push_back({*q, bytes});
  return e;
}

static void lib_pop(sfk_ctx *c) {
  hipFree(c->xmem.back().first);
  c->xmem.pop_back();
}

// records the start event of a timed stage; returns its pool index or -1
static int stage_begin(sfk_ctx *c, int stage, hipStream_t st) {
  if (!c->timing) return -1;
  const size_t need = c->ev_used.size() * 2 + 2;
  while (c->ev_pool.size() < need) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    c->ev_pool.push_back(e);
  }
  const int idx = (int)c->ev_used.size() * 2;
  hipEventRecord(c->ev_pool[idx], st);
  c->ev_used.push_back({stage, idx});
  return idx;
}

static void stage_end(sfk_ctx *c, int idx, hipStream_t st) {
  if (idx >= 0) hipEventRecord(c->ev_pool[idx + 1], st);
}

static void collect_stage_times(sfk_ctx *c) {
  for (auto &u : c->ev_used) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_pool[u.second], c->ev_pool[u.second + 1]) == hipSuccess) {
      c->stage_ms[u.first] += ms;
      c->stage_count[u.first] += 1;
    }
  }
  c->ev_used.clear();
}

// One lockstep iteration k of Algorithm 1 (sFLSQR) / Algorithm 2 (sFLSMR) for
// every instance.  The data-parallel stages A, B, C, D run on the context's
// stream; the sketch of the new vector and the least-squares update run on the
// side stream as soon as their input exists.  The raw products are kept in a
// ring of kRawSlots slots, so the main stream waits for the side stream only
// every few iterations (enqueue_iteration).  The reweighting needs y_k before
// D(k), so it waits for LS(k).
static void run_stage(sfk_ctx *c, int stage, int k, hipStream_t st) {
  if (c->multi) {
    launch_group_stage(c->grp, stage, k, st);
    return;
  }
  switch (stage) {
    case kStageA: launch_stage_A(c->L, k, st); break;
    case kStageB: launch_stage_B(c->L, k, st); break;
    case kStageC: launch_stage_C(c->L, k, st); break;
    default: launch_stage_D(c->L, k, st); break;
  }
}

// Sketches and least-squares updates of iterations js[0..n) (in order) on the
// side stream, after what the main stream has been given so far (one event).
static void enqueue_side(sfk_ctx *c, const int *js, int n) {
  const Launch &L = c->L;
  hipStream_t st = c->stream, sd = c->side;
  const int r0 = js[0] % sfk_ctx::kRing;
  hipEventRecord(c->ev_main[r0], st);
  hipStreamWaitEvent(sd, c->ev_main[r0], 0);
  for (int i = 0; i < n; ++i) {
    const int j = js[i], r = j % sfk_ctx::kRing;
    int t = stage_begin(c, SFK_STAGE_SKETCH, sd);
    launch_sketch(L, j, sd);
    stage_end(c, t, sd);
    hipEventRecord(c->ev_sk[r], sd);
    t = stage_begin(c, SFK_STAGE_LS, sd);
    launch_ls(L, j, sd);
    stage_end(c, t, sd);
    if (c->resid) launch_true_iter(c->inst[0].D, j, sd);
    hipEventRecord(c->ev_ls[r], sd);
  }
}

// Sketch of iteration k on the main stream, then its least-squares update on
// the side stream (the reweighting, where D(k) needs LS(k)).
static void sketch_main_ls_side(sfk_ctx *c, int k) {
  const Launch &L = c->L;
  hipStream_t st = c->stream, sd = c->side;
  const int r = k % sfk_ctx::kRing;
  int t = stage_begin(c, SFK_STAGE_SKETCH, st);
  launch_sketch(L, k, st);
  stage_end(c, t, st);
  hipEventRecord(c->ev_sk[r], st);
  hipStreamWaitEvent(sd, c->ev_sk[r], 0);
  t = stage_begin(c, SFK_STAGE_LS, sd);
  launch_ls(L, k, sd);
  stage_end(c, t, sd);
  if (c->resid) launch_true_iter(c->inst[0].D, k, sd);
  hipEventRecord(c->ev_ls[r], sd);
}

static void flush_side(sfk_ctx *c) {
  int n = 0;
  while (n < 2 && c->pending_side[n] >= 0) ++n;
  if (n > 0) enqueue_side(c, c->pending_side, n);
  c->pending_side[0] = c->pending_side[1] = -1;
}

static void defer_side(sfk_ctx *c, int k) {
  if (c->pending_side[0] < 0) c->pending_side[0] = k;
  else c->pending_side[1] = k;
}

// z~_{k+1} = tau_r(p~_{k+1}) of the low-rank operators, after D(k) (or after the
// full path's p_{k+1}); k = 0 is the initial basis vector.
static void enqueue_tau(sfk_ctx *c, int k) {
  Inst &I = c->inst[0];
  const Dev &D = I.D;
  const double *pin = c->full ? D.Pf + (size_t)k * D.n
                              : D.P + (size_t)((k + 1) % (D.ell + 1)) * D.n;
  const int t = stage_begin(c, SFK_STAGE_TAU, c->stream);
  lr_apply(I.lr, D.sc, D.maxit, c->full ? 1 : 0, k, pin, D.Z + (size_t)k * D.n, c->stream);
  stage_end(c, t, c->stream);
}

// One iteration.  The sketch of iteration k reads raw product slot
// k % kRawSlots, rewritten by iteration k + kRawSlots; the main stream waits
// for the side stream once every four iterations (before A(k), k = 0 mod 4:
// for the sketch of iteration k - 5, and with it every earlier one), and the
// sketches go out in pairs after a sparse product, where their workgroups run
// beside a light vector stage instead of taking CU slots from a product's:
// sFLSQR after C(k), sFLSMR after A(k) (sketches k - 2 and k - 1), k even.
// The reweighting needs LS(k) before D(k): then each sketch runs on the main
// stream as soon as its input exists (a sketch beside a sparse product is
// slowed about tenfold, ~5 -> ~50 us for a sparse-sign sketch, and D(k) would
// wait for it), and only the least-squares update goes to the side stream.
static void enqueue_iteration(sfk_ctx *c, int k) {
  static_assert(sfk_ctx::kRing >= 8 && kRawSlots >= 8, "side-stream lag");
  hipStream_t st = c->stream;
  const bool late = !c->any_rew;
  if (k >= 8 && k % 4 == 0 && k - 5 >= c->ev_from)
    hipStreamWaitEvent(st, c->ev_sk[(k - 5) % sfk_ctx::kRing], 0);
  int t = stage_begin(c, SFK_STAGE_SPMV_A, st);
  run_stage(c, kStageA, k, st);
  stage_end(c, t, st);
  if (late && c->sketch_after_C && k % 2 == 0) flush_side(c);
  if (!late && !c->sketch_after_C) sketch_main_ls_side(c, k);
  t = stage_begin(c, SFK_STAGE_W_UPDATE, st);
  run_stage(c, kStageB, k, st);
  stage_end(c, t, st);
  t = stage_begin(c, SFK_STAGE_SPMV_B, st);
  run_stage(c, kStageC, k, st);
  stage_end(c, t, st);
  if (c->tape && k % c->tape == 0) {
    const Dev &D0 = c->inst[0].D;
    launch_checkpoint_w(D0, k, D0.ck + (size_t)(k / c->tape) * (D0.ell + 2) * D0.m, st);
  }
  if (late) {
    defer_side(c, k);
    if (!c->sketch_after_C && k % 2 == 0) flush_side(c);
  } else if (c->sketch_after_C) {
    sketch_main_ls_side(c, k);
  }
  if (c->any_rew) hipStreamWaitEvent(st, c->ev_ls[k % sfk_ctx::kRing], 0);
  t = stage_begin(c, SFK_STAGE_P_UPDATE, st);
  run_stage(c, kStageD, k, st);
  stage_end(c, t, st);
  if (c->inst[0].lowrank) enqueue_tau(c, k);
}

// Stage timing of the full-orthogonalisation iteration (begin = 1 / 0).
static void full_mark(void *ctx, int stage, int begin) {
  sfk_ctx *c = static_cast<sfk_ctx *>(ctx);
  if (begin) c->open_stage[stage] = stage_begin(c, stage, c->stream);
  else stage_end(c, c->open_stage[stage], c->stream);
}

static void enqueue_full_iteration(sfk_ctx *c, int k) {
  const Dev &D = c->inst[0].D;
  launch_full_iteration(D, k, D.vwA, D.vwB, c->stream, c->timing ? full_mark : nullptr, c);
  if (c->inst[0].lowrank) enqueue_tau(c, k);
  if (c->resid) launch_true_iter(D, k, c->stream);
}

// Iterations k0 .. k0 + n - 1 captured from the two streams into one HIP
// graph (the side stream forks from and joins back into the capture), then
// launched on the context's stream.  Kernel arguments depend on k, so each
// batch is captured anew; the executable graph is updated in place when the
// topology allows it, else instantiated again.  Work of earlier batches is
// complete before a graph launch starts (stream order), so waits on events of
// earlier batches are dropped (ev_from).
static hipError_t enqueue_graph_batch(sfk_ctx *c, int k0, int n) {
  hipStream_t user = c->stream, st = c->gstream;
  hipError_t e = hipEventRecord(c->ev_fork, user);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, c->ev_fork, 0);
  if (e != hipSuccess) return e;
  c->ev_from = k0;
  e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  c->stream = st;                       // the stage sequence runs on the capture stream
  for (int i = 0; i < n; ++i) enqueue_iteration(c, k0 + i);
  flush_side(c);
  hipEventRecord(c->ev_join, c->side);
  hipStreamWaitEvent(st, c->ev_join, 0);
  c->stream = user;
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(st, &g);
  if (e != hipSuccess) return e;
  if (c->gexec) {
    hipGraphNode_t bad = nullptr;
    hipGraphExecUpdateResult res;
    if (hipGraphExecUpdate(c->gexec, g, &bad, &res) != hipSuccess || res != hipGraphExecUpdateSuccess) {
      (void)hipGetLastError();
      hipGraphExecDestroy(c->gexec);
      c->gexec = nullptr;
    }
  }
  if (!c->gexec) e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) return e;
  e = hipGraphLaunch(c->gexec, st);
  if (e == hipSuccess) e = hipEventRecord(c->ev_done, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(user, c->ev_done, 0);
  c->ev_from = k0 + n;
  return e;
}

static thread_local char g_err[512];

static void set_err(char *dst, const char *src) { std::snprintf(dst, 512, "%s", src); }

// prefixes the error of a context (or the thread's) with "<what> <i>: "
static void prefix_err(char *dst, const char *what, int i) {
  char tmp[512];
  std::snprintf(tmp, sizeof tmp, "%s %d: %s", what, i, dst);
  set_err(dst, tmp);
}

static sfk_status fail(sfk_ctx *c, sfk_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_err(c ? c->err : g_err, buf);
  return st;
}

#define HIPCHK(ctx, expr)                                                                    \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(ctx, SFK_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

// --------------------------------------------------------------------------
// parameters and validation
// --------------------------------------------------------------------------
extern "C" void sfk_params_default(sfk_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->method = SFK_SFLSQR;
  p->ell = 2;
  p->maxit = 50;
  p->sketch = SFK_SK_SPARSE_SIGN;
  p->s = 101;
  p->zeta = 8;
  p->seed = 0;
  p->tau = SFK_TAU_IDENTITY;
  p->eps = 1e-3;
  p->eta = 1.01;
  p->noise_norm = 0.0;
  p->tol = 0.0;
  p->driver = SFK_DRIVER_AUTO;
  p->vw = -2;
  p->lr_q = 1;
}

static bool is_lowrank(const sfk_params *p) {
  return p->tau == SFK_TAU_LOWRANK || p->tau == SFK_TAU_LOWRANK_RND;
}

// test vectors l of the low-rank operators (0 when the sizes are invalid)
static int lr_block(const sfk_params *p, int64_t n) {
  if (p->lr_rows < 1 || n % p->lr_rows) return 0;
  const int64_t nr = p->lr_rows, nc = n / nr, mn = std::min(nr, nc);
  int64_t l;
  if (p->lr_over > 0) l = (int64_t)p->lr_rank + p->lr_over;
  else if (p->tau == SFK_TAU_LOWRANK)
    l = std::min<int64_t>(std::max<int64_t>(2 * (int64_t)p->lr_rank, (int64_t)p->lr_rank + 16), kLrMaxL);
  else l = (int64_t)p->lr_rank + 10;
  return (int)std::min(l, mn);
}

// checks of the low-rank operators' parameters (n unknowns)
static sfk_status validate_lowrank(sfk_ctx *c, const sfk_params *p, int64_t n, bool multi) {
  if (multi) return fail(c, SFK_EINVAL, "the low-rank tau runs in single-instance contexts");
  if (p->perm) return fail(c, SFK_EINVAL, "the low-rank tau needs the image order (no perm)");
  if (p->driver == SFK_DRIVER_GRAPH)
    return fail(c, SFK_EINVAL, "the low-rank tau runs with the MULTI driver");
  if (p->tape != 0) return fail(c, SFK_EINVAL, "no derivative tape with the low-rank tau");
  if (p->lr_rows < 1 || n % p->lr_rows != 0)
    return fail(c, SFK_EINVAL, "lr_rows %d must divide n = %lld", p->lr_rows, (long long)n);
  const int64_t nr = p->lr_rows, nc = n / nr, mn = std::min(nr, nc);
  if (p->lr_rank < 1 || p->lr_rank >= mn)
    return fail(c, SFK_EINVAL, "lr_rank %d not in [1, min(nr, nc) = %lld) (rank >= min(nr, nc) "
                "is the identity)", p->lr_rank, (long long)mn);
  if (p->lr_over < 0) return fail(c, SFK_EINVAL, "lr_over must be >= 0");
  const int l = lr_block(p, n);
  if (l > kLrMaxL || l < p->lr_rank)
    return fail(c, SFK_EINVAL, "lr_rank + lr_over = %d test vectors exceed %d", l, kLrMaxL);
  if (p->lr_q < 0 || p->lr_q > 16) return fail(c, SFK_EINVAL, "lr_q %d not in [0, 16]", p->lr_q);
  if (p->lr_maxit < 0 || p->lr_maxit > 100000)
    return fail(c, SFK_EINVAL, "lr_maxit %d not in [0, 100000]", p->lr_maxit);
  if (!(p->lr_tol >= 0.0) || !std::isfinite(p->lr_tol))
    return fail(c, SFK_EINVAL, "lr_tol must be finite >= 0");
  return SFK_OK;
}

static int64_t next_pow2(int64_t d) {
  int64_t N = 1;
  while (N < d) N <<= 1;
  return N;
}

static sfk_status validate(sfk_ctx *c, const sfk_csr *A, const sfk_csr *B, const sfk_params *p,
                           bool multi = false) {
  if (!A || !p) return fail(c, SFK_EINVAL, "A and params must not be NULL");
  const int64_t m = A->rows, n = A->cols;
  if (m < 1 || n < 1 || m >= (1ll << 30) || n >= (1ll << 30))
    return fail(c, SFK_EINVAL, "A dimensions %lld x %lld out of range", (long long)m, (long long)n);
  if (A->nnz < 0 || A->nnz >= (1ll << 31))
    return fail(c, SFK_EINVAL, "A nnz %lld out of range [0, 2^31)", (long long)A->nnz);
  if (B) {
    if (B->rows != n || B->cols != m)
      return fail(c, SFK_EINVAL, "B must be %lld x %lld (n x m), got %lld x %lld", (long long)n,
                  (long long)m, (long long)B->rows, (long long)B->cols);
    if (B->nnz < 0 || B->nnz >= (1ll << 31))
      return fail(c, SFK_EINVAL, "B nnz %lld out of range", (long long)B->nnz);
  }
  if (p->method < SFK_SFLSQR || p->method > SFK_FLSMR)
    return fail(c, SFK_EINVAL, "unknown method %d", p->method);
  if (p->method == SFK_FLSQR || p->method == SFK_FLSMR) {
    // full orthogonalisation: no sketch, no window; one instance per context
    if (multi) return fail(c, SFK_EINVAL, "FLSQR / FLSMR run in single-instance contexts");
    if (p->maxit < 1 || p->maxit > 1024)
      return fail(c, SFK_EINVAL, "maxit %d not in [1, 1024] for FLSQR / FLSMR", p->maxit);
    if (p->tau < SFK_TAU_IDENTITY || p->tau > SFK_TAU_LOWRANK_RND)
      return fail(c, SFK_EINVAL, "unknown tau %d", p->tau);
    if (p->tau == SFK_TAU_REWEIGHT_L1 && !(p->eps > 0.0 && std::isfinite(p->eps)))
      return fail(c, SFK_EINVAL, "reweighting needs finite eps > 0");
    if (is_lowrank(p)) {
      sfk_status s = validate_lowrank(c, p, n, multi);
      if (s != SFK_OK) return s;
    }
    if (!(p->eta >= 0.0) || !std::isfinite(p->eta)) return fail(c, SFK_EINVAL, "eta must be finite >= 0");
    if (!(p->noise_norm >= 0.0) || !std::isfinite(p->noise_norm))
      return fail(c, SFK_EINVAL, "noise_norm must be finite >= 0");
    if (!(p->tol >= 0.0) || !std::isfinite(p->tol)) return fail(c, SFK_EINVAL, "tol must be finite >= 0");
    if (p->method == SFK_FLSMR && p->noise_norm > 0.0 && p->resid != 2)
      return fail(c, SFK_EINVAL, "FLSMR's projected residual is not ||b - A x||: for the "
                  "discrepancy principle set resid = 2");
    if (p->resid < 0 || p->resid > 2) return fail(c, SFK_EINVAL, "resid must be 0, 1 or 2");
    if (p->copies != 0 && p->copies != 1) return fail(c, SFK_EINVAL, "copies must be 0 or 1");
    if (p->copies && (p->perm || p->vw == 1)) return fail(c, SFK_EINVAL, "copies = 1 excludes perm and vw = 1");
    if (p->perm) return fail(c, SFK_EINVAL, "FLSQR / FLSMR do not take perm");
    if (p->driver < 0 || p->driver > 2) return fail(c, SFK_EINVAL, "unknown driver %d", p->driver);
    if (p->tape != 0) return fail(c, SFK_EINVAL, "the derivative tape is for sFLSQR");
    return SFK_OK;
  }
  if (p->ell < 0 || p->ell > kMaxEll) return fail(c, SFK_EINVAL, "ell %d not in [0, %d]", p->ell, kMaxEll);
  if (p->s < 1 || p->s > kMaxS) return fail(c, SFK_EINVAL, "s %d not in [1, %d]", p->s, kMaxS);
  if (p->maxit < 1 || p->maxit >= p->s)
    return fail(c, SFK_EINVAL, "maxit %d must satisfy 1 <= maxit < s = %d (the sketched "
                "least-squares problem must stay overdetermined)", p->maxit, p->s);
  const int64_t d = p->method == SFK_SFLSQR ? m : n;
  switch (p->sketch) {
    case SFK_SK_SPARSE_SIGN:
      if (p->zeta < 1 || p->zeta > 64 || p->zeta > p->s)
        return fail(c, SFK_EINVAL, "zeta %d must be in [1, min(s, 64)]", p->zeta);
      if (p->s > d) return fail(c, SFK_EINVAL, "s %d exceeds the sketched length %lld", p->s, (long long)d);
      break;
    case SFK_SK_SRHT:
      if (p->s > next_pow2(d)) return fail(c, SFK_EINVAL, "s %d exceeds the SRHT length", p->s);
      if (next_pow2(d) >= (1ll << 30)) return fail(c, SFK_EINVAL, "SRHT length too large");
      break;
    case SFK_SK_IDENTITY:
      if (p->s != d) return fail(c, SFK_EINVAL, "identity sketch needs s = %lld", (long long)d);
      break;
    default:
      return fail(c, SFK_EINVAL, "unknown sketch kind %d", p->sketch);
  }
  if (p->tau < SFK_TAU_IDENTITY || p->tau > SFK_TAU_LOWRANK_RND)
    return fail(c, SFK_EINVAL, "unknown tau %d", p->tau);
  if (p->tau == SFK_TAU_REWEIGHT_L1 && !(p->eps > 0.0 && std::isfinite(p->eps)))
    return fail(c, SFK_EINVAL, "reweighting needs finite eps > 0");
  if (is_lowrank(p)) {
    sfk_status s = validate_lowrank(c, p, n, multi);
    if (s != SFK_OK) return s;
  }
  if (!(p->eta >= 0.0) || !std::isfinite(p->eta)) return fail(c, SFK_EINVAL, "eta must be finite >= 0");
  if (!(p->noise_norm >= 0.0) || !std::isfinite(p->noise_norm))
    return fail(c, SFK_EINVAL, "noise_norm must be finite >= 0");
  if (!(p->tol >= 0.0) || !std::isfinite(p->tol)) return fail(c, SFK_EINVAL, "tol must be finite >= 0");
  if (p->driver < 0 || p->driver > 2) return fail(c, SFK_EINVAL, "unknown driver %d", p->driver);
  auto vw_ok = [&](int v) {
    return v == -2 || v == -1 || v == 0 || v == 1 || v == 8 || v == 16 || v == 32 || v == 64 ||
           (multi && v == 2);
  };
  if (!vw_ok(p->vw) || (p->vw_split && !vw_ok(p->vw_b)))
    return fail(c, SFK_EINVAL, multi ? "vw must be -2, -1, 0, 1, 2, 8, 16, 32 or 64"
                                     : "vw must be -2, -1, 0, 1, 8, 16, 32 or 64 (2 only for "
                                       "right-hand sides sharing A and B)");
  if (p->vw_split != 0 && p->vw_split != 1) return fail(c, SFK_EINVAL, "vw_split must be 0 or 1");
  if (p->resid < 0 || p->resid > 2) return fail(c, SFK_EINVAL, "resid must be 0, 1 or 2");
  if (p->copies != 0 && p->copies != 1) return fail(c, SFK_EINVAL, "copies must be 0 or 1");
  if (p->tape < 0 || p->tape > p->maxit) return fail(c, SFK_EINVAL, "tape must be in [0, maxit]");
  if (p->tape > 0 && (p->method != SFK_SFLSQR || B != nullptr || p->perm || multi || p->maxit > 1024))
    return fail(c, SFK_EINVAL, "the derivative tape (tape > 0) needs sFLSQR with B = A^T (B NULL), "
                "no perm, maxit <= 1024, in a single-instance context");
  if (p->copies && (p->perm || p->vw == 1 || (p->vw_split && p->vw_b == 1)))
    return fail(c, SFK_EINVAL, "copies = 1 excludes perm and the SELL-64 kernel (vw = 1)");
  if (p->method == SFK_SFLSMR && p->noise_norm > 0.0 && p->resid != 2)
    return fail(c, SFK_EINVAL, "the sketched discrepancy test is defined for sFLSQR; for sFLSMR "
                "set resid = 2 (stop on ||b - A x_k|| <= eta * noise_norm)");
  if (p->wg_per_cu < 0 || p->wg_per_cu > 64) return fail(c, SFK_EINVAL, "wg_per_cu out of range");
  return SFK_OK;
}

extern "C" sfk_status sfk_validate(const sfk_csr *A, const sfk_csr *B, const sfk_params *p) {
  return validate(nullptr, A, B, p);
}

// --------------------------------------------------------------------------
// workspace layout
// --------------------------------------------------------------------------
struct Layout {
  size_t off = 0;
  template <class T>
  size_t take(size_t count) {
    const size_t o = off;
    off += ((count * sizeof(T) + 255) / 256) * 256;
    return o;
  }
};

struct Plan {
  int64_t m, n, nnzA, nnzB;
  int nw, nwmax, vwA, vwB, d, N, log2L, nblk, nchunk;
  bool transpose;
  // offsets
  size_t o_sc, o_err, o_scalar, o_part, o_sigw, o_sigp, o_H, o_T, o_rho;
  size_t o_W, o_P, o_Z, o_wraw, o_zraw, o_x, o_Apart, o_Bpart;
  size_t o_skcode, o_skent, o_skrp, o_chunk, o_srows, o_sd, o_spart, o_SK, o_skrhs;
  size_t o_V, o_tauv, o_R, o_c, o_y, o_ytmp, o_rtrue, o_xres;
  size_t o_Wf, o_Pf, o_fscr, o_gc, o_gs, o_gR, o_gg, o_ck, o_brl, o_mscr;
  size_t o_brp, o_bci, o_bva, o_cursor, o_lr;
  size_t total;
};

// SpMV kernel codes: 0 CSR-stream, 1 SELL-64, 8/16/32/64 lanes per row
static int pick_vw(int64_t nnz, int64_t rows, int user) {
  const double avg = rows > 0 ? (double)nnz / (double)rows : 0.0;
  if (user >= 0) return user;
  if (user == -2) return avg >= 32 ? -2 : 0;  // automatic: timed at init for long rows
  // user == -1: row-parallel with a width from the mean row length
  if (avg >= 96) return 64;
  if (avg >= 40) return 32;
  if (avg >= 16) return 16;
  return 8;
}

// Workgroups of the data-parallel stages: one per 8192 nonzeros, and at least
// one per CU while each still gets 2048 nonzeros (a small operator's product
// is a chain of chunk latencies per workgroup: on the 64^2 workload 230
// workgroups instead of 58 take it from 18.9k to 23.8k iterations/s), one per
// 2048 rows at least; at most one wave of resident workgroups.
static int default_nws(const sfk_csr *A, const sfk_csr *B, const sfk_params *p, int cus,
                       int blocks_per_cu) {
  const int64_t nnzmax = std::max(A->nnz, B ? B->nnz : A->nnz);
  const int cap = cus * (p->wg_per_cu ? p->wg_per_cu : std::max(1, blocks_per_cu));
  int64_t nw = (nnzmax + 8191) / 8192;
  nw = std::max<int64_t>(nw, std::min<int64_t>(cus, (nnzmax + 2047) / 2048));
  nw = std::max<int64_t>(nw, (std::max(A->rows, A->cols) + 2047) / 2048);
  nw = std::min<int64_t>(std::max<int64_t>(nw, 1), cap);
  return (int)nw;
}

// member = true: a right-hand side of a shared-operator group, whose long
// vectors, row partitions and transposed B live in the group's workspace; its
// own x (n) is then contiguous scratch for the true residual.
static Plan make_plan(const sfk_csr *A, const sfk_csr *B, const sfk_params *p, int cus, int nws,
                      bool member = false, bool beam = false) {
  Plan P{};
  P.m = A->rows;
  P.n = A->cols;
  P.nnzA = A->nnz;
  P.transpose = (B == nullptr);
  P.nnzB = B ? B->nnz : A->nnz;
  P.nw = nws;
  P.vwA = pick_vw(P.nnzA, P.m, p->vw);
  P.vwB = pick_vw(P.nnzB, P.n, p->vw_split ? p->vw_b : p->vw);
  P.d = (int)(p->method == SFK_SFLSQR ? P.m : P.n);
  P.N = (int)next_pow2(P.d);
  const int L = std::min(P.N, kSrhtL);
  P.log2L = 0;
  while ((1 << P.log2L) < L) ++P.log2L;
  P.nblk = P.N / L;
  P.nchunk = (P.d + 255) / 256;
  const int64_t m = P.m, n = P.n, s = p->s, mi = p->maxit, ell = p->ell, zeta = p->zeta;
  Layout L_;
  P.o_sc = L_.take<Scal>(1);
  P.o_err = L_.take<int>(1);
  P.o_scalar = L_.take<double>(1);
  // sized for the largest grid any occupancy could give, so that the workspace size
  // does not depend on the device's register allocation
  const int nw_alloc = std::max(P.nw, cus * 8);
  P.nwmax = nw_alloc;
  P.o_part = L_.take<double>((size_t)kNumPart * kMaxQ * nw_alloc);
  P.o_sigw = L_.take<double>(mi + 2);
  P.o_sigp = L_.take<double>(mi + 2);
  P.o_H = L_.take<double>((mi + 1) * mi);
  P.o_T = L_.take<double>((mi + 1) * (mi + 1));
  P.o_rho = L_.take<double>(mi);
  const int64_t vm = member ? 0 : 1;
  P.o_W = L_.take<double>(vm * (ell + 2) * m + 1);
  P.o_P = L_.take<double>(p->tau != SFK_TAU_IDENTITY ? vm * (ell + 1) * n + 1 : 1);
  P.o_Z = L_.take<double>(vm * (mi + 1) * n + 1);      // z~_1 .. z~_{maxit+1}
  P.o_wraw = L_.take<double>(vm * kRawSlots * m + 1);
  P.o_zraw = L_.take<double>(vm * kRawSlots * std::max<int64_t>(n, (P.N + 1) / 2 + 1) + 1);
  P.o_x = L_.take<double>(n);
  P.o_Apart = L_.take<int>(vm * (nw_alloc + 1) + 1);
  P.o_Bpart = L_.take<int>(vm * (nw_alloc + 1) + 1);
  const bool ss = p->sketch == SFK_SK_SPARSE_SIGN;
  const bool sr = p->sketch == SFK_SK_SRHT;
  P.o_skcode = L_.take<int>(ss ? zeta * P.d : 1);
  P.o_skent = L_.take<int>(ss ? zeta * P.d : 1);
  P.o_skrp = L_.take<int>(s + 1);
  P.o_chunk = L_.take<int>(ss ? (size_t)P.nchunk * s : 1);
  P.o_srows = L_.take<int>(sr ? s : 1);
  P.o_sd = L_.take<unsigned long long>(sr ? P.N / 64 + 1 : 1);
  P.o_spart = L_.take<double>(sr ? (size_t)P.nblk * s : 1);
  P.o_SK = L_.take<double>(s * (mi + 1));
  P.o_skrhs = L_.take<double>(s);
  P.o_V = L_.take<double>(s * mi);
  P.o_tauv = L_.take<double>(mi);
  P.o_R = L_.take<double>(mi * mi);
  P.o_c = L_.take<double>(s);
  P.o_y = L_.take<double>(mi);
  P.o_ytmp = L_.take<double>(mi);
  P.o_rtrue = L_.take<double>(p->resid ? mi : 1);
  P.o_xres = L_.take<double>(p->resid ? n : 1);
  const bool full = p->method == SFK_FLSQR || p->method == SFK_FLSMR;
  P.o_Wf = L_.take<double>(full ? (mi + 1) * m : 1);
  P.o_Pf = L_.take<double>(full ? (mi + 1) * n : 1);
  P.o_fscr = L_.take<double>(full ? full_scratch_doubles((int)mi) : 1);
  P.o_gc = L_.take<double>(full ? mi : 1);
  P.o_gs = L_.take<double>(full ? mi : 1);
  P.o_gR = L_.take<double>(full ? mi * mi : 1);
  P.o_gg = L_.take<double>(full ? mi + 1 : 1);
  P.o_ck = L_.take<double>(adjoint_checkpoint_doubles((int)mi, p->tape, (int)ell, (int)m));
  P.o_brl = L_.take<double>(beam ? 2 * m : 1);
  P.o_mscr = L_.take<double>(beam ? m : 1);
  P.o_lr = L_.take<double>(is_lowrank(p) ? lr_doubles(p->lr_rows, (int)(n / p->lr_rows), p->lr_rank,
                                                      lr_block(p, n)) : 1);
  if (P.transpose && !member) {
    P.o_brp = L_.take<int>(n + 1);
    P.o_bci = L_.take<int>(P.nnzB);
    P.o_bva = L_.take<double>(P.nnzB);
    P.o_cursor = L_.take<int>(n);
  }
  P.total = L_.off;
  return P;
}

static int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return cus;
}

static bool is_full(const sfk_params &p) { return p.method == SFK_FLSQR || p.method == SFK_FLSMR; }

// The parameters the library works with: FLSQR / FLSMR draw no sketch (an
// internal kind without arrays) and keep no window.
static sfk_params internal_params(const sfk_params &p) {
  sfk_params q = p;
  if (is_full(p)) {
    q.sketch = 3;
    q.s = 1;
    q.zeta = 1;
    q.ell = 0;
  }
  return q;
}

extern "C" size_t sfk_workspace_bytes(const sfk_csr *A, const sfk_csr *B, const sfk_params *p) {
  if (validate(nullptr, A, B, p) != SFK_OK) return 0;
  int cus = device_cus();
  if (cus <= 0) cus = 256;
  const sfk_params q = internal_params(*p);
  return make_plan(A, B, &q, cus, default_nws(A, B, &q, cus, 2)).total;
}

// --------------------------------------------------------------------------
// init
// --------------------------------------------------------------------------
template <class T>
static T *at(void *base, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

static sfk_status read_scal(sfk_ctx *c) {
  const int nb = (int)c->inst.size();
  for (int i = 0; i < nb; ++i)
    HIPCHK(c, hipMemcpyAsync(c->h_scal + i, c->inst[i].D.sc, sizeof(Scal), hipMemcpyDeviceToHost,
                             c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < nb; ++i) {
    Inst &I = c->inst[i];
    const Scal &S = c->h_scal[i];
    I.k_done = S.k_done;
    I.stopped = S.stopped;
    I.breakdown = S.breakdown;
    I.halted = S.halt || S.klimit <= S.k_done;
    I.rhsnorm = S.rhsnorm;
  }
  return SFK_OK;
}

// SELL-64 copy of one operator (rows x cols CSR on the device), memory owned by
// the context.  *ok = false when padding would grow the copy beyond 1.5x the
// nonzeros (rows of very uneven length in one slice) or past 32-bit indices;
// the CSR-stream kernel is used instead.
static sfk_status build_sell(sfk_ctx *c, const int *rp, const int *ci, const double *va, int rows,
                             int cols, int64_t nnz, int *nsl_out, const int **soff_out,
                             const int **slen_out, const int **scol_out,
                             const uint16_t **scol16_out, const double **sval_out, bool *ok) {
  // (the allocations are the last one or two entries of c->xmem)
  hipStream_t st = c->stream;
  *ok = false;
  const int nsl = (rows + kSellC - 1) / kSellC;
  void *meta = nullptr;
  HIPCHK(c, lib_malloc(c, &meta, sizeof(int) * (2 * (size_t)nsl + 1)));
  int *slen = static_cast<int *>(meta), *soff = slen + nsl;
  launch_sell_len(rp, rows, nsl, slen, st);
  std::vector<int> h(nsl);
  HIPCHK(c, hipMemcpyAsync(h.data(), slen, sizeof(int) * nsl, hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  std::vector<int> hoff(nsl + 1);
  int64_t tot = 0;
  for (int q = 0; q < nsl; ++q) {
    hoff[q] = (int)std::min<int64_t>(tot, (1ll << 31) - 1);
    tot += (int64_t)h[q] * kSellC;
  }
  if (tot >= (1ll << 31) || (double)tot > 1.5 * (double)nnz + 64.0 * kSellC * kSellPad) return SFK_OK;
  hoff[nsl] = (int)tot;
  HIPCHK(c, hipMemcpyAsync(soff, hoff.data(), sizeof(int) * (nsl + 1), hipMemcpyHostToDevice, st));
  // values, 32-bit columns and, for at most 65536 columns, a 16-bit copy
  const bool narrow = cols <= 65536;
  const size_t tot1 = (size_t)std::max<int64_t>(tot, 1);
  void *mem = nullptr;
  HIPCHK(c, lib_malloc(c, &mem, tot1 * (sizeof(int) + sizeof(double) + (narrow ? sizeof(uint16_t) : 0))));
  double *sval = static_cast<double *>(mem);
  int *scol = reinterpret_cast<int *>(sval + tot1);
  uint16_t *scol16 = narrow ? reinterpret_cast<uint16_t *>(scol + tot1) : nullptr;
  launch_sell_fill(rp, ci, va, rows, soff, slen, scol, sval, st);
  if (narrow) launch_to_u16(scol, scol16, tot, st);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(st));
  *nsl_out = nsl;
  *soff_out = soff;
  *slen_out = slen;
  *scol_out = scol;
  *scol16_out = scol16;
  *sval_out = sval;
  *ok = true;
  return SFK_OK;
}

// Builds the instance's sketch from its seed and computes beta = ||b||, w~_1 = b
// (Algorithm 1 / 2, first line).
static sfk_status setup_sketch_and_b(sfk_ctx *c, Inst &I, hipStream_t st) {
  const sfk_params &p = I.p;
  Dev &D = I.D;
  const uint64_t key0 = p.seed;
  const uint64_t key1 = 0ull + ((uint64_t)(uint32_t)p.instance << 32);
  const uint64_t key1_rows = 1ull + ((uint64_t)(uint32_t)p.instance << 32);
  // SRHT: the row draw permutes an index array of N ints held in the (not yet
  // used) raw product buffer
  int *scratch = p.sketch == SFK_SK_SPARSE_SIGN ? I.chunk_scratch : reinterpret_cast<int *>(D.zraw);
  launch_sketch_build(D, key0, key1, key1_rows, scratch, I.d_err, st);
  int herr = 0;
  HIPCHK(c, hipMemcpyAsync(&herr, I.d_err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  if (herr) return fail(c, SFK_EINVAL, "initialisation failed (code %d): transposed rows longer "
                        "than 4096 entries or sketch generation exhausted", herr);
  HIPCHK(c, hipGetLastError());
  const int use_disc = (p.method == SFK_SFLSQR && p.noise_norm > 0.0) ? 1 : 0;
  launch_init_b(D, p.eta, p.noise_norm, p.tol, use_disc, st);
  return SFK_OK;
}

// Carves the workspace of one instance, checks its CSR structures, builds B = A^T
// if needed, the row partitions and the sketch, and computes beta = ||b||.
// grp != NULL: right-hand side r of a shared-operator group whose shared
// arrays (vectors, partitions, B) are already set up.
// Copies of the operators in the caller's order of the unknowns
// (sfk_params.perm): A' has column j renamed perm[j] (each row re-sorted by
// column), B' (when B is given) has row i moved to row perm[i]; also a copy of
// perm (read by the sketches of n-vectors) and its inverse (the solution
// output).  Memory owned by the context.  *bci is left NULL when B is NULL.
static sfk_status relabel(sfk_ctx *c, const int *perm, const sfk_csr *A, const sfk_csr *B,
                          int *err, const int **perm_copy, const int **pinv, const int **aci,
                          const double **ava, const int **brp, const int **bci,
                          const double **bva) {
  hipStream_t st = c->stream;
  const int m = (int)A->rows, n = (int)A->cols;
  auto alloc = [&](void **q, size_t bytes) -> sfk_status {
    HIPCHK(c, lib_malloc(c, q, std::max<size_t>(bytes, 256)));
    return SFK_OK;
  };
  void *pc = nullptr, *pi = nullptr, *cnt = nullptr;
  sfk_status e = alloc(&pc, sizeof(int) * (size_t)n);
  if (e == SFK_OK) e = alloc(&pi, sizeof(int) * (size_t)n);
  if (e == SFK_OK) e = alloc(&cnt, sizeof(int) * (size_t)n);   // released below
  if (e != SFK_OK) return e;
  HIPCHK(c, hipMemcpyAsync(pc, perm, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemsetAsync(cnt, 0, sizeof(int) * (size_t)n, st));
  HIPCHK(c, hipMemsetAsync(err, 0, sizeof(int), st));
  launch_perm_check(static_cast<int *>(pc), n, static_cast<int *>(cnt), static_cast<int *>(pi), err,
                    st);
  int herr = 0;
  HIPCHK(c, hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  lib_pop(c);   // cnt
  if (herr) return fail(c, SFK_EINVAL, "perm must hold each of 0..n-1 exactly once");
  void *ca = nullptr, *va = nullptr;
  e = alloc(&ca, sizeof(int) * (size_t)A->nnz);
  if (e == SFK_OK) e = alloc(&va, sizeof(double) * (size_t)A->nnz);
  if (e != SFK_OK) return e;
  launch_relabel_cols(A->rowptr, A->colind, A->val, m, (int)A->nnz, static_cast<int *>(pc),
                      static_cast<int *>(ca), static_cast<double *>(va), err, st);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  if (herr) return fail(c, SFK_EINVAL, "with perm, rows of A may have at most 4096 entries");
  *perm_copy = static_cast<const int *>(pc);
  *pinv = static_cast<const int *>(pi);
  *aci = static_cast<const int *>(ca);
  *ava = static_cast<const double *>(va);
  *bci = nullptr;
  if (B) {
    void *rb = nullptr, *cb = nullptr, *vb = nullptr;
    e = alloc(&rb, sizeof(int) * ((size_t)n + 1));
    if (e == SFK_OK) e = alloc(&cb, sizeof(int) * (size_t)B->nnz);
    if (e == SFK_OK) e = alloc(&vb, sizeof(double) * (size_t)B->nnz);
    if (e != SFK_OK) return e;
    launch_perm_rows(B->rowptr, B->colind, B->val, n, static_cast<int *>(pc), static_cast<int *>(rb),
                     static_cast<int *>(cb), static_cast<double *>(vb), st);
    HIPCHK(c, hipGetLastError());
    *brp = static_cast<const int *>(rb);
    *bci = static_cast<const int *>(cb);
    *bva = static_cast<const double *>(vb);
  }
  return SFK_OK;
}

static sfk_status setup_instance(sfk_ctx *c, Inst &I, const sfk_csr *A, const sfk_csr *B,
                                 const double *b, void *workspace, size_t ws_bytes, int cus,
                                 int nws, const Grp *grp = nullptr, int r = 0,
                                 const sfk_beam *beam = nullptr) {
  const sfk_params &p = I.p;
  if (!beam && ((A->nnz > 0 && (!A->rowptr || !A->colind || !A->val)) || !A->rowptr))
    return fail(c, SFK_EINVAL, "A arrays must be device pointers");
  if (!b) return fail(c, SFK_EINVAL, "b must be a device pointer");
  if (!beam && B && ((B->nnz > 0 && (!B->colind || !B->val)) || !B->rowptr))
    return fail(c, SFK_EINVAL, "B arrays must be device pointers");
  const Plan P = make_plan(A, B, &p, cus, nws, grp != nullptr, beam != nullptr);
  if (workspace) {
    if (ws_bytes < P.total)
      return fail(c, SFK_ENOMEM, "workspace of %zu bytes is smaller than the %zu required",
                  ws_bytes, P.total);
    I.ws = workspace;
    I.owns_ws = false;
  } else {
    hipError_t e = hipMalloc(&I.ws, P.total);
    if (e != hipSuccess) {
      I.ws = nullptr;
      return fail(c, SFK_ENOMEM, "hipMalloc of %zu bytes failed: %s", P.total, hipGetErrorString(e));
    }
    I.owns_ws = true;
  }
  I.ws_bytes = P.total;
  void *w = I.ws;
  hipStream_t st = c->stream;
  launch_zero_bytes(w, P.total, st);

  Dev &D = I.D;
  std::memset(&D, 0, sizeof D);
  D.m = (int)P.m;
  D.n = (int)P.n;
  D.s = p.s;
  D.ell = p.ell;
  D.maxit = p.maxit;
  D.method = p.method;
  D.tau = p.tau;
  D.sketch = p.sketch;
  D.zeta = p.zeta;
  D.d_sk = P.d;
  D.resid = p.resid;
  D.N = P.N;
  D.log2L = P.log2L;
  D.nblk = P.nblk;
  D.nws = P.nw;
  D.nwv = P.nw;
  D.vs = 1;
  D.vwA = P.vwA;
  D.vwB = P.vwB;
  // non-temporal operator loads in CSR-stream once the nonzeros exceed the
  // 256 MB last-level cache (they cannot stay there; the gathered vector can)
  {
    const int64_t llc = 256ll << 20;
    D.ntA = P.nnzA * (8 + (P.n <= 65536 ? 2 : 4)) > llc ? 1 : 0;
    D.ntB = P.nnzB * (8 + (P.m <= 65536 ? 2 : 4)) > llc ? 1 : 0;
  }
  D.nwmax = P.nwmax;
  D.nsg = p.sketch == SFK_SK_SPARSE_SIGN ? p.s                       // a workgroup per sketch row
        : p.sketch == SFK_SK_IDENTITY ? (p.s + kWG - 1) / kWG : 0;
  D.eps = p.eps;
  D.sk_scale = p.sketch == SFK_SK_SPARSE_SIGN ? 1.0 / std::sqrt((double)p.zeta)
             : p.sketch == SFK_SK_SRHT ? 1.0 / std::sqrt((double)p.s) : 1.0;
  D.Arp = A->rowptr; D.Aci = A->colind; D.Ava = A->val;
  D.b = b;
  D.Apart = at<int>(w, P.o_Apart);
  D.Bpart = at<int>(w, P.o_Bpart);
  D.W = at<double>(w, P.o_W);
  D.P = at<double>(w, P.o_P);
  D.Z = at<double>(w, P.o_Z);
  D.wraw = at<double>(w, P.o_wraw);
  D.zraw = at<double>(w, P.o_zraw);
  D.x = at<double>(w, P.o_x);
  D.sk_rp = at<int>(w, P.o_skrp);
  D.sk_ent = at<int>(w, P.o_skent);
  D.sk_code = at<int>(w, P.o_skcode);
  D.srht_rows = at<int>(w, P.o_srows);
  D.srht_d = at<unsigned long long>(w, P.o_sd);
  D.srht_part = at<double>(w, P.o_spart);
  D.SK = at<double>(w, P.o_SK);
  D.skrhs = at<double>(w, P.o_skrhs);
  D.part = at<double>(w, P.o_part);
  D.sc = at<Scal>(w, P.o_sc);
  D.sigw = at<double>(w, P.o_sigw);
  D.sigp = at<double>(w, P.o_sigp);
  D.H = at<double>(w, P.o_H);
  D.T = at<double>(w, P.o_T);
  D.rho = at<double>(w, P.o_rho);
  D.V = at<double>(w, P.o_V);
  D.tauv = at<double>(w, P.o_tauv);
  D.R = at<double>(w, P.o_R);
  D.c = at<double>(w, P.o_c);
  D.y = at<double>(w, P.o_y);
  D.rtrue = at<double>(w, P.o_rtrue);
  D.xres = at<double>(w, P.o_xres);
  D.Wf = at<double>(w, P.o_Wf);
  D.Pf = at<double>(w, P.o_Pf);
  D.fscr = at<double>(w, P.o_fscr);
  D.gc = at<double>(w, P.o_gc);
  D.gs = at<double>(w, P.o_gs);
  D.gR = at<double>(w, P.o_gR);
  D.gg = at<double>(w, P.o_gg);
  D.tape = p.tape;
  D.ck = at<double>(w, P.o_ck);
  D.brl = at<double>(w, P.o_brl);
  D.mscr = at<double>(w, P.o_mscr);
  I.d_err = at<int>(w, P.o_err);
  I.d_scalar = at<double>(w, P.o_scalar);
  I.d_ytmp = at<double>(w, P.o_ytmp);
  I.chunk_scratch = at<int>(w, P.o_chunk);
  if (is_lowrank(&p)) {
    LrBufs &L = I.lr;
    L.nr = p.lr_rows;
    L.nc = (int)(P.n / p.lr_rows);
    L.r = p.lr_rank;
    L.l = lr_block(&p, P.n);
    L.rnd = p.tau == SFK_TAU_LOWRANK_RND ? 1 : 0;
    L.q = p.lr_q;
    L.maxit = p.lr_maxit > 0 ? p.lr_maxit : 300;
    L.check = 4;
    L.tol = p.lr_tol > 0.0 ? p.lr_tol : 1e-13;
    L.seed = p.seed;
    L.instance = p.instance;
    lr_carve(L, at<double>(w, P.o_lr));
    I.lowrank = true;
  }

  if (grp) {
    D.skperm = p.method == SFK_SFLSMR ? c->gperm : nullptr;
    D.pinv = c->gpinv;
    D.vs = grp->RS;
    D.W = grp->W + r;
    D.P = grp->P + r;
    D.Z = grp->Z + r;
    D.wraw = grp->wraw + r;
    D.zraw = grp->zraw + r;
    D.Brp = grp->Brp; D.Bci = grp->Bci; D.Bva = grp->Bva;
    D.Apart = grp->Apart;
    D.Bpart = grp->Bpart;
    return setup_sketch_and_b(c, I, st);
  }

  if (beam) {
    // matrix-free operators: directions, per-ray intervals, even row ranges
    D.bN = beam->N; D.bNz = beam->nz; D.bNa = beam->n_angles; D.bNd = beam->n_det;
    D.bBack = beam->back; D.bCos = beam->cos_a; D.bSin = beam->sin_a;
    D.Arp = nullptr; D.Aci = nullptr; D.Ava = nullptr;
    D.vwA = D.vwB = 3;
    launch_beam_rays(D, st);
    launch_uniform_part(D.m, D.nws, at<int>(w, P.o_Apart), st);
    launch_uniform_part(D.n, D.nws, at<int>(w, P.o_Bpart), st);
    HIPCHK(c, hipGetLastError());
    return setup_sketch_and_b(c, I, st);
  }
  // structure checks
  launch_csr_check(A->rowptr, A->colind, D.m, D.n, A->nnz, I.d_err, st);
  if (B) {
    launch_csr_check(B->rowptr, B->colind, D.n, D.m, B->nnz, I.d_err, st);
    D.Brp = B->rowptr; D.Bci = B->colind; D.Bva = B->val;
  }
  int herr = 0;
  HIPCHK(c, hipMemcpyAsync(&herr, I.d_err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  if (herr) return fail(c, SFK_EINVAL, "invalid CSR structure (code %d): row pointers must rise "
                        "from 0 to nnz and column indices lie in range", herr);
  if (p.perm) {
    const int *pc = nullptr, *pinv = nullptr, *aci = nullptr, *brp = nullptr, *bci = nullptr;
    const double *ava = nullptr, *bva = nullptr;
    sfk_status e = relabel(c, p.perm, A, B, I.d_err, &pc, &pinv, &aci, &ava, &brp, &bci, &bva);
    if (e != SFK_OK) return e;
    I.user_aci = A->colind;
    I.user_ava = A->val;
    D.Aci = aci;
    D.Ava = ava;
    if (B) { D.Brp = brp; D.Bci = bci; D.Bva = bva; }
    D.skperm = p.method == SFK_SFLSMR ? pc : nullptr;
    D.pinv = pinv;
  }
  if (!B) {
    int *brp = at<int>(w, P.o_brp);
    int *bci = at<int>(w, P.o_bci);
    double *bva = at<double>(w, P.o_bva);
    launch_transpose(D.Arp, D.Aci, D.Ava, D.m, D.n, brp, bci, bva, at<int>(w, P.o_cursor),
                     I.d_err, st);
    D.Brp = brp; D.Bci = bci; D.Bva = bva;
  }
  launch_partition(D.Arp, D.m, P.nnzA, D.nws, at<int>(w, P.o_Apart), st);
  launch_partition(D.Brp, D.n, P.nnzB, D.nws, at<int>(w, P.o_Bpart), st);
  // 16-bit column indices for an operator with at most 65536 columns: the
  // CSR-stream and SELL-64 products read 10 bytes per stored nonzero instead of 12
  for (int op = 0; op < 2; ++op) {
    const bool isa = op == 0;
    const int64_t cols = isa ? D.n : D.m, nnz = isa ? P.nnzA : P.nnzB;
    if (cols > 65536 || nnz <= 0 || p.copies) continue;
    void *m16 = nullptr;
    HIPCHK(c, lib_malloc(c, &m16, sizeof(uint16_t) * (size_t)nnz));
    launch_to_u16(isa ? D.Aci : D.Bci, static_cast<uint16_t *>(m16), nnz, st);
    (isa ? D.Aci16 : D.Bci16) = static_cast<const uint16_t *>(m16);
  }
  HIPCHK(c, hipGetLastError());
  // SpMV kernel per operator: an explicit choice is taken as given (SELL-64
  // falls back to CSR-stream when its copy is refused); the automatic choice
  // times the cores of CSR-stream, wave-per-row and SELL-64 on scratch vectors
  // and keeps the fastest.
  for (int op = 0; op < 2; ++op) {
    const bool isa = op == 0;
    int &vw = isa ? D.vwA : D.vwB;
    if (vw != 1 && vw != -2) continue;
    const bool tune = vw == -2;
    const size_t mark = c->xmem.size();
    bool ok = false;
    sfk_status e = p.copies ? SFK_OK
                 : isa ? build_sell(c, D.Arp, D.Aci, D.Ava, D.m, D.n, P.nnzA, &D.Ansl, &D.Asoff,
                                    &D.Aslen, &D.Ascol, &D.Ascol16, &D.Asval, &ok)
                       : build_sell(c, D.Brp, D.Bci, D.Bva, D.n, D.m, P.nnzB, &D.Bnsl, &D.Bsoff,
                                    &D.Bslen, &D.Bscol, &D.Bscol16, &D.Bsval, &ok);
    if (e != SFK_OK) return e;
    if (!tune) {
      vw = ok ? 1 : 0;
      continue;
    }
    // scratch (all zeros at this point): A reads Z ((maxit + 1) n >= n entries)
    // and writes the raw A-product buffer (2 m); B reads the W ring
    // ((ell + 2) m >= m) and writes the raw B-product buffer (>= 2 n)
    const double *x = isa ? D.Z : D.W;
    double *y = isa ? D.wraw : D.zraw;
    const int cand[3] = {0, 64, 1};
    float best = 1e30f;
    int pick = 0;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    for (int q = 0; q < 3; ++q) {
      if (cand[q] == 1 && !ok) continue;
      launch_spmv_core(D, isa, cand[q], x, y, st);          // warm-up
      HIPCHK(c, hipEventRecord(e0, st));
      for (int rep = 0; rep < 4; ++rep) launch_spmv_core(D, isa, cand[q], x, y, st);
      HIPCHK(c, hipEventRecord(e1, st));
      HIPCHK(c, hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) { best = ms; pick = cand[q]; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    HIPCHK(c, hipGetLastError());
    vw = pick;
    if (pick != 1) {          // the SELL copy lost (or was refused): release it
      HIPCHK(c, hipStreamSynchronize(st));
      while (c->xmem.size() > mark) lib_pop(c);
      if (isa) D.Ascol16 = nullptr; else D.Bscol16 = nullptr;
    }
  }
  return setup_sketch_and_b(c, I, st);
}
// Uploads the instance descriptors and the block maps of every stage type.
static sfk_status build_launch(sfk_ctx *c) {
  const int nb = (int)c->inst.size();
  std::vector<int2> ms, mv, mg, mb, mc;
  int smax = 0, maxitmax = 0;
  if (c->multi) {
    // right-hand sides of one group have identical sketch shapes; ordering the
    // sketch blocks tile-major puts the blocks that read the same interleaved
    // rows next to each other
    const Dev &D0 = c->inst[0].D;
    for (int w = 0; w < D0.nsg; ++w)
      for (int i = 0; i < nb; ++i) mg.push_back(make_int2(i, w));
    if (D0.sketch == SFK_SK_SRHT) {
      for (int w = 0; w < D0.nblk; ++w)
        for (int i = 0; i < nb; ++i) mb.push_back(make_int2(i, w));
      for (int w = 0; w < (D0.s + kWG - 1) / kWG; ++w)
        for (int i = 0; i < nb; ++i) mc.push_back(make_int2(i, w));
    }
  }
  for (int i = 0; i < nb; ++i) {
    const Dev &D = c->inst[i].D;
    if (!c->multi) {
      for (int w = 0; w < D.nws; ++w) ms.push_back(make_int2(i, w));
      for (int w = 0; w < D.nwv; ++w) mv.push_back(make_int2(i, w));
      for (int w = 0; w < D.nsg; ++w) mg.push_back(make_int2(i, w));
      if (D.sketch == SFK_SK_SRHT) {
        for (int w = 0; w < D.nblk; ++w) mb.push_back(make_int2(i, w));
        for (int w = 0; w < (D.s + kWG - 1) / kWG; ++w) mc.push_back(make_int2(i, w));
      }
    }
    smax = std::max(smax, D.s);
    maxitmax = std::max(maxitmax, D.maxit);
    if (D.method == SFK_SFLSMR) c->sketch_after_C = true;
    if (D.tau == SFK_TAU_REWEIGHT_L1) c->any_rew = true;
    if (c->inst[i].p.driver == SFK_DRIVER_GRAPH) c->graph = true;
  }
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  const size_t o_dev = 0;
  const size_t o_ms = al(o_dev + sizeof(Dev) * nb);
  const size_t o_mv = al(o_ms + sizeof(int2) * ms.size());
  const size_t o_mg = al(o_mv + sizeof(int2) * mv.size());
  const size_t o_mb = al(o_mg + sizeof(int2) * mg.size());
  const size_t o_mc = al(o_mb + sizeof(int2) * mb.size());
  const size_t total = al(o_mc + sizeof(int2) * mc.size()) + 256;
  HIPCHK(c, hipMalloc(&c->hdr, total));
  c->hdr_bytes = total;
  std::vector<char> h(total, 0);
  for (int i = 0; i < nb; ++i) std::memcpy(h.data() + o_dev + sizeof(Dev) * i, &c->inst[i].D, sizeof(Dev));
  auto put = [&](size_t off, const std::vector<int2> &v) {
    if (!v.empty()) std::memcpy(h.data() + off, v.data(), sizeof(int2) * v.size());
  };
  put(o_ms, ms); put(o_mv, mv); put(o_mg, mg); put(o_mb, mb); put(o_mc, mc);
  HIPCHK(c, hipMemcpyAsync(c->hdr, h.data(), total, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  Launch &L = c->L;
  char *base = static_cast<char *>(c->hdr);
  L.devs = reinterpret_cast<const Dev *>(base + o_dev);
  L.map_spmv = reinterpret_cast<const int2 *>(base + o_ms);
  L.map_vec = reinterpret_cast<const int2 *>(base + o_mv);
  L.map_sg = reinterpret_cast<const int2 *>(base + o_mg);
  L.map_sb = reinterpret_cast<const int2 *>(base + o_mb);
  L.map_sc = reinterpret_cast<const int2 *>(base + o_mc);
  L.nspmv = (int)ms.size();
  L.nvec = (int)mv.size();
  L.nsg = (int)mg.size();
  L.nsb = (int)mb.size();
  L.nsc = (int)mc.size();
  L.ninst = nb;
  L.smax = smax;
  L.maxitmax = maxitmax;
  L.tau = c->any_rew ? 1 : 0;
  L.ellmax = 0;
  for (int i = 0; i < nb; ++i) L.ellmax = std::max(L.ellmax, c->inst[i].D.ell);
  // one launch serves every instance, so all run one SpMV kernel: instance 0's
  // when every instance has its data, else CSR-stream (valid for all)
  L.vwA = c->inst[0].D.vwA;
  L.vwB = c->inst[0].D.vwB;
  for (int i = 1; i < nb; ++i) {
    if (c->inst[i].D.vwA != L.vwA) L.vwA = 0;
    if (c->inst[i].D.vwB != L.vwB) L.vwB = 0;
  }
  c->maxitmax = maxitmax;
  c->grp.devs = L.devs;
  return SFK_OK;
}

static sfk_status create_streams(sfk_ctx *c, int nb) {
  HIPCHK(c, hipHostMalloc((void **)&c->h_scal, sizeof(Scal) * nb, hipHostMallocDefault));
  HIPCHK(c, hipHostMalloc((void **)&c->h_halt, sizeof(int) * sfk_ctx::kChkSlots * nb,
                          hipHostMallocDefault));
  HIPCHK(c, hipMalloc((void **)&c->d_halt, sizeof(int) * sfk_ctx::kChkSlots * nb));
  for (int i = 0; i < sfk_ctx::kChkSlots; ++i)
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_chk[i], hipEventDisableTiming));
  HIPCHK(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  HIPCHK(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  HIPCHK(c, hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming));
  HIPCHK(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
  for (int i = 0; i < sfk_ctx::kRing; ++i) {
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_main[i], hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_sk[i], hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_ls[i], hipEventDisableTiming));
  }
  return SFK_OK;
}

// Algorithm 1 / 2 initial lines after every instance has its beta: z = B w_1,
// the initial sketch (S b, or S B w_1), the rhs and the first basis vector.
static sfk_status init_common(sfk_ctx *c) {
  sfk_status s = build_launch(c);
  if (s != SFK_OK) return s;
  hipStream_t st = c->stream;
  if (c->full) {
    launch_full_init(c->inst[0].D, c->inst[0].D.vwB, st);
  } else {
    run_stage(c, kStageC, 0, st);
    if (c->tape) launch_checkpoint_w(c->inst[0].D, 0, c->inst[0].D.ck, st);
    launch_sketch(c->L, 0, st);
    for (auto &I : c->inst) launch_init_rhs(I.D, st);
    run_stage(c, kStageD, 0, st);
  }
  if (c->inst[0].lowrank) enqueue_tau(c, 0);
  HIPCHK(c, hipGetLastError());
  s = read_scal(c);
  if (s != SFK_OK) return s;
  for (size_t i = 0; i < c->inst.size(); ++i) {
    const Scal &S = c->h_scal[i];
    if (S.err & 16)
      return fail(c, SFK_EINVAL, "right-hand side b%s is zero or not finite (||b|| = %g)",
                  c->inst.size() > 1 ? " of an instance" : "", S.beta);
  }
  return SFK_OK;
}

static void release(sfk_ctx *c) {
  hipStreamSynchronize(c->stream);
  if (c->side) hipStreamSynchronize(c->side);
  for (int i = 0; i < sfk_ctx::kRing; ++i) {
    if (c->ev_main[i]) hipEventDestroy(c->ev_main[i]);
    if (c->ev_sk[i]) hipEventDestroy(c->ev_sk[i]);
    if (c->ev_ls[i]) hipEventDestroy(c->ev_ls[i]);
  }
  for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
  for (int i = 0; i < sfk_ctx::kChkSlots; ++i)
    if (c->ev_chk[i]) hipEventDestroy(c->ev_chk[i]);
  if (c->ev_join) hipEventDestroy(c->ev_join);
  if (c->ev_fork) hipEventDestroy(c->ev_fork);
  if (c->ev_done) hipEventDestroy(c->ev_done);
  if (c->gexec) hipGraphExecDestroy(c->gexec);
  if (c->d_halt) hipFree(c->d_halt);
  if (c->h_halt) hipHostFree(c->h_halt);
  if (c->side) hipStreamDestroy(c->side);
  if (c->gstream) {
    hipStreamSynchronize(c->gstream);
    hipStreamDestroy(c->gstream);
  }
  for (auto &I : c->inst)
    if (I.owns_ws && I.ws) hipFree(I.ws);
  if (c->gws) hipFree(c->gws);
  for (auto &q : c->xmem) hipFree(q.first);
  if (c->hdr) hipFree(c->hdr);
  if (c->h_scal) hipHostFree(c->h_scal);
  delete c;
}

extern "C" sfk_status sfk_init(sfk_ctx **out, const sfk_csr *A, const sfk_csr *B, const double *b,
                               const sfk_params *p, void *workspace, size_t workspace_bytes,
                               void *stream) {
  if (!out) return fail(nullptr, SFK_EINVAL, "out must not be NULL");
  *out = nullptr;
  sfk_status s = validate(nullptr, A, B, p);
  if (s != SFK_OK) return s;
  const int cus = device_cus();
  if (cus <= 0) return fail(nullptr, SFK_EDEVICE, "no HIP device available");
  sfk_ctx *c = new sfk_ctx();
  c->stream = static_cast<hipStream_t>(stream);
  c->inst.resize(1);
  c->inst[0].p = internal_params(*p);
  c->resid = p->resid;
  c->full = is_full(*p);
  c->tape = p->tape;
  s = create_streams(c, 1);
  if (s == SFK_OK)
    s = setup_instance(c, c->inst[0], A, B, b, workspace, workspace_bytes, cus,
                       default_nws(A, B, p, cus, spmv_blocks_per_cu()));
  if (s == SFK_OK) s = init_common(c);
  if (s != SFK_OK) {
    set_err(g_err, c->err);
    release(c);
    return s;
  }
  *out = c;
  return SFK_OK;
}

extern "C" sfk_status sfk_init_beam(sfk_ctx **out, const sfk_beam *geo, const double *b,
                                    const sfk_params *p, void *workspace, size_t workspace_bytes,
                                    void *stream) {
  if (!out) return fail(nullptr, SFK_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (!geo || !p) return fail(nullptr, SFK_EINVAL, "geometry and params must not be NULL");
  if (geo->N < 1 || geo->nz < 1 || geo->n_angles < 1 || geo->n_det < 1 || !geo->cos_a || !geo->sin_a)
    return fail(nullptr, SFK_EINVAL, "beam geometry: N, nz, n_angles, n_det >= 1 and device "
                "direction arrays required");
  if (geo->back != 0 && geo->back != 1) return fail(nullptr, SFK_EINVAL, "back must be 0 or 1");
  const int64_t m = (int64_t)geo->nz * geo->n_angles * geo->n_det;
  const int64_t n = (int64_t)geo->nz * geo->N * geo->N;
  if (m >= (1ll << 31) || n >= (1ll << 31)) return fail(nullptr, SFK_EINVAL, "beam geometry too large");
  if (p->perm || p->tape || p->vw == 1)
    return fail(nullptr, SFK_EINVAL, "matrix-free operators take no perm, tape or SELL kernel");
  // descriptors of the operators for the size checks and the work split: the
  // number of pieces per ray is at most 2 N + 2
  const int64_t nnz_est = std::min<int64_t>(m * (2 * (int64_t)geo->N + 2), (1ll << 31) - 1);
  const sfk_csr Ad{m, n, nnz_est, nullptr, nullptr, nullptr};
  const sfk_csr Bd{n, m, nnz_est, nullptr, nullptr, nullptr};
  sfk_params q = *p;
  q.vw = 3;
  q.vw_split = 0;
  q.copies = 1;
  sfk_status s = validate(nullptr, &Ad, &Bd, p);
  if (s != SFK_OK) return s;
  const int cus = device_cus();
  if (cus <= 0) return fail(nullptr, SFK_EDEVICE, "no HIP device available");
  sfk_ctx *c = new sfk_ctx();
  c->stream = static_cast<hipStream_t>(stream);
  c->inst.resize(1);
  c->inst[0].p = internal_params(q);
  c->resid = p->resid;
  c->full = is_full(*p);
  s = create_streams(c, 1);
  if (s == SFK_OK)
    s = setup_instance(c, c->inst[0], &Ad, &Bd, b, workspace, workspace_bytes, cus,
                       default_nws(&Ad, &Bd, &q, cus, spmv_blocks_per_cu()), nullptr, 0, geo);
  if (s == SFK_OK) s = init_common(c);
  if (s != SFK_OK) {
    set_err(g_err, c->err);
    release(c);
    return s;
  }
  *out = c;
  return SFK_OK;
}

extern "C" sfk_status sfk_init_batch(sfk_ctx **out, int32_t nb, const sfk_csr *A,
                                     const sfk_csr *B, const double *const *b,
                                     const sfk_params *p, void *stream) {
  if (!out) return fail(nullptr, SFK_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (nb < 1 || nb > 4096) return fail(nullptr, SFK_EINVAL, "batch size %d not in [1, 4096]", nb);
  if (!A || !b || !p) return fail(nullptr, SFK_EINVAL, "A, b and params arrays must not be NULL");
  for (int i = 0; i < nb; ++i) {
    const sfk_csr *Bi = (B && B[i].rows > 0) ? &B[i] : nullptr;
    sfk_status s = validate(nullptr, &A[i], Bi, &p[i]);
    if (s == SFK_OK && p[i].resid != 0)
      s = fail(nullptr, SFK_EINVAL, "resid must be 0 in a batch (single-instance contexts only)");
    if (s == SFK_OK && is_full(p[i]))
      s = fail(nullptr, SFK_EINVAL, "FLSQR / FLSMR run in single-instance contexts");
    if (s == SFK_OK && is_lowrank(&p[i]) && nb > 1)
      s = fail(nullptr, SFK_EINVAL, "the low-rank tau runs in single-instance contexts");
    if (s != SFK_OK) {
      prefix_err(g_err, "instance", i);
      return s;
    }
  }
  const int cus = device_cus();
  if (cus <= 0) return fail(nullptr, SFK_EDEVICE, "no HIP device available");
  // Every instance gets the row partition it would have on its own: while all
  // instances are live the grid is oversubscribed and the hardware balances
  // it; once some have stopped (their workgroups exit at once), the ones still
  // running keep the whole device.
  const int bpc = spmv_blocks_per_cu();
  sfk_ctx *c = new sfk_ctx();
  c->stream = static_cast<hipStream_t>(stream);
  c->inst.resize(nb);
  sfk_status s = create_streams(c, nb);
  for (int i = 0; i < nb && s == SFK_OK; ++i) {
    c->inst[i].p = p[i];
    const sfk_csr *Bi = (B && B[i].rows > 0) ? &B[i] : nullptr;
    const int nws = default_nws(&A[i], Bi, &p[i], cus, bpc);
    s = setup_instance(c, c->inst[i], &A[i], Bi, b[i], nullptr, 0, cus, nws);
    if (s != SFK_OK) prefix_err(c->err, "instance", i);
  }
  if (s == SFK_OK) s = init_common(c);
  if (s != SFK_OK) {
    set_err(g_err, c->err);
    release(c);
    return s;
  }
  *out = c;
  return SFK_OK;
}

// --------------------------------------------------------------------------
// right-hand sides sharing one operator pair
// --------------------------------------------------------------------------
static sfk_status same_params(const sfk_params &a, const sfk_params &b, int r) {
  const char *what = nullptr;
  if (a.method != b.method) what = "method";
  else if (a.ell != b.ell) what = "ell";
  else if (a.maxit != b.maxit) what = "maxit";
  else if (a.sketch != b.sketch) what = "sketch";
  else if (a.s != b.s) what = "s";
  else if (a.sketch == SFK_SK_SPARSE_SIGN && a.zeta != b.zeta) what = "zeta";
  else if (a.tau != b.tau) what = "tau";
  else if (a.tau == SFK_TAU_REWEIGHT_L1 && a.eps != b.eps) what = "eps";
  else if (a.perm != b.perm) what = "perm";
  else if (a.copies != b.copies) what = "copies";
  if (what)
    return fail(nullptr, SFK_EINVAL, "right-hand side %d: '%s' differs from right-hand side 0 "
                "(right-hand sides sharing A and B may differ only in seed, instance, eta, "
                "noise_norm and tol)", r, what);
  return SFK_OK;
}

// Automatic choice of the LDS-staged product: at least this many nonzeros per
// staged source row.
constexpr double kLdsMinReuse = 5.0;
// Work of staging one source row, in records (one L2 read and one LDS write
// of the row against one LDS read of it per record), for the workgroup split.
constexpr int kStageWeight = 2;

// Plans the LDS-staged units of a sliced operator on the host (sfk_units.h)
// and, when taken (mode 2, or mode 1 with at least kLdsMinReuse nonzeros per
// staged row), rewrites the record offsets and uploads the unit tables.
// Leaves X on the gathers (SFK_OK) when a segment reads more source rows than
// a staged block holds.  touch: the scanned slice-major segment ids.
static sfk_status plan_lds(sfk_ctx *c, XOp &X, const int *touch, int RS, int cus, int mode,
                           int64_t nrec) {
  hipStream_t st = c->stream;
  const int rowbytes = RS * (int)sizeof(double);
  const int cap = kLdsRows / rowbytes;
  const int nbw = std::max(1, cus * gspmm_l_blocks_per_cu(RS) / kXcds);
  const int ng = gspmm_x_units_per_block(RS);
  std::vector<int32_t> sbeg(X.NS + 1), seg(4 * (size_t)X.nseg);
  std::vector<XNz> nz((size_t)nrec);
  for (int q = 0; q < X.NS; ++q)
    HIPCHK(c, hipMemcpyAsync(&sbeg[q], touch + (size_t)q * X.rows, sizeof(int),
                             hipMemcpyDeviceToHost, st));
  sbeg[X.NS] = X.nseg;
  HIPCHK(c, hipMemcpyAsync(seg.data(), X.seg, sizeof(int4) * (size_t)X.nseg, hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipMemcpyAsync(nz.data(), X.nz, sizeof(XNz) * (size_t)nrec, hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  std::vector<int32_t> off((size_t)nrec);
  for (int64_t e = 0; e < nrec; ++e) off[e] = nz[e].off;
  UnitPlan P;
  if (!plan_units(X.NS, sbeg.data(), seg.data(), off.data(), nrec, X.cols, rowbytes, kXPadOff,
                  cap, kLdsRecs - kSegAlign, ng, nbw, kStageWeight, P))
    return SFK_OK;
  if (mode == 1 && (double)P.nonzeros < kLdsMinReuse * (double)P.staged) return SFK_OK;
  for (int64_t e = 0; e < nrec; ++e) {
    nz[e].off = P.off[e];
    nz[e].pad = P.endslot[e];
  }
  // device tables: every unit's records at a fixed stride of kLdsRecs (then
  // padding), per unit and lane group the record range inside that block
  const size_t nunit = P.unit.size() / 4;
  std::vector<int32_t> meta, grp;
  unit_tables(P, seg.data(), ng, meta, grp);
  std::vector<XNz> urec(nunit * (size_t)kLdsRecs, XNz{0.0, kLdsRows, -1});
  for (size_t u = 0; u < nunit; ++u) {
    if (meta[2 * u + 1] > kLdsRecs - kSegAlign)
      return fail(c, SFK_EDEVICE, "staged unit larger than planned");
    std::copy(nz.begin() + meta[2 * u], nz.begin() + meta[2 * u] + meta[2 * u + 1],
              urec.begin() + u * (size_t)kLdsRecs);
  }
  Layout L;
  const size_t o_rec = L.take<XNz>(std::max<size_t>(urec.size(), 1));
  const size_t o_stage = L.take<int>(std::max<size_t>(P.stage.size(), 1));
  const size_t o_grp = L.take<int2>(std::max<size_t>(grp.size() / 2, 1));
  const size_t o_upart = L.take<int>(P.upart.size());
  void *mem = nullptr;
  HIPCHK(c, lib_malloc(c, &mem, L.off));
  HIPCHK(c, hipMemcpyAsync(at<XNz>(mem, o_rec), urec.data(), sizeof(XNz) * urec.size(),
                           hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(at<int>(mem, o_stage), P.stage.data(), sizeof(int32_t) * P.stage.size(),
                           hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(at<int2>(mem, o_grp), grp.data(), sizeof(int32_t) * grp.size(),
                           hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(at<int>(mem, o_upart), P.upart.data(), sizeof(int32_t) * P.upart.size(),
                           hipMemcpyHostToDevice, st));
  HIPCHK(c, hipStreamSynchronize(st));
  X.nbw = nbw;
  X.urec = at<XNz>(mem, o_rec);
  X.stage = at<int>(mem, o_stage);
  X.ugrp = at<int2>(mem, o_grp);
  X.upart = at<int>(mem, o_upart);
  return SFK_OK;
}

// Column-sliced copy of one operator (rows x cols CSR on the device) for the
// shared-operator products: slices of at most ~2 MB of source-block rows each,
// a multiple of kXcds of them, nbs workgroups per slice.  *ok = false (and
// SFK_OK) when the operator cannot be sliced (columns not increasing within a
// row, or index ranges beyond 32-bit offsets): the row kernel is used instead.
static sfk_status build_xop(sfk_ctx *c, XOp &X, const int *rp, const int *ci, const double *va,
                            int rows, int cols, int64_t nnz, int RS, int cus, int lds_mode,
                            bool *ok) {
  hipStream_t st = c->stream;
  *ok = false;
  const int64_t cps = std::max<int64_t>(1, (int64_t)(2 << 20) / (RS * (int64_t)sizeof(double)));
  const int64_t per = (int64_t)kXcds * cps;
  const int NS = (int)(kXcds * std::max<int64_t>(1, (cols + per - 1) / per));
  if ((int64_t)NS * rows + 1 >= (1ll << 31) || nnz * 4 + kXPad >= (1ll << 31) ||
      (int64_t)NS * cus * 64 * 16 >= (1ll << 31) ||
      (int64_t)cols * RS * (int64_t)sizeof(double) >= (1ll << 31))
    return SFK_OK;

  const int nbs = std::max(1, cus * gspmm_x_blocks_per_cu(RS) / kXcds);
  const int upb = gspmm_x_units_per_block(RS);     // lane groups per workgroup
  Layout L1;
  const size_t o_cb = L1.take<int>(NS + 1);
  const size_t o_touch = L1.take<int>((size_t)NS * rows + 1);
  const size_t o_err = L1.take<int>(1);
  const size_t s1 = L1.off;
  void *scr = nullptr;
  HIPCHK(c, hipMalloc(&scr, s1));
  struct Guard {
    void *p;
    ~Guard() { if (p) hipFree(p); }
  } g1{scr};
  void *crp_mem = nullptr;
  HIPCHK(c, lib_malloc(c, &crp_mem, sizeof(int) * ((size_t)rows + 1)));
  int *cb = at<int>(scr, o_cb), *touch = at<int>(scr, o_touch), *err = at<int>(scr, o_err);
  int *crp = static_cast<int *>(crp_mem);
  std::vector<int> hcb(NS + 1);
  for (int q = 0; q <= NS; ++q) hcb[q] = (int)((int64_t)q * cols / NS);
  HIPCHK(c, hipMemsetAsync(scr, 0, s1, st));
  HIPCHK(c, hipMemsetAsync(crp, 0, sizeof(int) * ((size_t)rows + 1), st));
  HIPCHK(c, hipMemcpyAsync(cb, hcb.data(), sizeof(int) * (NS + 1), hipMemcpyHostToDevice, st));
  launch_xs_count(rp, ci, rows, NS, cb, touch, crp, err, st);
  int herr = 0;
  HIPCHK(c, hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  if (herr) return SFK_OK;            // unsorted columns: keep the row kernel
  launch_scan(touch, NS * rows + 1, st);
  launch_scan(crp, rows + 1, st);
  int nseg = 0;
  HIPCHK(c, hipMemcpyAsync(&nseg, touch + (size_t)NS * rows, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  if (nseg <= 0) return SFK_OK;       // no nonzeros: keep the row kernel
  Layout L2;
  const size_t o_seg = L2.take<int4>(std::max(nseg, 1));
  const size_t o_spart = L2.take<int>((size_t)NS * ((size_t)nbs * upb + 1));
  // each segment grows by at most kSegAlign - 1 padding nonzeros
  const int64_t nzcap = nnz + (int64_t)nseg * (kSegAlign - 1) + kXPad;
  const size_t o_nz = L2.take<XNz>(nzcap);
  const size_t o_part = L2.take<double>((size_t)std::max(nseg, 1) * RS);
  void *mem = nullptr;
  HIPCHK(c, lib_malloc(c, &mem, L2.off));
  Layout L3;
  const size_t o_len = L3.take<int>((size_t)nseg + 1);
  const size_t o_src = L3.take<int>(std::max(nseg, 1));
  const size_t o_row = L3.take<int>(std::max(nseg, 1));
  const size_t o_slot = L3.take<int>(std::max(nseg, 1));
  const size_t o_cnt = L3.take<int>(std::max(nseg, 1));
  void *scr2 = nullptr;
  HIPCHK(c, hipMalloc(&scr2, L3.off));
  Guard g2{scr2};
  HIPCHK(c, hipMemsetAsync(mem, 0, L2.off, st));
  HIPCHK(c, hipMemsetAsync(scr2, 0, L3.off, st));
  int *seglen = at<int>(scr2, o_len), *segsrc = at<int>(scr2, o_src), *segrow = at<int>(scr2, o_row);
  int *slot = at<int>(scr2, o_slot), *segcnt = at<int>(scr2, o_cnt);
  launch_xs_fill1(rp, ci, rows, NS, cb, touch, crp, slot, seglen, segsrc, segrow, segcnt, st);
  launch_scan(seglen, nseg + 1, st);
  int nzpad = 0;      // nonzeros of the padded copy
  HIPCHK(c, hipMemcpyAsync(&nzpad, seglen + nseg, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  if ((int64_t)nzpad + kXPad > nzcap) return fail(c, SFK_EDEVICE, "sliced copy larger than planned");
  launch_xs_fill2(ci, va, nseg, seglen, segsrc, segrow, segcnt, slot, RS, at<int4>(mem, o_seg),
                  at<XNz>(mem, o_nz), st);
  launch_xs_part(touch, rows, NS, nseg, seglen, nbs * upb, at<int>(mem, o_spart), st);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(st));
  X.rows = rows; X.cols = cols; X.NS = NS; X.nbs = nbs; X.nseg = nseg; X.upb = upb;
  X.seg = at<int4>(mem, o_seg);
  X.spart = at<int>(mem, o_spart);
  X.nz = at<XNz>(mem, o_nz);
  X.crp = crp;
  X.part = at<double>(mem, o_part);
  X.urec = nullptr;
  *ok = true;
  if (lds_mode) return plan_lds(c, X, touch, RS, cus, lds_mode, (int64_t)nzpad + kXPad);
  return SFK_OK;
}

extern "C" sfk_status sfk_init_multi(sfk_ctx **out, const sfk_csr *A, const sfk_csr *B,
                                     const double *b_block, int32_t R, const sfk_params *p,
                                     void *stream) {
  if (!out) return fail(nullptr, SFK_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (R < 1 || R > kMaxRhs) return fail(nullptr, SFK_EINVAL, "R = %d not in [1, %d]", R, kMaxRhs);
  if (!A || !b_block || !p) return fail(nullptr, SFK_EINVAL, "A, b_block and params must not be NULL");
  for (int r = 0; r < R; ++r) {
    sfk_status s = validate(nullptr, A, B, &p[r], true);
    if (s == SFK_OK && p[r].resid != 0)
      s = fail(nullptr, SFK_EINVAL, "resid must be 0 for right-hand sides sharing A and B "
               "(single-instance contexts only)");
    if (s != SFK_OK) {
      prefix_err(g_err, "right-hand side", r);
      return s;
    }
    s = same_params(p[0], p[r], r);
    if (s != SFK_OK) return s;
  }
  if ((A->nnz > 0 && (!A->colind || !A->val)) || !A->rowptr)
    return fail(nullptr, SFK_EINVAL, "A arrays must be device pointers");
  if (B && ((B->nnz > 0 && (!B->colind || !B->val)) || !B->rowptr))
    return fail(nullptr, SFK_EINVAL, "B arrays must be device pointers");
  const int cus = device_cus();
  if (cus <= 0) return fail(nullptr, SFK_EDEVICE, "no HIP device available");
  int RS = 8;
  while (RS < R) RS <<= 1;
  const sfk_params &p0 = p[0];
  const int64_t m = A->rows, n = A->cols, nnzA = A->nnz, nnzB = B ? B->nnz : A->nnz;
  const int64_t ell = p0.ell, mi = p0.maxit;
  const int bpc = gspmm_blocks_per_cu(RS);
  const int cap = cus * (p0.wg_per_cu ? p0.wg_per_cu : bpc);
  int64_t nw64 = std::max((std::max(nnzA, nnzB) + 8191) / 8192, (std::max(m, n) + 2047) / 2048);
  const int nw = (int)std::min<int64_t>(std::max<int64_t>(nw64, 1), cap);
  const int64_t d = p0.method == SFK_SFLSQR ? m : n;
  const int64_t N = next_pow2(d);

  Layout L_;
  const size_t o_err = L_.take<int>(1);
  const size_t o_W = L_.take<double>((ell + 2) * m * RS);
  const size_t o_P = L_.take<double>(p0.tau == SFK_TAU_REWEIGHT_L1 ? (ell + 1) * n * RS : 1);
  const size_t o_Z = L_.take<double>((mi + 1) * n * RS);
  const size_t o_wraw = L_.take<double>(kRawSlots * m * RS);
  const size_t o_zraw = L_.take<double>(kRawSlots * std::max<int64_t>(n, (N + 1) / 2 + 1) * RS);
  const size_t o_x = L_.take<double>(p0.tau == SFK_TAU_REWEIGHT_L1 ? n * RS : 1);
  const size_t o_Apart = L_.take<int>(nw + 1);
  const size_t o_Bpart = L_.take<int>(nw + 1);
  const size_t o_coef = L_.take<double>((size_t)RS * kCoefStride);
  const size_t o_act = L_.take<int>(RS);
  const size_t o_gx = L_.take<double>(p0.tau == SFK_TAU_REWEIGHT_L1 ? mi * RS : 1);
  size_t o_brp = 0, o_bci = 0, o_bva = 0, o_cursor = 0;
  if (!B) {
    o_brp = L_.take<int>(n + 1);
    o_bci = L_.take<int>(nnzB);
    o_bva = L_.take<double>(nnzB);
    o_cursor = L_.take<int>(n);
  }
  const size_t total = L_.off;

  sfk_ctx *c = new sfk_ctx();
  c->stream = static_cast<hipStream_t>(stream);
  c->multi = true;
  c->inst.resize(R);
  sfk_status s = create_streams(c, R);
  hipStream_t st = c->stream;
  Grp &G = c->grp;
  auto setup_group = [&]() -> sfk_status {
    hipError_t e = hipMalloc(&c->gws, total);
    c->gws_bytes = total;
    if (e != hipSuccess) {
      c->gws = nullptr;
      return fail(c, SFK_ENOMEM, "hipMalloc of %zu bytes failed: %s", total, hipGetErrorString(e));
    }
    void *w = c->gws;
    HIPCHK(c, hipMemsetAsync(w, 0, total, st));
    int *err = at<int>(w, o_err);
    G.R = R; G.RS = RS;
    G.m = (int)m; G.n = (int)n; G.ell = p0.ell; G.maxit = p0.maxit; G.tau = p0.tau;
    G.nws = nw; G.nwv = nw; G.eps = p0.eps;
    G.Arp = A->rowptr; G.Aci = A->colind; G.Ava = A->val;
    G.W = at<double>(w, o_W); G.P = at<double>(w, o_P); G.Z = at<double>(w, o_Z);
    G.wraw = at<double>(w, o_wraw); G.zraw = at<double>(w, o_zraw); G.x = at<double>(w, o_x);
    G.Apart = at<int>(w, o_Apart); G.Bpart = at<int>(w, o_Bpart);
    G.coef = at<double>(w, o_coef); G.act = at<int>(w, o_act); G.gx = at<double>(w, o_gx);
    launch_csr_check(A->rowptr, A->colind, (int)m, (int)n, nnzA, err, st);
    if (B) {
      launch_csr_check(B->rowptr, B->colind, (int)n, (int)m, nnzB, err, st);
      G.Brp = B->rowptr; G.Bci = B->colind; G.Bva = B->val;
    }
    int herr = 0;
    HIPCHK(c, hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (herr) return fail(c, SFK_EINVAL, "invalid CSR structure (code %d): row pointers must rise "
                          "from 0 to nnz and column indices lie in range", herr);
    if (p0.perm) {
      const int *brp = nullptr, *bci = nullptr;
      const double *bva = nullptr;
      sfk_status e = relabel(c, p0.perm, A, B, err, &c->gperm, &c->gpinv, &G.Aci, &G.Ava, &brp, &bci,
                             &bva);
      if (e != SFK_OK) return e;
      if (B) { G.Brp = brp; G.Bci = bci; G.Bva = bva; }
    }
    if (!B) {
      int *brp = at<int>(w, o_brp);
      int *bci = at<int>(w, o_bci);
      double *bva = at<double>(w, o_bva);
      launch_transpose(G.Arp, G.Aci, G.Ava, (int)m, (int)n, brp, bci, bva,
                       at<int>(w, o_cursor), err, st);
      G.Brp = brp; G.Bci = bci; G.Bva = bva;
      HIPCHK(c, hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(c, hipStreamSynchronize(st));
      if (herr) return fail(c, SFK_EINVAL, "transposing A failed (code %d): a column of A has "
                            "more than 4096 entries", herr);
    }
    launch_partition(G.Arp, (int)m, nnzA, nw, at<int>(w, o_Apart), st);
    launch_partition(G.Brp, (int)n, nnzB, nw, at<int>(w, o_Bpart), st);
    HIPCHK(c, hipGetLastError());
    return SFK_OK;
  };
  if (s == SFK_OK) s = setup_group();
  // sliced products (vw automatic, 0 or 2) unless the row kernel is asked for
  // (any other vw) or an operator cannot be sliced; LDS-staged units where
  // they pay (vw automatic), never (0) or wherever they fit (2)
  if (s == SFK_OK && !p0.copies && (p0.vw == 0 || p0.vw == -2 || p0.vw == 2)) {
    bool oka = false, okb = false;
    const int lds = p0.vw == -2 ? 1 : p0.vw == 2 ? 2 : 0;
    s = build_xop(c, G.xa, G.Arp, G.Aci, G.Ava, (int)m, (int)n, nnzA, RS, cus, lds, &oka);
    if (s == SFK_OK && oka)
      s = build_xop(c, G.xb, G.Brp, G.Bci, G.Bva, (int)n, (int)m, nnzB, RS, cus, lds, &okb);
    G.sliced = (oka && okb) ? 1 : 0;
  }
  for (int r = 0; r < R && s == SFK_OK; ++r) {
    c->inst[r].p = p[r];
    s = setup_instance(c, c->inst[r], A, B, b_block + (size_t)r * m, nullptr, 0, cus, nw, &G, r);
    if (s != SFK_OK) prefix_err(c->err, "right-hand side", r);
  }
  if (s == SFK_OK) s = init_common(c);
  if (s != SFK_OK) {
    set_err(g_err, c->err);
    release(c);
    return s;
  }
  *out = c;
  return SFK_OK;
}

// --------------------------------------------------------------------------
// iterate / results
// --------------------------------------------------------------------------
extern "C" sfk_status sfk_iterate(sfk_ctx *c, int32_t k, int32_t *iters_done_host,
                                  int32_t *stopped_host) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  if (k < 0) return fail(c, SFK_EINVAL, "k must be >= 0");
  const int nb = (int)c->inst.size();
  auto all_halted = [&]() {
    for (auto &I : c->inst) if (!I.halted) return false;
    return true;
  };
  auto report = [&]() {
    if (nb == 1) {
      if (iters_done_host) *iters_done_host = c->inst[0].k_done;
      if (stopped_host) *stopped_host = c->inst[0].stopped;
    } else {
      if (iters_done_host) *iters_done_host = c->k_iter;
      if (stopped_host) *stopped_host = all_halted() ? 1 : 0;
    }
  };
  if (all_halted()) {
    report();
    if (nb == 1 && c->inst[0].breakdown)
      return fail(c, SFK_BREAKDOWN, "the basis broke down at iteration %d", c->inst[0].k_done);
    return fail(c, SFK_ESTATE, "the run has stopped (iteration %d)", c->k_iter);
  }
  const int room = c->maxitmax - c->k_iter;
  if (k > room) return fail(c, SFK_ESTATE, "capacity maxit = %d exhausted (done %d, asked %d)",
                            c->maxitmax, c->k_iter, k);
  // Iterations are enqueued in batches.  After each batch the side stream
  // (which runs the least-squares updates that set the stop flags) copies the
  // run state of every instance to pinned memory; the host runs at most two
  // batches ahead of the device and stops enqueueing once every instance has
  // halted, so a run that stops early does not pay for the rest of k.
  const int k0 = c->k_iter;
  // graphs are not used while the stages are timed (events between kernels)
  const bool graph = c->graph && !c->timing && !c->full;
  const int kBatch = graph ? 8 : 4;
  hipStream_t chk = (graph || c->full) ? c->stream : c->side;
  int enq = 0, nbatch = 0;
  bool all_done = false;
  while (enq < k && !all_done) {
    const int n = std::min(kBatch, k - enq);
    if (graph) HIPCHK(c, enqueue_graph_batch(c, k0 + enq + 1, n));
    else if (c->full) for (int i = 1; i <= n; ++i) enqueue_full_iteration(c, k0 + enq + i);
    else for (int i = 1; i <= n; ++i) enqueue_iteration(c, k0 + enq + i);
    enq += n;
    const int slot = nbatch % sfk_ctx::kChkSlots;
    int *dh = c->d_halt + (size_t)slot * nb;
    int *hh = c->h_halt + (size_t)slot * nb;
    if (nbatch >= sfk_ctx::kChkSlots) {
      // the slot's previous batch: wait for it (the device still has the batch
      // enqueued since then) and look at its flags
      HIPCHK(c, hipEventSynchronize(c->ev_chk[slot]));
      all_done = true;
      for (int i = 0; i < nb; ++i) all_done = all_done && hh[i] != 0;
    }
    if (!all_done && enq < k) {
      launch_collect_halt(c->L, k0 + enq, dh, chk);
      HIPCHK(c, hipMemcpyAsync(hh, dh, sizeof(int) * nb, hipMemcpyDeviceToHost, chk));
      HIPCHK(c, hipEventRecord(c->ev_chk[slot], chk));
    }
    ++nbatch;
  }
  if (!graph && !c->full) {
    flush_side(c);
    if (enq > 0 && k0 + enq >= c->ev_from)
      HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_ls[(k0 + enq) % sfk_ctx::kRing], 0));
  }
  HIPCHK(c, hipGetLastError());
  c->k_iter = k0 + enq;
  sfk_status s = read_scal(c);
  if (s != SFK_OK) return s;
  collect_stage_times(c);
  report();
  if (nb == 1 && c->inst[0].breakdown)
    return fail(c, SFK_BREAKDOWN, "the basis broke down after iteration %d", c->inst[0].k_done);
  return SFK_OK;
}

static sfk_status instance_of(sfk_ctx *c, int i, Inst **I) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  if (i < 0 || i >= (int)c->inst.size())
    return fail(c, SFK_EINVAL, "instance %d not in [0, %d)", i, (int)c->inst.size());
  *I = &c->inst[i];
  return SFK_OK;
}

static sfk_status solution_impl(sfk_ctx *c, Inst &I, int j, double *x) {
  if (!x) return fail(c, SFK_EINVAL, "x must not be NULL");
  if (j < 0 || j > I.k_done) return fail(c, SFK_ESTATE, "iterate %d not available (done %d)", j, I.k_done);
  if (j == 0) {
    HIPCHK(c, hipMemsetAsync(x, 0, sizeof(double) * I.D.n, c->stream));
  } else {
    if (c->full) launch_full_backsub(I.D, j, I.d_ytmp, c->stream);
    else launch_backsub(I.D, j, I.d_ytmp, c->stream);
    launch_solution(I.D, j, I.d_ytmp, x, c->stream);
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SFK_OK;
}

extern "C" sfk_status sfk_solution_at(sfk_ctx *c, int32_t j, double *x) {
  Inst *I;
  sfk_status s = instance_of(c, 0, &I);
  return s != SFK_OK ? s : solution_impl(c, *I, j, x);
}

extern "C" sfk_status sfk_solution(sfk_ctx *c, double *x) {
  Inst *I;
  sfk_status s = instance_of(c, 0, &I);
  return s != SFK_OK ? s : solution_impl(c, *I, I->k_done, x);
}

extern "C" sfk_status sfk_instance_solution(sfk_ctx *c, int32_t i, double *x) {
  Inst *I;
  sfk_status s = instance_of(c, i, &I);
  return s != SFK_OK ? s : solution_impl(c, *I, I->k_done, x);
}

extern "C" sfk_status sfk_instance_solution_at(sfk_ctx *c, int32_t i, int32_t j, double *x) {
  Inst *I;
  sfk_status s = instance_of(c, i, &I);
  return s != SFK_OK ? s : solution_impl(c, *I, j, x);
}

static sfk_status true_residual_impl(sfk_ctx *c, Inst &I, double *out_host);
static sfk_status explicit_residual_at(sfk_ctx *c, Inst &I, int j, double *out_host);

// Residual histories (sfk_res_kind) of one instance for j = 1..k_done.
static sfk_status norms_impl(sfk_ctx *c, Inst &I, int kind, double *out_host, int32_t cap,
                             int32_t *count_host, double *rhs_norm_host) {
  if (kind < SFK_RES_SKETCHED || kind > SFK_RES_TRUE_EXPLICIT)
    return fail(c, SFK_EINVAL, "unknown residual kind %d", kind);
  const int n = std::min(cap, I.k_done);
  if (n > 0 && !out_host) return fail(c, SFK_EINVAL, "out_host must not be NULL");
  const double beta = c->h_scal[&I - &c->inst[0]].beta;
  if (kind == SFK_RES_SKETCHED) {
    if (n > 0) HIPCHK(c, hipMemcpy(out_host, I.D.rho, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (rhs_norm_host) *rhs_norm_host = I.rhsnorm;
  } else if (kind == SFK_RES_TRUE_RECURRENCE) {
    // || beta e_1 - H_{j+1,j} y_j || from the stored H column band and y_j
    const int ldh = I.D.maxit + 1;
    std::vector<double> H((size_t)ldh * std::max(n, 1)), y(std::max(n, 1));
    if (n > 0)
      HIPCHK(c, hipMemcpy(H.data(), I.D.H, sizeof(double) * (size_t)ldh * n, hipMemcpyDeviceToHost));
    for (int j = 1; j <= n; ++j) {
      if (c->full) launch_full_backsub(I.D, j, I.d_ytmp, c->stream);
      else launch_backsub(I.D, j, I.d_ytmp, c->stream);
      HIPCHK(c, hipGetLastError());
      HIPCHK(c, hipMemcpyAsync(y.data(), I.d_ytmp, sizeof(double) * j, hipMemcpyDeviceToHost,
                               c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      double r2 = 0.0;
      for (int i = 0; i <= j; ++i) {      // row i of beta e_1 - H_{j+1,j} y
        double v = i == 0 ? beta : 0.0;
        for (int q = 0; q < j; ++q) v -= H[(size_t)q * ldh + i] * y[q];
        r2 += v * v;
      }
      out_host[j - 1] = std::sqrt(r2);
    }
    if (rhs_norm_host) *rhs_norm_host = beta;
  } else {
    if (I.p.resid) {
      if (n > 0) HIPCHK(c, hipMemcpy(out_host, I.D.rtrue, sizeof(double) * n, hipMemcpyDeviceToHost));
    } else {
      for (int j = 1; j <= n; ++j) {
        sfk_status s = explicit_residual_at(c, I, j, out_host + (j - 1));
        if (s != SFK_OK) return s;
      }
    }
    if (rhs_norm_host) *rhs_norm_host = beta;
  }
  if (count_host) *count_host = I.k_done;
  return SFK_OK;
}

extern "C" sfk_status sfk_residual_norms(sfk_ctx *c, int32_t kind, double *out_host, int32_t cap,
                                         int32_t *count_host, double *rhs_norm_host) {
  Inst *I;
  sfk_status s = instance_of(c, 0, &I);
  return s != SFK_OK ? s : norms_impl(c, *I, kind, out_host, cap, count_host, rhs_norm_host);
}

extern "C" sfk_status sfk_instance_residual_norms(sfk_ctx *c, int32_t i, int32_t kind,
                                                  double *out_host, int32_t cap,
                                                  int32_t *count_host, double *rhs_norm_host) {
  Inst *I;
  sfk_status s = instance_of(c, i, &I);
  return s != SFK_OK ? s : norms_impl(c, *I, kind, out_host, cap, count_host, rhs_norm_host);
}

extern "C" sfk_status sfk_memory(const sfk_ctx *c, size_t *workspace_host, size_t *library_host) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  size_t ws = c->gws_bytes, lib = c->hdr_bytes;
  for (const auto &I : c->inst) ws += I.ws_bytes;
  for (const auto &q : c->xmem) lib += q.second;
  if (c->d_halt) lib += sizeof(int) * sfk_ctx::kChkSlots * c->inst.size();
  if (workspace_host) *workspace_host = ws;
  if (library_host) *library_host = lib;
  return SFK_OK;
}

extern "C" sfk_status sfk_instance_status(sfk_ctx *c, int32_t i, int32_t *iters_done_host,
                                          int32_t *stopped_host, int32_t *breakdown_host) {
  Inst *I;
  sfk_status s = instance_of(c, i, &I);
  if (s != SFK_OK) return s;
  if (iters_done_host) *iters_done_host = I->k_done;
  if (stopped_host) *stopped_host = I->stopped;
  if (breakdown_host) *breakdown_host = I->breakdown;
  return SFK_OK;
}

extern "C" int32_t sfk_batch_size(const sfk_ctx *c) { return c ? (int32_t)c->inst.size() : 0; }

// ||b - A x_j|| of instance I (x_j assembled in the caller's order, multiplied
// by the caller's A)
static sfk_status explicit_residual_at(sfk_ctx *c, Inst &I, int j, double *out_host) {
  if (!out_host) return fail(c, SFK_EINVAL, "NULL argument");
  // D.x is scratch: the p-update of the reweighting writes x_k there but no
  // stage reads it back; for shared operators it is a right-hand side's own
  // contiguous n-vector
  double *xtmp = I.D.x;
  sfk_status s = solution_impl(c, I, j, xtmp);
  if (s != SFK_OK) return s;
  // x is in the caller's order: the residual uses the caller's A
  Dev D = I.D;
  if (I.user_aci) { D.Aci = I.user_aci; D.Ava = I.user_ava; }
  launch_true_residual(D, xtmp, I.d_scalar, c->stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(out_host, I.d_scalar, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SFK_OK;
}

static sfk_status true_residual_impl(sfk_ctx *c, Inst &I, double *out_host) {
  return explicit_residual_at(c, I, I.k_done, out_host);
}

extern "C" sfk_status sfk_true_residual(sfk_ctx *c, double *out_host) {
  Inst *I;
  sfk_status s = instance_of(c, 0, &I);
  return s != SFK_OK ? s : true_residual_impl(c, *I, out_host);
}

extern "C" sfk_status sfk_instance_true_residual(sfk_ctx *c, int32_t i, double *out_host) {
  Inst *I;
  sfk_status s = instance_of(c, i, &I);
  return s != SFK_OK ? s : true_residual_impl(c, *I, out_host);
}

extern "C" sfk_status sfk_set_timing(sfk_ctx *c, int32_t on) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  c->timing = on != 0;
  for (int i = 0; i < SFK_NUM_STAGES; ++i) { c->stage_ms[i] = 0.0; c->stage_count[i] = 0; }
  return SFK_OK;
}

extern "C" sfk_status sfk_stage_times(sfk_ctx *c, double *ms_host, int32_t *count_host) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  for (int i = 0; i < SFK_NUM_STAGES; ++i) {
    if (ms_host) ms_host[i] = c->stage_ms[i];
    if (count_host) count_host[i] = c->stage_count[i];
  }
  return SFK_OK;
}

extern "C" sfk_status sfk_destroy(sfk_ctx *c) {
  if (!c) return SFK_OK;
  release(c);
  return SFK_OK;
}

extern "C" const char *sfk_last_error(const sfk_ctx *c) {
  if (c) return c->err;
  return g_err;
}

extern "C" sfk_status sfk_sketch_sparse_sign(sfk_ctx *c, int32_t *rows_host, int8_t *neg_host) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  if (c->inst[0].p.sketch != SFK_SK_SPARSE_SIGN) return fail(c, SFK_ESTATE, "sketch is not sparse-sign");
  const size_t cnt = (size_t)c->inst[0].D.d_sk * c->inst[0].D.zeta;
  int *h = new int[cnt];
  hipError_t e = hipMemcpy(h, c->inst[0].D.sk_code, sizeof(int) * cnt, hipMemcpyDeviceToHost);
  if (e != hipSuccess) { delete[] h; return fail(c, SFK_EDEVICE, "copy failed: %s", hipGetErrorString(e)); }
  for (size_t i = 0; i < cnt; ++i) {
    if (rows_host) rows_host[i] = h[i] >> 1;
    if (neg_host) neg_host[i] = (int8_t)(h[i] & 1);
  }
  delete[] h;
  return SFK_OK;
}

extern "C" sfk_status sfk_sketch_srht(sfk_ctx *c, int32_t *rows_host, int8_t *neg_host,
                                      int64_t *N_host) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  if (c->inst[0].p.sketch != SFK_SK_SRHT) return fail(c, SFK_ESTATE, "sketch is not SRHT");
  const int N = c->inst[0].D.N;
  if (N_host) *N_host = N;
  if (rows_host) HIPCHK(c, hipMemcpy(rows_host, c->inst[0].D.srht_rows, sizeof(int) * c->inst[0].D.s, hipMemcpyDeviceToHost));
  if (neg_host) {
    const int nw = N / 64 + (N < 64 ? 1 : 0);
    unsigned long long *h = new unsigned long long[nw];
    hipError_t e = hipMemcpy(h, c->inst[0].D.srht_d, sizeof(unsigned long long) * nw, hipMemcpyDeviceToHost);
    if (e != hipSuccess) { delete[] h; return fail(c, SFK_EDEVICE, "copy failed: %s", hipGetErrorString(e)); }
    for (int i = 0; i < N; ++i) neg_host[i] = (int8_t)((h[i >> 6] >> (i & 63)) & 1ull);
    delete[] h;
  }
  return SFK_OK;
}

extern "C" sfk_status sfk_coefficients(sfk_ctx *c, double *H_host, double *T_host, int32_t k) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  if (k < 0 || k > c->inst[0].k_done) return fail(c, SFK_ESTATE, "k = %d not available", k);
  const int ld = c->inst[0].p.maxit + 1;
  for (int j = 0; j < k; ++j) {
    if (H_host) HIPCHK(c, hipMemcpy(H_host + (size_t)j * (k + 1), c->inst[0].D.H + (size_t)j * ld,
                                    sizeof(double) * (k + 1), hipMemcpyDeviceToHost));
    if (T_host) HIPCHK(c, hipMemcpy(T_host + (size_t)j * k, c->inst[0].D.T + (size_t)j * ld,
                                    sizeof(double) * k, hipMemcpyDeviceToHost));
  }
  return SFK_OK;
}

extern "C" sfk_status sfk_basis_vector(sfk_ctx *c, int32_t i, int32_t kind, int32_t j, double *out) {
  Inst *I;
  sfk_status s = instance_of(c, i, &I);
  if (s != SFK_OK) return s;
  if (!out) return fail(c, SFK_EINVAL, "out must not be NULL");
  if (kind < 0 || kind > 2) return fail(c, SFK_EINVAL, "unknown basis kind %d", kind);
  const Dev &D = I->D;
  const int k = I->k_done;
  if (I->halted) return fail(c, SFK_ESTATE, "basis vectors are available while the run is live");
  const int lo = c->full ? 1 : kind == 0 ? std::max(1, k + 1 - (D.ell + 1))
               : (kind == 1 && D.tau != SFK_TAU_IDENTITY) ? std::max(1, k + 1 - D.ell) : 1;
  // the scale of p_{k+1} (and z_{k+1}) is formed by the next iteration's first stage
  const int hi = (kind == 0 || c->full) ? k + 1 : k;
  if (j < lo || j > hi)
    return fail(c, SFK_ESTATE, "basis vector %d not kept (available %d..%d)", j, lo, hi);
  const double *src, *scale;
  int len;
  const int *pinv = nullptr;
  if (c->full) {
    src = (kind == 0 ? D.Wf : kind == 1 ? D.Pf : D.Z) + (size_t)(j - 1) * (kind == 0 ? D.m : D.n);
    scale = (kind == 0 ? D.sigw : D.sigp) + j;    // 1: the stored vectors are unit
    len = kind == 0 ? D.m : D.n;
  } else if (kind == 0) {
    src = D.W + (size_t)(j % (D.ell + 2)) * D.m * D.vs;
    scale = D.sigw + j;
    len = D.m;
  } else {
    src = (kind == 2 || D.tau == SFK_TAU_IDENTITY) ? D.Z + (size_t)(j - 1) * D.n * D.vs
                                                   : D.P + (size_t)(j % (D.ell + 1)) * D.n * D.vs;
    scale = D.sigp + j;
    len = D.n;
    pinv = D.pinv;
  }
  launch_export_vec(src, D.vs, len, scale, pinv, out, c->stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SFK_OK;
}

namespace sfk {
void run_adjoint(const Dev &D, int K, int tape, const double *ck, const double *xbar_in,
                 double *bbar, double *eacc_host, const AdjBufs &B, hipStream_t st);
}  // namespace sfk

extern "C" sfk_status sfk_adjoint(sfk_ctx *c, const double *xbar, double *bbar, double *epsbar_host) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  if (!xbar || !bbar) return fail(c, SFK_EINVAL, "xbar and bbar must not be NULL");
  if (!c->tape) return fail(c, SFK_ESTATE, "the context keeps no derivative tape (sfk_params.tape = 0)");
  Inst &I = c->inst[0];
  const Dev &D = I.D;
  const int K = I.k_done;
  if (K < 1 || I.stopped || I.breakdown || K != c->k_iter)
    return fail(c, SFK_ESTATE, "the derivative needs a run of K >= 1 steps that neither stopped "
                "nor broke down (done %d, launched %d)", K, c->k_iter);
  AdjBufs B;
  const size_t cnt = carve_adjoint(nullptr, D.m, D.n, D.s, K, D.maxit, c->tape, D.ell, B);
  void *mem = nullptr;
  if (hipMalloc(&mem, cnt * sizeof(double)) != hipSuccess)
    return fail(c, SFK_ENOMEM, "hipMalloc of %zu bytes for the adjoint failed", cnt * sizeof(double));
  const size_t used = carve_adjoint(static_cast<double *>(mem), D.m, D.n, D.s, K, D.maxit, c->tape,
                                    D.ell, B);
  if (used != cnt) {
    hipFree(mem);
    return fail(c, SFK_EDEVICE, "adjoint scratch layout mismatch");
  }
  std::vector<double> eacc(K);
  run_adjoint(D, K, c->tape, D.ck, xbar, bbar, eacc.data(), B, c->stream);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  hipFree(mem);
  if (e != hipSuccess) return fail(c, SFK_EDEVICE, "adjoint failed: %s", hipGetErrorString(e));
  double ebar = 0.0;
  for (int k = 0; k < K; ++k) ebar += eacc[k];
  if (epsbar_host) *epsbar_host = ebar;
  return SFK_OK;
}

extern "C" sfk_status sfk_apply(sfk_ctx *c, int32_t op, const double *x, double *y) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  if (!x || !y || (op != 0 && op != 1)) return fail(c, SFK_EINVAL, "op must be 0 (A) or 1 (B)");
  if (c->multi || c->inst.size() != 1 || c->inst[0].p.perm)
    return fail(c, SFK_EINVAL, "sfk_apply takes single-instance contexts without perm");
  const Dev &D = c->inst[0].D;
  launch_spmv_core(D, op == 0, op == 0 ? D.vwA : D.vwB, x, y, c->stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SFK_OK;
}

extern "C" sfk_status sfk_tau_apply(sfk_ctx *c, const double *x, double *y, int32_t call) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  if (c->inst.size() != 1 || !c->inst[0].lowrank)
    return fail(c, SFK_EINVAL, "sfk_tau_apply needs a single-instance context with a low-rank tau");
  if (!x || !y || x == y) return fail(c, SFK_EINVAL, "x and y must be distinct device vectors");
  if (call < 1) return fail(c, SFK_EINVAL, "call must be >= 1");
  Inst &I = c->inst[0];
  HIPCHK(c, lr_apply(I.lr, I.D.sc, I.D.maxit, 2, call - 1, x, y, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SFK_OK;
}

extern "C" sfk_status sfk_tau_stats(sfk_ctx *c, int32_t *out_host, double *resmax_host) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  if (c->inst.size() != 1 || !c->inst[0].lowrank)
    return fail(c, SFK_EINVAL, "sfk_tau_stats needs a single-instance context with a low-rank tau");
  const LrBufs &L = c->inst[0].lr;
  int st[4] = {0, 0, 0, 0};
  double rm = 0.0;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(st, L.stat, sizeof st, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(&rm, L.rb, sizeof rm, hipMemcpyDeviceToHost));
  if (out_host) { out_host[0] = st[2]; out_host[1] = st[1]; out_host[2] = st[3]; }
  if (resmax_host) *resmax_host = rm;
  return SFK_OK;
}

extern "C" sfk_status sfk_spmv_variant(const sfk_ctx *c, int32_t *vwA_host, int32_t *vwB_host) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  const Grp &G = c->grp;
  const int ga = !G.sliced ? -3 : G.xa.urec ? -4 : -2, gb = !G.sliced ? -3 : G.xb.urec ? -4 : -2;
  if (vwA_host) *vwA_host = c->multi ? ga : c->L.vwA;
  if (vwB_host) *vwB_host = c->multi ? gb : c->L.vwB;
  return SFK_OK;
}

extern "C" const char *sfk_version(void) {
  return "sfk 0.1 (gfx950, FP64, sFLSQR / sFLSMR)";
}

// --------------------------------------------------------------------------
// the allocation-free solve
// --------------------------------------------------------------------------
// Device memory of sfk_solve_noalloc: one array per device, held while the
// process runs.  Host code never uses its name as an address: the address on
// each device comes from hipGetSymbolAddress, taken once per device with that
// device current.
static __device__ __align__(256) unsigned char scratch[SFK_NOALLOC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mutex[kMaxDevices];   // one call at a time per device
void *g_noalloc_ptr[kMaxDevices];          // the array's address on each device
}  // namespace

extern "C" sfk_status sfk_solve_noalloc(const sfk_csr *A, const sfk_csr *B, const double *b,
                                        const sfk_params *p_in, int32_t k, double *x,
                                        double *rho_host, int32_t *iters_done_host,
                                        int32_t *stopped_host, void *stream) {
  if (!p_in || !x) return fail(nullptr, SFK_EINVAL, "params and x must not be NULL");
  if (k < 0) return fail(nullptr, SFK_EINVAL, "k must be >= 0");
  sfk_params p = *p_in;
  // no copies of the operators and no autotuning (the tuner's events are
  // allocations): CSR-stream unless a row kernel is asked for
  if (p.perm) return fail(nullptr, SFK_EINVAL, "sfk_solve_noalloc does not take perm");
  if (p.tape) return fail(nullptr, SFK_EINVAL, "sfk_solve_noalloc keeps no derivative tape");
  if (p.vw == 1 || (p.vw_split && p.vw_b == 1))
    return fail(nullptr, SFK_EINVAL, "sfk_solve_noalloc does not take the SELL-64 kernel (vw = 1)");
  p.copies = 1;
  if (p.vw == -2) p.vw = 0;
  if (p.vw_split && p.vw_b == -2) p.vw_b = 0;
  sfk_status s = validate(nullptr, A, B, &p);
  if (s != SFK_OK) return s;
  if (k > p.maxit) return fail(nullptr, SFK_EINVAL, "k = %d exceeds maxit = %d", k, p.maxit);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(nullptr, SFK_EDEVICE, "no usable HIP device");
  const int cus = device_cus();
  if (cus <= 0) return fail(nullptr, SFK_EDEVICE, "no HIP device available");
  const int nws = default_nws(A, B, &p, cus, spmv_blocks_per_cu());
  const Plan P = make_plan(A, B, &p, cus, nws);
  // descriptor and block maps after the instance's workspace
  const int nsg = p.sketch == SFK_SK_SPARSE_SIGN ? p.s
                : p.sketch == SFK_SK_IDENTITY ? (p.s + kWG - 1) / kWG : 0;
  const int nsb = p.sketch == SFK_SK_SRHT ? P.nblk : 0;
  const int nsc = p.sketch == SFK_SK_SRHT ? (p.s + kWG - 1) / kWG : 0;
  Layout L_;
  L_.off = P.total;
  const size_t o_dev = L_.take<Dev>(1);
  const size_t o_ms = L_.take<int2>(nws);
  const size_t o_mv = L_.take<int2>(nws);
  const size_t o_mg = L_.take<int2>(std::max(nsg, 1));
  const size_t o_mb = L_.take<int2>(std::max(nsb, 1));
  const size_t o_mc = L_.take<int2>(std::max(nsc, 1));
  if (L_.off > (size_t)SFK_NOALLOC_BYTES)
    return fail(nullptr, SFK_ENOMEM, "the problem needs %zu bytes of device scratch, more than "
                "the %zu of sfk_solve_noalloc (SFK_NOALLOC_BYTES); use sfk_init", L_.off,
                (size_t)SFK_NOALLOC_BYTES);

  std::lock_guard<std::mutex> lock(g_noalloc_mutex[dev]);
  if (!g_noalloc_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(nullptr, SFK_EDEVICE, "hipGetSymbolAddress of the scratch array failed: %s",
                  hipGetErrorString(e));
    g_noalloc_ptr[dev] = ptr;
  }
  void *base = g_noalloc_ptr[dev];

  // a context on the stack: one instance, the caller's stream only (the
  // sketch and the least-squares update run in order between the products)
  sfk_ctx c;
  c.stream = static_cast<hipStream_t>(stream);
  hipStream_t st = c.stream;
  Inst I;
  I.p = p;
  s = setup_instance(&c, I, A, B, b, base, P.total, cus, nws);
  if (s != SFK_OK) {
    set_err(g_err, c.err);
    hipStreamSynchronize(st);
    return s;
  }
  Dev &D = I.D;
  char *hb = static_cast<char *>(base);
  Launch &L = c.L;
  L.devs = reinterpret_cast<const Dev *>(hb + o_dev);
  L.map_spmv = reinterpret_cast<const int2 *>(hb + o_ms);
  L.map_vec = reinterpret_cast<const int2 *>(hb + o_mv);
  L.map_sg = reinterpret_cast<const int2 *>(hb + o_mg);
  L.map_sb = reinterpret_cast<const int2 *>(hb + o_mb);
  L.map_sc = reinterpret_cast<const int2 *>(hb + o_mc);
  L.nspmv = D.nws;
  L.nvec = D.nwv;
  L.nsg = D.nsg;
  L.nsb = nsb;
  L.nsc = nsc;
  L.ninst = 1;
  L.smax = D.s;
  L.maxitmax = D.maxit;
  L.tau = D.tau;
  L.ellmax = D.ell;
  L.vwA = D.vwA;
  L.vwB = D.vwB;
  HIPCHK(nullptr, hipMemcpyAsync(hb + o_dev, &D, sizeof(Dev), hipMemcpyHostToDevice, st));
  launch_iota_map(reinterpret_cast<int2 *>(hb + o_ms), D.nws, st);
  launch_iota_map(reinterpret_cast<int2 *>(hb + o_mv), D.nwv, st);
  launch_iota_map(reinterpret_cast<int2 *>(hb + o_mg), D.nsg, st);
  launch_iota_map(reinterpret_cast<int2 *>(hb + o_mb), nsb, st);
  launch_iota_map(reinterpret_cast<int2 *>(hb + o_mc), nsc, st);
  // Algorithm 1 / 2 initial lines, then k iterations in stage order
  launch_stage_C(L, 0, st);
  launch_sketch(L, 0, st);
  launch_init_rhs(D, st);
  launch_stage_D(L, 0, st);
  for (int it = 1; it <= k; ++it) {
    launch_stage_A(L, it, st);
    launch_stage_B(L, it, st);
    if (D.method == SFK_SFLSQR) launch_sketch(L, it, st);
    launch_stage_C(L, it, st);
    if (D.method == SFK_SFLSMR) launch_sketch(L, it, st);
    launch_ls(L, it, st);
    if (D.resid) launch_true_iter(D, it, st);
    launch_stage_D(L, it, st);
  }
  HIPCHK(nullptr, hipGetLastError());
  Scal S;
  HIPCHK(nullptr, hipMemcpyAsync(&S, D.sc, sizeof(Scal), hipMemcpyDeviceToHost, st));
  HIPCHK(nullptr, hipStreamSynchronize(st));
  if (S.err & 16)
    return fail(nullptr, SFK_EINVAL, "right-hand side b is zero or not finite (||b|| = %g)", S.beta);
  const int done = S.k_done;
  if (done == 0) {
    launch_zero_bytes(x, sizeof(double) * (size_t)D.n, st);
  } else {
    launch_backsub(D, done, I.d_ytmp, st);
    launch_solution(D, done, I.d_ytmp, x, st);
  }
  HIPCHK(nullptr, hipGetLastError());
  if (rho_host && done > 0)
    HIPCHK(nullptr, hipMemcpyAsync(rho_host, D.rho, sizeof(double) * done, hipMemcpyDeviceToHost, st));
  HIPCHK(nullptr, hipStreamSynchronize(st));
  if (iters_done_host) *iters_done_host = done;
  if (stopped_host) *stopped_host = S.stopped;
  if (S.breakdown) return fail(nullptr, SFK_BREAKDOWN, "the basis broke down after iteration %d", done);
  return SFK_OK;
}
