// Host side of the C ABI declared in include/sfk.h: validation, workspace
// layout, initialisation and the per-iteration stage sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "sfk.h"
#include "sfk_dev.h"

namespace sfk {
void launch_stage_A(const Dev &D, int k, hipStream_t st);
void launch_stage_B(const Dev &D, int k, hipStream_t st);
void launch_stage_C(const Dev &D, int k, hipStream_t st);
void launch_ls(const Dev &D, int k, hipStream_t st);
int spmv_blocks_per_cu();
void launch_stage_D(const Dev &D, int k, hipStream_t st);
void launch_sketch(const Dev &D, int k, const double *v, double *dst, hipStream_t st);
const double *sketch_src(const Dev &D, int k);
double *sketch_dst(const Dev &D, int k);
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
void launch_backsub(const Dev &D, int j, double *yout, hipStream_t st);
void launch_solution(const Dev &D, int kk, const double *yv, double *x, hipStream_t st);
void launch_true_residual(const Dev &D, const double *x, double *out, hipStream_t st);
}  // namespace sfk

using namespace sfk;

struct sfk_ctx {
  sfk_params p;
  Dev D;
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;       // sketch + least-squares stream (default priority)
  static constexpr int kRing = 4;   // iterations of synchronisation events kept
  hipEvent_t ev_main[kRing] = {}, ev_sk[kRing] = {}, ev_ls[kRing] = {};
  void *ws = nullptr;
  size_t ws_bytes = 0;
  bool owns_ws = false;
  int k_done = 0;
  int stopped = 0;
  int breakdown = 0;
  int halted = 0;
  int *d_err = nullptr;
  double *d_scalar = nullptr;     // one double of scratch (true residual)
  double *d_ytmp = nullptr;       // maxit
  Scal *h_scal = nullptr;         // pinned copy of the device scalars
  std::string err;
  // optional per-stage timing with HIP events on the context's stream
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_used;   // (stage, index of the start event)
  double stage_ms[SFK_NUM_STAGES] = {};
  int stage_count[SFK_NUM_STAGES] = {};
};

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

// One iteration k of Algorithm 1 (sFLSQR) or Algorithm 2 (sFLSMR).  The
// data-parallel stages A, B, C, D run on the context's stream; the sketch of
// the new vector and the least-squares update run on the side stream as soon
// as their input exists.  The raw vectors are double-buffered by iteration
// parity, so iteration k + 2 waits for the sketch of iteration k only.  The
// reweighting needs y_k before D(k), so it waits for LS(k).
static void enqueue_iteration(sfk_ctx *c, int k) {
  const Dev &D = c->D;
  hipStream_t st = c->stream, sd = c->side;
  const int r = k % sfk_ctx::kRing;
  if (k >= 3) hipStreamWaitEvent(st, c->ev_sk[(k - 2) % sfk_ctx::kRing], 0);
  int t = stage_begin(c, SFK_STAGE_SPMV_A, st);
  launch_stage_A(D, k, st);
  stage_end(c, t, st);
  t = stage_begin(c, SFK_STAGE_W_UPDATE, st);
  launch_stage_B(D, k, st);
  stage_end(c, t, st);
  if (D.method == 0) hipEventRecord(c->ev_main[r], st);
  t = stage_begin(c, SFK_STAGE_SPMV_B, st);
  launch_stage_C(D, k, st);
  stage_end(c, t, st);
  if (D.method == 1) hipEventRecord(c->ev_main[r], st);

  hipStreamWaitEvent(sd, c->ev_main[r], 0);
  t = stage_begin(c, SFK_STAGE_SKETCH, sd);
  launch_sketch(D, k, sketch_src(D, k), sketch_dst(D, k), sd);
  stage_end(c, t, sd);
  hipEventRecord(c->ev_sk[r], sd);
  t = stage_begin(c, SFK_STAGE_LS, sd);
  launch_ls(D, k, sd);
  stage_end(c, t, sd);
  hipEventRecord(c->ev_ls[r], sd);

  if (D.tau == 1) hipStreamWaitEvent(st, c->ev_ls[r], 0);
  t = stage_begin(c, SFK_STAGE_P_UPDATE, st);
  launch_stage_D(D, k, st);
  stage_end(c, t, st);
}

static thread_local std::string g_err;

static sfk_status fail(sfk_ctx *c, sfk_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf; else g_err = buf;
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
}

static int64_t next_pow2(int64_t d) {
  int64_t N = 1;
  while (N < d) N <<= 1;
  return N;
}

static sfk_status validate(sfk_ctx *c, const sfk_csr *A, const sfk_csr *B, const sfk_params *p) {
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
  if (p->method != SFK_SFLSQR && p->method != SFK_SFLSMR)
    return fail(c, SFK_EINVAL, "unknown method %d", p->method);
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
  if (p->tau != SFK_TAU_IDENTITY && p->tau != SFK_TAU_REWEIGHT_L1)
    return fail(c, SFK_EINVAL, "unknown tau %d", p->tau);
  if (p->tau == SFK_TAU_REWEIGHT_L1 && !(p->eps > 0.0 && std::isfinite(p->eps)))
    return fail(c, SFK_EINVAL, "reweighting needs finite eps > 0");
  if (!(p->eta >= 0.0) || !std::isfinite(p->eta)) return fail(c, SFK_EINVAL, "eta must be finite >= 0");
  if (!(p->noise_norm >= 0.0) || !std::isfinite(p->noise_norm))
    return fail(c, SFK_EINVAL, "noise_norm must be finite >= 0");
  if (!(p->tol >= 0.0) || !std::isfinite(p->tol)) return fail(c, SFK_EINVAL, "tol must be finite >= 0");
  if (p->driver < 0 || p->driver > 2) return fail(c, SFK_EINVAL, "unknown driver %d", p->driver);
  if (p->vw != 0 && p->vw != -1 && p->vw != 8 && p->vw != 16 && p->vw != 32 && p->vw != 64)
    return fail(c, SFK_EINVAL, "vw must be -1, 0, 8, 16, 32 or 64");
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
  int nw, vwA, vwB, d, N, log2L, nblk, nchunk;
  bool transpose;
  // offsets
  size_t o_sc, o_err, o_scalar, o_part, o_sigw, o_sigp, o_H, o_T, o_rho;
  size_t o_W, o_P, o_Z, o_wraw, o_zraw, o_x, o_Apart, o_Bpart;
  size_t o_skcode, o_skent, o_skrp, o_chunk, o_srows, o_sd, o_spart, o_SK, o_skrhs;
  size_t o_V, o_tauv, o_R, o_c, o_y, o_ytmp;
  size_t o_brp, o_bci, o_bva, o_cursor;
  size_t total;
};

static int pick_vw(int64_t nnz, int64_t rows, int user) {
  if (user > 0) return user;
  if (user == 0) return 0;     // CSR-stream
  // user < 0: row-parallel with a width from the mean row length
  const double avg = rows > 0 ? (double)nnz / (double)rows : 0.0;
  if (avg >= 96) return 64;
  if (avg >= 40) return 32;
  if (avg >= 16) return 16;
  return 8;
}

static Plan make_plan(const sfk_csr *A, const sfk_csr *B, const sfk_params *p, int cus,
                      int blocks_per_cu) {
  Plan P{};
  P.m = A->rows;
  P.n = A->cols;
  P.nnzA = A->nnz;
  P.transpose = (B == nullptr);
  P.nnzB = B ? B->nnz : A->nnz;
  const int64_t nnzmax = std::max(P.nnzA, P.nnzB);
  const int cap = cus * (p->wg_per_cu ? p->wg_per_cu : std::max(1, blocks_per_cu));
  int64_t nw = (nnzmax + 8191) / 8192;
  nw = std::max<int64_t>(nw, (std::max(P.m, P.n) + 2047) / 2048);
  nw = std::min<int64_t>(std::max<int64_t>(nw, 1), cap);
  P.nw = (int)nw;
  P.vwA = pick_vw(P.nnzA, P.m, p->vw);
  P.vwB = pick_vw(P.nnzB, P.n, p->vw);
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
  P.o_part = L_.take<double>((size_t)kNumPart * kMaxQ * nw_alloc);
  P.o_sigw = L_.take<double>(mi + 2);
  P.o_sigp = L_.take<double>(mi + 2);
  P.o_H = L_.take<double>((mi + 1) * mi);
  P.o_T = L_.take<double>((mi + 1) * (mi + 1));
  P.o_rho = L_.take<double>(mi);
  P.o_W = L_.take<double>((ell + 2) * m);
  P.o_P = L_.take<double>(p->tau == SFK_TAU_REWEIGHT_L1 ? (ell + 1) * n : 1);
  P.o_Z = L_.take<double>((mi + 1) * n);      // z~_1 .. z~_{maxit+1}
  P.o_wraw = L_.take<double>(2 * m);
  P.o_zraw = L_.take<double>(2 * std::max<int64_t>(n, (P.N + 1) / 2 + 1));
  P.o_x = L_.take<double>(n);
  P.o_Apart = L_.take<int>(nw_alloc + 1);
  P.o_Bpart = L_.take<int>(nw_alloc + 1);
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
  if (P.transpose) {
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

extern "C" size_t sfk_workspace_bytes(const sfk_csr *A, const sfk_csr *B, const sfk_params *p) {
  if (validate(nullptr, A, B, p) != SFK_OK) return 0;
  int cus = device_cus();
  if (cus <= 0) cus = 256;
  return make_plan(A, B, p, cus, 2).total;
}

// --------------------------------------------------------------------------
// init
// --------------------------------------------------------------------------
template <class T>
static T *at(void *base, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

static sfk_status read_scal(sfk_ctx *c) {
  HIPCHK(c, hipMemcpyAsync(c->h_scal, c->D.sc, sizeof(Scal), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->k_done = c->h_scal->k_done;
  c->stopped = c->h_scal->stopped;
  c->breakdown = c->h_scal->breakdown;
  c->halted = c->h_scal->halt;
  return SFK_OK;
}

static sfk_status init_impl(sfk_ctx *c, const sfk_csr *A, const sfk_csr *B, const double *b,
                            void *workspace, size_t ws_bytes) {
  const sfk_params &p = c->p;
  const int cus = device_cus();
  if (cus <= 0) return fail(c, SFK_EDEVICE, "no HIP device available");
  if ((A->nnz > 0 && (!A->rowptr || !A->colind || !A->val)) || !A->rowptr || !b)
    return fail(c, SFK_EINVAL, "A arrays and b must be device pointers");
  if (B && ((B->nnz > 0 && (!B->colind || !B->val)) || !B->rowptr))
    return fail(c, SFK_EINVAL, "B arrays must be device pointers");
  const Plan P = make_plan(A, B, &p, cus, spmv_blocks_per_cu());
  if (workspace) {
    if (ws_bytes < P.total)
      return fail(c, SFK_ENOMEM, "workspace of %zu bytes is smaller than the %zu required",
                  ws_bytes, P.total);
    c->ws = workspace;
    c->owns_ws = false;
  } else {
    hipError_t e = hipMalloc(&c->ws, P.total);
    if (e != hipSuccess) {
      c->ws = nullptr;
      return fail(c, SFK_ENOMEM, "hipMalloc of %zu bytes failed: %s", P.total, hipGetErrorString(e));
    }
    c->owns_ws = true;
  }
  c->ws_bytes = P.total;
  HIPCHK(c, hipHostMalloc((void **)&c->h_scal, sizeof(Scal), hipHostMallocDefault));
  HIPCHK(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  for (int i = 0; i < sfk_ctx::kRing; ++i) {
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_main[i], hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_sk[i], hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_ls[i], hipEventDisableTiming));
  }
  void *w = c->ws;
  hipStream_t st = c->stream;
  HIPCHK(c, hipMemsetAsync(w, 0, P.total, st));

  Dev &D = c->D;
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
  D.N = P.N;
  D.log2L = P.log2L;
  D.nblk = P.nblk;
  D.nw = P.nw;
  D.vwA = P.vwA;
  D.vwB = P.vwB;
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
  D.zraw = at<double>(w, P.o_zraw);   // slot 1 starts at zraw + n
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
  c->d_err = at<int>(w, P.o_err);
  c->d_scalar = at<double>(w, P.o_scalar);
  c->d_ytmp = at<double>(w, P.o_ytmp);

  // structure checks
  launch_csr_check(A->rowptr, A->colind, D.m, D.n, A->nnz, c->d_err, st);
  if (B) {
    launch_csr_check(B->rowptr, B->colind, D.n, D.m, B->nnz, c->d_err, st);
    D.Brp = B->rowptr; D.Bci = B->colind; D.Bva = B->val;
  }
  int herr = 0;
  HIPCHK(c, hipMemcpyAsync(&herr, c->d_err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  if (herr) return fail(c, SFK_EINVAL, "invalid CSR structure (code %d): row pointers must rise "
                        "from 0 to nnz and column indices lie in range", herr);
  if (!B) {
    int *brp = at<int>(w, P.o_brp);
    int *bci = at<int>(w, P.o_bci);
    double *bva = at<double>(w, P.o_bva);
    launch_transpose(A->rowptr, A->colind, A->val, D.m, D.n, brp, bci, bva, at<int>(w, P.o_cursor),
                     c->d_err, st);
    D.Brp = brp; D.Bci = bci; D.Bva = bva;
  }
  launch_partition(D.Arp, D.m, P.nnzA, D.nw, at<int>(w, P.o_Apart), st);
  launch_partition(D.Brp, D.n, P.nnzB, D.nw, at<int>(w, P.o_Bpart), st);

  // sketch
  const uint64_t key0 = p.seed;
  const uint64_t key1 = 0ull + ((uint64_t)(uint32_t)p.instance << 32);
  const uint64_t key1_rows = 1ull + ((uint64_t)(uint32_t)p.instance << 32);
  int *scratch = p.sketch == SFK_SK_SPARSE_SIGN ? at<int>(w, P.o_chunk) : reinterpret_cast<int *>(D.zraw);
  launch_sketch_build(D, key0, key1, key1_rows, scratch, c->d_err, st);
  HIPCHK(c, hipMemcpyAsync(&herr, c->d_err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  if (herr) return fail(c, SFK_EINVAL, "initialisation failed (code %d): transposed rows longer "
                        "than 4096 entries or sketch generation exhausted", herr);
  HIPCHK(c, hipGetLastError());

  // Algorithm 1 / 2 initial lines
  const int use_disc = (p.method == SFK_SFLSQR && p.noise_norm > 0.0) ? 1 : 0;
  launch_init_b(D, p.eta, p.noise_norm, p.tol, use_disc, st);
  if (p.method == SFK_SFLSQR) launch_sketch(D, 0, b, D.skrhs, st);
  launch_stage_C(D, 0, st);
  if (p.method == SFK_SFLSMR) launch_sketch(D, 0, D.zraw, D.SK, st);
  launch_init_rhs(D, st);
  launch_stage_D(D, 0, st);
  HIPCHK(c, hipGetLastError());
  sfk_status s = read_scal(c);
  if (s != SFK_OK) return s;
  if (c->h_scal->err & 16)
    return fail(c, SFK_EINVAL, "right-hand side b is zero or not finite (||b|| = %g)", c->h_scal->beta);
  if (c->h_scal->breakdown)
    return fail(c, SFK_BREAKDOWN, "B b is zero: the first basis vector does not exist");
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
  if (c->side) hipStreamDestroy(c->side);
  if (c->owns_ws && c->ws) hipFree(c->ws);
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
  sfk_ctx *c = new sfk_ctx();
  c->p = *p;
  c->stream = static_cast<hipStream_t>(stream);
  s = init_impl(c, A, B, b, workspace, workspace_bytes);
  if (s != SFK_OK) {
    g_err = c->err;
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
  auto report = [&]() {
    if (iters_done_host) *iters_done_host = c->k_done;
    if (stopped_host) *stopped_host = c->stopped;
  };
  if (c->halted) {
    report();
    if (c->breakdown) return fail(c, SFK_BREAKDOWN, "the basis broke down at iteration %d", c->k_done);
    return fail(c, SFK_ESTATE, "the run has stopped at iteration %d", c->k_done);
  }
  const int room = c->p.maxit - c->k_done;
  if (k > room) return fail(c, SFK_ESTATE, "capacity maxit = %d exhausted (done %d, asked %d)",
                            c->p.maxit, c->k_done, k);
  const int k0 = c->k_done;
  for (int i = 1; i <= k; ++i) enqueue_iteration(c, k0 + i);
  if (k > 0) HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_ls[(k0 + k) % sfk_ctx::kRing], 0));
  HIPCHK(c, hipGetLastError());
  sfk_status s = read_scal(c);
  if (s != SFK_OK) return s;
  collect_stage_times(c);
  report();
  if (c->breakdown) return fail(c, SFK_BREAKDOWN, "the basis broke down after iteration %d", c->k_done);
  return SFK_OK;
}

extern "C" sfk_status sfk_solution_at(sfk_ctx *c, int32_t j, double *x) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  if (!x) return fail(c, SFK_EINVAL, "x must not be NULL");
  if (j < 0 || j > c->k_done) return fail(c, SFK_ESTATE, "iterate %d not available (done %d)", j, c->k_done);
  if (j == 0) {
    HIPCHK(c, hipMemsetAsync(x, 0, sizeof(double) * c->D.n, c->stream));
  } else {
    launch_backsub(c->D, j, c->d_ytmp, c->stream);
    launch_solution(c->D, j, c->d_ytmp, x, c->stream);
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SFK_OK;
}

extern "C" sfk_status sfk_solution(sfk_ctx *c, double *x) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  if (!x) return fail(c, SFK_EINVAL, "x must not be NULL");
  if (c->k_done == 0) {
    HIPCHK(c, hipMemsetAsync(x, 0, sizeof(double) * c->D.n, c->stream));
  } else {
    launch_backsub(c->D, c->k_done, c->d_ytmp, c->stream);
    launch_solution(c->D, c->k_done, c->d_ytmp, x, c->stream);
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SFK_OK;
}

extern "C" sfk_status sfk_residual_norms(sfk_ctx *c, double *out_host, int32_t cap,
                                         int32_t *count_host, double *rhs_norm_host) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  const int n = std::min(cap, c->k_done);
  if (n > 0) {
    if (!out_host) return fail(c, SFK_EINVAL, "out_host must not be NULL");
    HIPCHK(c, hipMemcpy(out_host, c->D.rho, sizeof(double) * n, hipMemcpyDeviceToHost));
  }
  if (count_host) *count_host = c->k_done;
  if (rhs_norm_host) *rhs_norm_host = c->h_scal->rhsnorm;
  return SFK_OK;
}

extern "C" sfk_status sfk_true_residual(sfk_ctx *c, double *out_host) {
  if (!c || !out_host) return fail(c, SFK_EINVAL, "NULL argument");
  // D.x is scratch for tau = I and holds x_k itself for the reweighting
  double *xtmp = c->D.x;
  sfk_status s = sfk_solution(c, xtmp);
  if (s != SFK_OK) return s;
  launch_true_residual(c->D, xtmp, c->d_scalar, c->stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(out_host, c->d_scalar, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SFK_OK;
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
  if (c) return c->err.c_str();
  return g_err.c_str();
}

extern "C" sfk_status sfk_sketch_sparse_sign(sfk_ctx *c, int32_t *rows_host, int8_t *neg_host) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  if (c->p.sketch != SFK_SK_SPARSE_SIGN) return fail(c, SFK_ESTATE, "sketch is not sparse-sign");
  const size_t cnt = (size_t)c->D.d_sk * c->D.zeta;
  int *h = new int[cnt];
  hipError_t e = hipMemcpy(h, c->D.sk_code, sizeof(int) * cnt, hipMemcpyDeviceToHost);
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
  if (c->p.sketch != SFK_SK_SRHT) return fail(c, SFK_ESTATE, "sketch is not SRHT");
  const int N = c->D.N;
  if (N_host) *N_host = N;
  if (rows_host) HIPCHK(c, hipMemcpy(rows_host, c->D.srht_rows, sizeof(int) * c->D.s, hipMemcpyDeviceToHost));
  if (neg_host) {
    const int nw = N / 64 + (N < 64 ? 1 : 0);
    unsigned long long *h = new unsigned long long[nw];
    hipError_t e = hipMemcpy(h, c->D.srht_d, sizeof(unsigned long long) * nw, hipMemcpyDeviceToHost);
    if (e != hipSuccess) { delete[] h; return fail(c, SFK_EDEVICE, "copy failed: %s", hipGetErrorString(e)); }
    for (int i = 0; i < N; ++i) neg_host[i] = (int8_t)((h[i >> 6] >> (i & 63)) & 1ull);
    delete[] h;
  }
  return SFK_OK;
}

extern "C" sfk_status sfk_coefficients(sfk_ctx *c, double *H_host, double *T_host, int32_t k) {
  if (!c) return fail(nullptr, SFK_EINVAL, "NULL context");
  if (k < 0 || k > c->k_done) return fail(c, SFK_ESTATE, "k = %d not available", k);
  const int ld = c->p.maxit + 1;
  for (int j = 0; j < k; ++j) {
    if (H_host) HIPCHK(c, hipMemcpy(H_host + (size_t)j * (k + 1), c->D.H + (size_t)j * ld,
                                    sizeof(double) * (k + 1), hipMemcpyDeviceToHost));
    if (T_host) HIPCHK(c, hipMemcpy(T_host + (size_t)j * k, c->D.T + (size_t)j * ld,
                                    sizeof(double) * k, hipMemcpyDeviceToHost));
  }
  return SFK_OK;
}

extern "C" const char *sfk_version(void) {
  return "sfk 0.1 (gfx950, FP64, sFLSQR / sFLSMR)";
}
