/*
 * sfk.h -- C ABI of the sketched flexible LSQR / LSMR library (gfx950, FP64).
 *
 * Method (Bucci, Gazzola, Robol, "Randomized flexible LSQR and LSMR with
 * applications to inverse problems"):
 *   solve min ||A x - b||_2 (eq. (LS)) for b = A x_true + e (eq. (inverseproblem))
 *   with the partially orthogonalised flexible Golub-Kahan process (eq. (FGK)):
 *     A^T W_k = P_k T_k (here B W_k = P_k T_k, B = A^T or an unmatched
 *     back-projector), A Z_k = W_{k+1} H_{k+1,k}, Z_k = tau(P_k),
 *   and a sketched projected least-squares problem per step:
 *     sFLSQR (eq. (sFLSQR), Algorithm 1): y_k = argmin || S (A Z_k y - b) ||
 *     sFLSMR (eq. (sFLSMR), Algorithm 2): y_k = argmin || S (B A Z_k y - B b) ||
 *   with x_k = Z_k y_k and discrepancy-principle stopping (eq. (discrP)).
 *
 * Conventions
 *   - Every pointer argument is a DEVICE pointer unless its name ends in _host.
 *   - Matrices, vectors and workspaces passed in are BORROWED: they stay owned
 *     by the caller and must outlive the context.  The library never frees them.
 *   - All device work of a context is enqueued on the stream given to
 *     sfk_init (a hipStream_t passed as void*; NULL is the default stream).
 *   - Functions return sfk_status; on failure sfk_last_error(ctx) (or
 *     sfk_last_error(NULL) for failures before a context exists) describes it.
 *     Failures never leave work running on the device.
 *   - A context is not thread-safe: one thread at a time per context.
 *   - Index base is 0; CSR row pointers and column indices are int32, values
 *     float64; column indices of a row need not be sorted; rows may be empty.
 */
#ifndef SFK_H
#define SFK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfk_ctx sfk_ctx;

typedef enum {
  SFK_OK = 0,
  SFK_EINVAL = 1,     /* invalid argument: dims, params, CSR structure, b zero or non-finite */
  SFK_ENOMEM = 2,     /* device allocation failed, or caller workspace too small */
  SFK_EDEVICE = 3,    /* HIP runtime error or no suitable device */
  SFK_BREAKDOWN = 4,  /* basis cannot grow (t_kk or h_{k+1,k} zero); results stay valid */
  SFK_ESTATE = 5      /* call not allowed in the context's state (e.g. k out of range) */
} sfk_status;

/* Methods.  SFLSQR / SFLSMR: the sketched methods (Algorithms 1 and 2; window
 * ell, sketch S).  FLSQR / FLSMR: the flexible methods with full
 * orthogonalisation they are compared with (Sec. 2.2, eq. (flsqr-relations)):
 * every new w and z orthogonalised against the whole basis (two passes of
 * classical Gram-Schmidt), y_k = argmin ||beta e_1 - H_{k+1,k} y|| (FLSQR,
 * eq. (FLSQR)) or argmin ||T_{k+1}(beta e_1 - H_{k+1,k} y)|| (FLSMR); sketch,
 * s, zeta and ell are ignored, maxit <= 1024, single-instance contexts only.
 * For FLSQR the projected residual is ||b - A x_k||, so noise_norm > 0 stops
 * by the discrepancy principle directly. */
typedef enum { SFK_SFLSQR = 0, SFK_SFLSMR = 1, SFK_FLSQR = 2, SFK_FLSMR = 3 } sfk_method;

/* Sketch families (paper Sec. 2.7 names them; the concrete definitions and the
 * seeding are the library's, identical to the test oracle's):
 *   SPARSE_SIGN: zeta distinct rows per column with values +-1/sqrt(zeta); zeta = 1
 *                is CountSketch, the family of the paper's imaging experiments;
 *   SRHT:        sqrt(N/s) R H_N D pad(v), N = 2^ceil(log2 d), Sylvester-ordered H_N;
 *   IDENTITY:    S = I (requires s = d), which turns sFLSQR into FLSQR-type solves.
 * Randomness: Philox4x64-10 keyed (seed, stream + (instance << 32)). */
typedef enum { SFK_SK_SPARSE_SIGN = 0, SFK_SK_SRHT = 1, SFK_SK_IDENTITY = 2 } sfk_sketch_kind;

/* Flexible operator tau (paper eq. (modbasis); the l1 reweighting follows the
 * IRLS interpretation of Sec. 1.2): IDENTITY, or
 * REWEIGHT_L1: z_k = (x_{k-1}^2 + eps^2)^(1/4) * p_k elementwise, x_0 = 0;
 * LOWRANK: z_k = tau_r(p_k), the rank-r truncated SVD of p_k viewed as an
 *   lr_rows x (n / lr_rows) image in row-major order (eq. (def:lowr-trc), the
 *   operator of the deblurring experiments of Sec. 3.1).  Computed by
 *   randomized subspace iteration with l = r + p vectors (re-based by a
 *   shifted Cholesky QR after every product, orthonormalised by two more
 *   passes before each Rayleigh-Ritz step) and a Rayleigh-Ritz step,
 *   iterated until the Ritz residuals ||C v_i - theta_i x_i||, i < r, are at
 *   most lr_tol * theta_1 (theta_i the squared singular values): the full
 *   SVD's truncation to within that residual over the gap at r;
 * LOWRANK_RND: the randomized SVD (Halko, Martinsson, Tropp, Algorithms 4.4
 *   and 5.1) truncated to rank r, the paper's "-RND" solvers: lr_q power
 *   iterations, then the SVD of B = Q^T C.  The Gaussian test matrix of basis
 *   vector k (nc x l, column-major, entry e = j nc + i) is normal e mod 4 of
 *   the Philox4x64-10 block (k, e >> 2, 0, 0) keyed (seed, 2 + (instance << 32)),
 *   by Box-Muller: u1 = ((w_even >> 11) + 1/2) 2^-53, u2 = (w_odd >> 11) 2^-53,
 *   sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2) from words (w0, w1) and (w2, w3).
 * Both low-rank operators: single-instance contexts, no perm, driver MULTI
 * (LOWRANK reads its convergence flag on the host every 4 power iterations). */
typedef enum { SFK_TAU_IDENTITY = 0, SFK_TAU_REWEIGHT_L1 = 1, SFK_TAU_LOWRANK = 2,
               SFK_TAU_LOWRANK_RND = 3 } sfk_tau;

/* Iteration driver.  MULTI: every stage kernel of every iteration is launched
 * on the context's stream (and a second stream for the sketch and the small
 * least-squares update).  GRAPH: the same launches, captured once per batch of
 * iterations into a HIP graph that is launched as one unit (the host submits one
 * graph per batch instead of every kernel).  AUTO = MULTI.  Both give identical
 * results. */
typedef enum { SFK_DRIVER_AUTO = 0, SFK_DRIVER_MULTI = 1, SFK_DRIVER_GRAPH = 2 } sfk_driver;

/* Residual histories (sfk_residual_norms):
 *   SKETCHED:        rho_j, the minimised sketched objective of the small
 *                    least-squares problem (eq. (sFLSQR) / (sFLSMR)), which the
 *                    stop test of Algorithm 1 / 2 reads;
 *   TRUE_RECURRENCE: || beta e_1 - H_{j+1,j} y_j ||, the residual in the
 *                    coordinates of the basis W_{j+1} (eq. (FGK) gives
 *                    b - A x_j = W_{j+1} (beta e_1 - H_{j+1,j} y_j)); it equals
 *                    ||b - A x_j|| when the columns of W_{j+1} are orthonormal
 *                    (a window covering the whole basis) and estimates it with a
 *                    truncated window;
 *   TRUE_EXPLICIT:   ||b - A x_j||, the residual of the discrepancy principle
 *                    (eq. (discrP)): recorded every iteration when
 *                    sfk_params.resid >= 1, else computed when asked (one
 *                    solution assembly and one product per iterate). */
typedef enum { SFK_RES_SKETCHED = 0, SFK_RES_TRUE_RECURRENCE = 1, SFK_RES_TRUE_EXPLICIT = 2 } sfk_res_kind;

/* CSR matrix, device arrays: rowptr[rows + 1], colind[nnz], val[nnz]. */
typedef struct {
  int64_t rows, cols, nnz;
  const int32_t *rowptr;
  const int32_t *colind;
  const double *val;
} sfk_csr;

/* Matrix-free parallel-beam operators (computed on the fly, nothing stored).
 * An N x N image of unit pixels on [-N/2, N/2]^2, row-major (row = y index);
 * nz slices (parallel beam rotating about z, detector row z sees slice z; 1
 * for 2D); n_angles directions u_a = (cos_a[a], sin_a[a]) (device arrays);
 * n_det unit bins centred at t_d = d - (n_det - 1)/2.  Ray (z, a, d), index
 * (z n_angles + a) n_det + d, is the line t_d u_a + lambda (-sin_a, cos_a).
 * A: exact intersection lengths (Siddon: the ray's interval in the image cut
 * at every grid-line crossing, each piece to the pixel holding its midpoint,
 * pieces <= 1e-9 dropped).  B: back = 0 the exact transpose of A; back = 1
 * pixel-driven linear interpolation between the two bins nearest to the
 * pixel centre's projection (an unmatched back-projector). */
typedef struct {
  int32_t N, nz, n_angles, n_det;
  const double *cos_a, *sin_a;
  int32_t back;
  int32_t reserved;
} sfk_beam;

typedef struct {
  int32_t method;      /* sfk_method */
  int32_t ell;         /* orthogonalisation window, 0..8; the paper uses 2 (Sec. 3) */
  int32_t maxit;       /* capacity: maximum number of iterations, 1..s-1 */
  int32_t sketch;      /* sfk_sketch_kind */
  int32_t s;           /* sketch rows: 1..2048, s > maxit, s <= d (SRHT: s <= N) */
  int32_t zeta;        /* SPARSE_SIGN nonzeros per column, 1..min(s, 64) */
  uint64_t seed;       /* Philox key word 0 */
  int32_t instance;    /* Philox stream offset (distinct instances of a batch) */
  int32_t tau;         /* sfk_tau */
  double eps;          /* reweighting parameter, > 0 for REWEIGHT_L1 */
  double eta;          /* discrepancy safety factor (eq. (discrP)), e.g. 1.01 */
  double noise_norm;   /* delta_e = ||e||; > 0 enables the discrepancy stop (sFLSQR) */
  double tol;          /* relative tolerance of the sketched stop test when the
                          discrepancy stop is off; 0 runs to maxit */
  int32_t driver;      /* sfk_driver */
  int32_t vw;          /* SpMV kernel: -2 = automatic (the default: CSR-stream,
                          a wave per row and SELL-64 are timed at init on each
                          operator and the fastest is kept, so two contexts may
                          differ in kernel and hence in rounding; vw / vw_b from
                          sfk_spmv_variant repeat a choice), 0 = CSR-stream chunks,
                          1 = SELL-64 copy built at init (64-row slices stored
                          column-major), 8/16/32/64 = lanes per row, -1 = lanes per
                          row chosen from the mean row length.  Right-hand sides
                          sharing A and B (sfk_init_multi): column-sliced products
                          with the block rows gathered from L2 (0), staged through
                          LDS in units of nearby rows (2, where a unit's rows fit),
                          or staged where the plan reuses each staged row at least
                          5 times on average (-2); any other value = row kernel */
  int32_t vw_b;        /* SpMV kernel of B, coded as vw, when vw_split = 1 (vw then
                          applies to A only); e.g. to repeat the kernels an earlier
                          automatic choice made (sfk_spmv_variant) */
  int32_t vw_split;    /* 0: vw applies to A and B; 1: vw to A, vw_b to B */
  int32_t wg_per_cu;   /* data-parallel workgroups per CU; 0 = automatic */
  int32_t resid;       /* explicit true residual ||b - A x_k|| (eq. (discrP)):
                          0 = not computed during the iteration (sfk_residual_norms
                          computes it on request); 1 = recorded every iteration
                          (x_k assembled and one extra product A x_k per
                          iteration, on the side stream); 2 = recorded and used as
                          the stop test instead of the sketched one: stop at the
                          first k with ||b - A x_k|| <= eta * noise_norm (or
                          <= tol * ||b|| when noise_norm is 0), the discrepancy
                          principle as eq. (discrP) states it */
  int32_t copies;      /* 0: sfk_init may allocate device copies of A and B beyond
                          the workspace (SELL-64, 16-bit column indices, the
                          renumbered operators of perm; sfk_memory reports their
                          size); 1: it may not: CSR-stream or row kernels on the
                          caller's arrays (and the transpose in the workspace),
                          SFK_EINVAL with perm or vw = 1 */
  int32_t tape;        /* derivative tape for sfk_adjoint: 0 = none; c >= 1 keeps a
                          checkpoint of the w window every c iterations (the
                          adjoint regenerates the basis between checkpoints).
                          sFLSQR with B = A^T (B NULL), no perm, maxit <= 1024,
                          single-instance contexts */
  const int32_t *perm; /* optional order of the n unknowns: a device array of n
                          distinct values in [0, n), or NULL (identity).  Unknown j
                          is stored at position perm[j] inside the library: columns
                          of A and rows of B are renumbered at init (into copies the
                          context owns; the caller's arrays are not modified) and
                          sketches of n-vectors (sFLSMR) read through perm, so the
                          iterates are those of the caller's numbering up to the
                          summation order of the products; solutions and residuals
                          are returned in the caller's order.  An order that keeps
                          unknowns read by the same rows close together (e.g. 4 x 4
                          pixel tiles of an image) makes the gathers of the products
                          touch fewer cache lines.  With perm, rows of A must have at
                          most 4096 entries (SFK_EINVAL otherwise).  Must stay valid
                          until sfk_init returns. */
  /* low-rank operators (tau LOWRANK / LOWRANK_RND) */
  int32_t lr_rows;     /* image rows nr; n must be a multiple (nc = n / nr) */
  int32_t lr_rank;     /* r, 1 <= r < min(nr, nc) */
  int32_t lr_over;     /* oversampling p, l = min(r + p, nr, nc) <= 64; 0 = automatic:
                          LOWRANK l = min(max(2 r, r + 16), 64), LOWRANK_RND p = 10 */
  int32_t lr_q;        /* LOWRANK_RND power iterations, 0..16 (default 1) */
  int32_t lr_maxit;    /* LOWRANK power-iteration limit per call; 0 = 300 */
  int32_t lr_reserved;
  double lr_tol;       /* LOWRANK Ritz-residual tolerance relative to theta_1; 0 = 1e-13 */
} sfk_params;

/* Fills *p with defaults: sFLSQR, ell = 2, maxit = 50, sparse-sign s = 101, zeta = 8,
 * seed 0, tau identity, eps 1e-3, eta 1.01, no discrepancy stop, tol 0, AUTO,
 * vw -2 (automatic SpMV kernel), lr_q = 1, the other lr_ fields 0. */
void sfk_params_default(sfk_params *p);

/* Host-only check of dimensions and parameters (no device access).  A and B
 * may have NULL arrays here; B NULL means B = A^T.  Returns SFK_OK or
 * SFK_EINVAL with sfk_last_error(NULL) set. */
sfk_status sfk_validate(const sfk_csr *A, const sfk_csr *B, const sfk_params *p);

/* Device workspace the context needs for these sizes (bytes, 256-aligned
 * sub-buffers included).  Returns 0 when the arguments are invalid. */
size_t sfk_workspace_bytes(const sfk_csr *A, const sfk_csr *B, const sfk_params *p);

/* Creates a context (Algorithm 1 / 2 initialisation: beta = ||b||, w_1 = b / beta,
 * z = B w_1, S b or S B w_1, and the first basis vector).
 *   A: m x n CSR (forward projector).  B: n x m CSR, or NULL for B = A^T (built
 *   on the device).  b: m-vector.  workspace: device buffer of at least
 *   sfk_workspace_bytes(...) bytes, or NULL to let the library allocate (and
 *   free in sfk_destroy).  stream: hipStream_t or NULL.
 * Validates the CSR structures on the device (SFK_EINVAL on a bad row pointer
 * or column index) and b (SFK_EINVAL if zero or non-finite).  Synchronises the
 * stream before returning. */
sfk_status sfk_init(sfk_ctx **out, const sfk_csr *A, const sfk_csr *B, const double *b,
                    const sfk_params *p, void *workspace, size_t workspace_bytes, void *stream);

/* As sfk_init, with the matrix-free operators of geo (m = nz n_angles n_det,
 * n = nz N^2) instead of stored matrices: the products compute the
 * intersection lengths on the fly (SpMV kernel code 3).  Single instance;
 * perm, tape and vw = 1 are not taken (SFK_EINVAL). */
sfk_status sfk_init_beam(sfk_ctx **out, const sfk_beam *geo, const double *b, const sfk_params *p,
                         void *workspace, size_t workspace_bytes, void *stream);

/* y = A x (op 0, y an m-vector) or y = B x (op 1, y an n-vector) with the
 * context's operators and SpMV kernels (device vectors; contexts without perm,
 * single instance).  Synchronous. */
sfk_status sfk_apply(sfk_ctx *ctx, int32_t op, const double *x, double *y);

/* y = tau(x): the context's low-rank operator (tau LOWRANK or LOWRANK_RND,
 * eq. (def:lowr-trc)) applied to the n-vector x (device), into y (device; may
 * not alias x), as the solver applies it to basis vector `call` (>= 1: the
 * randomized variant's test matrix is that of call).  Uses the context's
 * low-rank scratch: do not overlap with sfk_iterate.  Synchronous.
 * SFK_EINVAL for other tau. */
sfk_status sfk_tau_apply(sfk_ctx *ctx, const double *x, double *y, int32_t call);

/* Counters of the low-rank operator's last application: out_host[0] power
 * iterations, out_host[1] 1 if its residual test passed (LOWRANK), out_host[2]
 * applications so far that reached lr_maxit unconverged; *resmax_host the last
 * max_i ||C v_i - theta_i x_i|| / theta_1 (LOWRANK).  SFK_EINVAL for other tau. */
sfk_status sfk_tau_stats(sfk_ctx *ctx, int32_t *out_host, double *resmax_host);

/* Runs up to k more iterations (Algorithm 1 / 2 loop body), stopping early on
 * the stop test or a breakdown.  Synchronous: returns after the device
 * finished.  *iters_done_host = total iterations completed so far (index of the
 * current iterate), *stopped_host = 1 if the stop test fired.  Returns
 * SFK_BREAKDOWN if the basis could not be extended (iterates up to
 * *iters_done_host stay valid), SFK_ESTATE if the capacity maxit is exhausted
 * or the run has already stopped.  For a batch: runs k lockstep iterations,
 * *iters_done_host = lockstep iterations so far, *stopped_host = 1 once every
 * instance has stopped; per-instance results via sfk_instance_status. */
sfk_status sfk_iterate(sfk_ctx *ctx, int32_t k, int32_t *iters_done_host, int32_t *stopped_host);

/* x_k = Z_k y_k for the current k, written to the device n-vector x. */
sfk_status sfk_solution(sfk_ctx *ctx, double *x);

/* x_j = Z_j y_j for 1 <= j <= current k (y_j from the stored factorisation). */
sfk_status sfk_solution_at(sfk_ctx *ctx, int32_t j, double *x);

/* Residual history of kind `kind` (sfk_res_kind) for j = 1..k, k = iterations
 * done: copies min(k, cap) values to out_host, *count_host = k.
 *   SFK_RES_SKETCHED: rho_j = min_y ||S(A Z_j y - b)|| (sFLSQR) or
 *     ||S(B A Z_j y - B b)|| (sFLSMR).
 *   SFK_RES_TRUE_RECURRENCE: ||beta e_1 - H_{j+1,j} y_j|| (host arithmetic on the
 *     stored coefficients and y_j).
 *   SFK_RES_TRUE_EXPLICIT: ||b - A x_j||; recorded values when sfk_params.resid
 *     >= 1, else each x_j is assembled and multiplied on the device when asked.
 * *rhs_norm_host (may be NULL) receives the scale of the matching stop test:
 * ||S b|| (resp. ||S B b||) for SKETCHED, ||b|| for the two true kinds.
 * SFK_EINVAL for an unknown kind or out_host NULL with cap > 0 and k > 0. */
sfk_status sfk_residual_norms(sfk_ctx *ctx, int32_t kind, double *out_host, int32_t cap,
                              int32_t *count_host, double *rhs_norm_host);

/* Explicit true residual ||b - A x_k|| of the current iterate (one extra SpMV). */
sfk_status sfk_true_residual(sfk_ctx *ctx, double *out_host);

/* Device memory of the context, in bytes: *workspace_host = the workspace
 * (borrowed from the caller or allocated by sfk_init), *library_host = what
 * sfk_init allocated besides it (copies of the operators: SELL-64, 16-bit column
 * indices, renumbered operators, column-sliced copies of shared operators;
 * descriptors and block maps; the halt flags).  sfk_params.copies = 1 keeps the
 * copies out.  Either pointer may be NULL. */
sfk_status sfk_memory(const sfk_ctx *ctx, size_t *workspace_host, size_t *library_host);

/* Frees the context and the workspace it allocated.  NULL is a no-op. */
sfk_status sfk_destroy(sfk_ctx *ctx);

/* Error description of the last failing call on ctx (NULL: of the calling
 * thread's last failure outside a context).  Never NULL. */
const char *sfk_last_error(const sfk_ctx *ctx);

/* ---- batches of independent instances ------------------------------------ */

/* Creates a context holding nb independent instances (uneven sizes allowed),
 * e.g. several tomography problems solved together.  Instance i has its own
 * A[i] (m_i x n_i), B (B == NULL, or B[i].rows == 0: A[i]^T built on the
 * device; else B[i], n_i x m_i), right-hand side b[i] (device, m_i) and
 * parameters p[i] (its own method, sketch, seed, tolerance and stop test).
 * All instances advance in lockstep: each stage kernel serves every live
 * instance in one launch, workgroups shared by nonzero count.  An instance
 * that stops (discrepancy principle, tolerance, breakdown) is skipped from then
 * on; the others continue.  Workspaces are allocated by the library.  The
 * plain entry points (sfk_iterate, sfk_solution, ...) act on instance 0 or on
 * the whole batch as documented there. */
sfk_status sfk_init_batch(sfk_ctx **out, int32_t nb, const sfk_csr *A, const sfk_csr *B,
                          const double *const *b, const sfk_params *p, void *stream);

/* ---- right-hand sides sharing one operator pair ----------------------------- */

/* Creates a context holding R right-hand sides (1 <= R <= 64) of one problem
 * pair A (m x n), B (n x m, or NULL for A^T built on the device), e.g. 32
 * phantoms measured with one scanner geometry.  b_block (device) holds the R
 * right-hand sides column after column: b_r = b_block + r * m.  p[r] gives
 * the parameters of right-hand side r; they must agree in method, ell, maxit,
 * sketch kind, s, zeta (sparse-sign) and tau / eps, and may differ in seed and
 * instance (each right-hand side draws its own sketch), eta, noise_norm and
 * tol (each has its own stop test).  Every iteration reads A and B once for
 * all right-hand sides: the long vectors are stored interleaved (element i of
 * right-hand side r next to that of r + 1), so the products run as a sparse
 * matrix times a block of vectors.  Each right-hand side is an instance of the
 * context: sfk_instance_status / _solution / _residual_norms report it, and
 * one that stops is skipped from then on while the others continue.
 * Workspaces are allocated by the library; A, B and b_block are borrowed and
 * must outlive the context.  SFK_EINVAL for an R out of range, parameters that
 * differ where they must agree, or any error sfk_init reports. */
sfk_status sfk_init_multi(sfk_ctx **out, const sfk_csr *A, const sfk_csr *B,
                          const double *b_block, int32_t R, const sfk_params *p, void *stream);

/* Number of instances of a context (1 for sfk_init). */
int32_t sfk_batch_size(const sfk_ctx *ctx);

/* Iterations completed, stop flag and breakdown bits (1: t_{k+1,k+1} = 0,
 * 2: h_{k+1,k} = 0, 4: zero sketched column) of instance i. */
sfk_status sfk_instance_status(sfk_ctx *ctx, int32_t i, int32_t *iters_done_host,
                               int32_t *stopped_host, int32_t *breakdown_host);

/* x_k of instance i at its own k (device n_i-vector x). */
sfk_status sfk_instance_solution(sfk_ctx *ctx, int32_t i, double *x);

/* x_j of instance i for 0 <= j <= its k (see sfk_solution_at). */
sfk_status sfk_instance_solution_at(sfk_ctx *ctx, int32_t i, int32_t j, double *x);

/* Residual history of instance i (see sfk_residual_norms). */
sfk_status sfk_instance_residual_norms(sfk_ctx *ctx, int32_t i, int32_t kind, double *out_host,
                                       int32_t cap, int32_t *count_host, double *rhs_norm_host);

/* ||b_i - A_i x_k|| of instance i at its own k (see sfk_true_residual). */
sfk_status sfk_instance_true_residual(sfk_ctx *ctx, int32_t i, double *out_host);

/* ---- introspection, for parity tests ------------------------------------ */

/* Sparse-sign sketch as generated on the device: rows_host[d * zeta] and
 * neg_host[d * zeta] (1 = negative), column-major in draw order, d = m
 * (sFLSQR) or n (sFLSMR).  SFK_ESTATE for other sketch kinds. */
sfk_status sfk_sketch_sparse_sign(sfk_ctx *ctx, int32_t *rows_host, int8_t *neg_host);

/* SRHT sketch: rows_host[s] and neg_host[N] (D signs), *N_host = N. */
sfk_status sfk_sketch_srht(sfk_ctx *ctx, int32_t *rows_host, int8_t *neg_host, int64_t *N_host);

/* Recurrence coefficients of eq. (FGK) for the first k steps: H_host
 * ((k+1) x k, column-major) and T_host (k x k, column-major). */
sfk_status sfk_coefficients(sfk_ctx *ctx, double *H_host, double *T_host, int32_t k);

/* Basis vector of eq. (FGK) of instance i after k iterations (a live run, not
 * stopped): kind 0 = w_j (unit m-vector; kept for k - ell <= j <= k + 1),
 * kind 1 = p_j (unit n-vector before tau; kept for every j <= k when tau is the
 * identity, for k + 1 - ell <= j <= k with the reweighting), kind 2 =
 * z_j = tau(p_j) (n-vector, kept for 1 <= j <= k).  n-vectors are written in
 * the caller's order of the unknowns.  out: device vector of m or n doubles.
 * SFK_ESTATE when the vector is not kept or the run has halted. */
sfk_status sfk_basis_vector(sfk_ctx *ctx, int32_t i, int32_t kind, int32_t j, double *out);

/* ---- allocation-free solve ------------------------------------------------ */

/* Device scratch of sfk_solve_noalloc, per device (bytes). */
#define SFK_NOALLOC_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture
 * elsewhere in the process, tight serving loops, harnesses that forbid
 * hipMalloc): sfk_init + sfk_iterate(k) + sfk_solution in one call for a
 * single instance, with every device buffer (workspace, transposed B,
 * descriptor, block maps) carved from a fixed array of SFK_NOALLOC_BYTES inside
 * the library, one per device, held until the process ends.  It calls no
 * hipMalloc / hipFree, creates no stream or event and allocates no host memory.
 *   A, B, b, p: as for sfk_init; perm must be NULL and vw must not be 1 (no
 *   copies of the operators are built; vw = -2 means CSR-stream, no tuning).
 *   Everything runs on `stream` (the sketch and the least-squares update in
 *   order between the products), and the call returns after synchronising it.
 *   k: iterations to run (0 <= k <= p->maxit; the stop test ends the run early).
 *   x: device n-vector receiving x_done.  rho_host: NULL or room for k doubles
 *   (rho_1..rho_done).  *iters_done_host, *stopped_host as for sfk_iterate.
 * Returns SFK_ENOMEM (before any device work) when the problem needs more than
 * SFK_NOALLOC_BYTES, SFK_BREAKDOWN as sfk_iterate, else the errors of sfk_init.
 * The array keeps the last call's contents; every call clears what it uses.
 * Calls on one device are serialised by the library (host threads wait for each
 * other); device work that overlaps a call from outside, e.g. a second process
 * loading the library, has its own copy of the array. */
sfk_status sfk_solve_noalloc(const sfk_csr *A, const sfk_csr *B, const double *b,
                             const sfk_params *p, int32_t k, double *x, double *rho_host,
                             int32_t *iters_done_host, int32_t *stopped_host, void *stream);

/* ---- derivative ------------------------------------------------------------- */

/* Reverse-mode derivative of x_K (K = iterations done) of a context created
 * with sfk_params.tape = c >= 1 (sFLSQR, B = A^T): given xbar = dL/dx_K
 * (device n-vector), writes bbar = dL/db (device m-vector) and *epsbar_host =
 * dL/deps, eps the parameter of the l1 reweighting (0 with tau = identity).
 * The derivative is that of the map b, eps -> x_K defined by K steps of eq.
 * (FGK) and eq. (sFLSQR) with the sketch held fixed; the basis between the
 * checkpoints is regenerated from eq. (FGK).  SFK_ESTATE if the context has no
 * tape or its run stopped or broke down before K.  Allocates its own scratch
 * (device), freed before returning; synchronous. */
sfk_status sfk_adjoint(sfk_ctx *ctx, const double *xbar, double *bbar, double *epsbar_host);

/* ---- timing ---------------------------------------------------------------- */

/* Stages of one iteration, in the order the multi-kernel driver runs them. */
typedef enum {
  SFK_STAGE_SPMV_A = 0,    /* w = A z_k with the window dot products   (paper Alg. 1/2) */
  SFK_STAGE_W_UPDATE = 1,  /* truncated Gram-Schmidt of w, ||w||                  */
  SFK_STAGE_SKETCH = 2,    /* one new sketched column                            */
  SFK_STAGE_LS = 3,        /* Householder update of the sketched least squares    */
  SFK_STAGE_SPMV_B = 4,    /* z = B w_{k+1} with the window dot products          */
  SFK_STAGE_P_UPDATE = 5,  /* truncated Gram-Schmidt of z, tau, ||p||             */
  SFK_STAGE_TAU = 6,       /* the low-rank operators' z = tau_r(p) (LOWRANK*)    */
  SFK_NUM_STAGES = 7
} sfk_stage;

/* Enables (on != 0) or disables timing of every stage kernel with HIP events
 * recorded on the context's stream, and clears the accumulated times.  Timing
 * adds event records between the kernels. */
sfk_status sfk_set_timing(sfk_ctx *ctx, int32_t on);

/* Accumulated kernel time per stage (ms_host[SFK_NUM_STAGES]) and number of
 * timed launches (count_host[SFK_NUM_STAGES]) since sfk_set_timing. */
sfk_status sfk_stage_times(sfk_ctx *ctx, double *ms_host, int32_t *count_host);

/* SpMV kernel in use for A and for B: 0 CSR-stream, 1 SELL-64, 64 a wave per
 * row with the whole row in flight, 8/16/32 lanes per row; for right-hand
 * sides sharing A and B -2 (column-sliced products gathering from L2), -4 (column-sliced
 * products staged through LDS) or -3 (row kernel).  A batch runs one kernel for
 * all instances: instance 0's, or CSR-stream when the instances differ. */
sfk_status sfk_spmv_variant(const sfk_ctx *ctx, int32_t *vwA_host, int32_t *vwB_host);

/* Library and device description (static string). */
const char *sfk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SFK_H */
