// Rank-r truncation of a basis vector viewed as an image (the flexible
// operator tau_r of eq. (def:lowr-trc), and its randomized-SVD variant used by
// the -RND solvers of Sec. 3.1): the host interface of sfk_lowrank.hip.
//
// C is the nr x nc image of the vector (row-major: entry (i, j) at i * nc + j).
// Both variants run the randomized subspace iteration of Halko, Martinsson and
// Tropp (Algorithm 4.4) on C with l = r + p test vectors, re-basing after
// every product (orthonormal before each Rayleigh-Ritz step), then a
// Rayleigh-Ritz step on span(Q): the eigenpairs
// (theta_i, e_i) of M = Z^T Z, Z = C^T Q, give x_i = Q e_i, v_i = C^T x_i =
// Z e_i and tau_r(C) = sum_{i<r} x_i v_i^T.  For the randomized variant M is
// B B^T with B = Q^T C, so this is their Algorithm 5.1 truncated to rank r
// after q power iterations.  The truncated-SVD variant continues the same
// iteration until the Ritz residuals ||C v_i - theta_i x_i||, i < r, are at
// most tol * theta_1: it then agrees with the full SVD's truncation to within
// that residual divided by the gap theta_r - sigma_{l+1}^2.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sfk {

struct Scal;

constexpr int kLrMaxL = 64;     // test vectors (r + p) at most
constexpr int kLrTM = 32;       // rows of a product / reduce / apply workgroup (one Gram slice)
constexpr int kLrSplit = 8;     // ranges of the inner dimension of a product

struct LrBufs {
  int nr = 0, nc = 0, r = 0, l = 0;
  int rnd = 0;                  // 1: randomized SVD with q power iterations; 0: truncated SVD
  int q = 1;                    // power iterations (randomized)
  int maxit = 300;              // power-iteration limit (truncated SVD)
  int check = 4;                // first Rayleigh-Ritz residual check (truncated SVD)
  double tol = 1e-13;           // residual tolerance relative to theta_1
  uint64_t seed = 0;
  int instance = 0;
  // device buffers (column-major, leading dimension = row count)
  double *Q = nullptr, *Y = nullptr;   // nr x l each
  double *Z = nullptr, *ZE = nullptr;  // nc x l each
  double *XE = nullptr;                // nr x l: Q E (Ritz vectors; the first r are x_i)
  double *CV = nullptr;                // nr x r: C v_i
  double *part = nullptr;              // kLrSplit x max(nr, nc) x l partial products
  double *Wp = nullptr;                // slices x l (l + 1) / 2 packed Gram partials
  double *R = nullptr;                 // l x l Cholesky factor (upper, column-major)
  double *E = nullptr, *th = nullptr;  // l x l eigenvectors (descending), l eigenvalues
  double *rb = nullptr;                // read back by the host: max_i res_i / theta_1,
                                       // theta_r, theta_l
  int *stat = nullptr;                 // [0] active, [1] converged, [2] iterations of
                                       // the last call, [3] calls that reached maxit,
                                       // [4] arrival counter of the last-block steps
};

// Doubles of workspace for these sizes (the int status words included).
size_t lr_doubles(int nr, int nc, int r, int l);
// Points the buffers of L into base (lr_doubles(...) doubles, 256-byte aligned).
void lr_carve(LrBufs &L, double *base);

// z~ = tau_r(p~) for the basis vector of call index k + 1 (p~ nr * nc long,
// unnormalised: tau_r is homogeneous).  sc, maxit and full decide on the
// device whether the iteration is live (the stage is skipped otherwise, as the
// stage kernels are): full = 0 for the sketched solvers' D(k), 1 for the full
// orthogonalisation path.  The truncated-SVD variant reads its convergence
// flag on the host every `check` iterations (a synchronisation of st); the
// randomized variant only enqueues.  Returns hipSuccess or the first launch
// error.
hipError_t lr_apply(const LrBufs &L, const Scal *sc, int maxit, int full, int k, const double *pin,
                    double *zout, hipStream_t st);

}  // namespace sfk
