// Internal device-side layout of one solver instance.  Everything here is
// FP64 except indices; all arrays live in one device workspace carved by the
// host (sfk_capi.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfk {

constexpr int kMaxEll = 8;                 // orthogonalisation window limit
constexpr int kMaxS = 2048;                // sketch rows limit (LS kept in one wave)
constexpr int kWG = 256;                   // threads per vector-stage workgroup
constexpr int kSpmvWG = 1024;              // threads per SpMV workgroup
constexpr int kRowsLDS = 2048;             // SpMV results kept in LDS for the epilogue
constexpr int kMaxQ = kMaxEll + 2;         // partial sums per workgroup and stage
constexpr int kSrhtL = 2048;               // SRHT block length staged in LDS
constexpr double kBreakdownTol = 1e-14;    // relative breakdown threshold

// Partial-sum buffers, one per producing stage.
enum Stage { kStageA = 0, kStageB = 1, kStageC = 2, kStageD = 3, kStageMisc = 4, kNumPart = 5 };

// Scalar state shared by the stages (device memory).  Slots: w_j lives in
// W ring slot j % (ell + 2), p_j in P ring slot j % (ell + 1).
struct Scal {
  double beta;        // ||b||
  double rhsnorm;     // ||S b|| (sFLSQR) or ||S B b|| (sFLSMR)
  double tol;         // relative tolerance of the stop test (0: none)
  double wpre;        // ||A z_k|| before orthogonalisation
  double zpre;        // ||B w_{k+1}|| before orthogonalisation
  double Gw[(kMaxEll + 2) * (kMaxEll + 2)];  // <w_i, w_j> by slot
  double Gp[(kMaxEll + 1) * (kMaxEll + 1)];  // <p_i, p_j> by slot
  int halt;           // 1: no further stage may run (stop test, or after a breakdown's LS)
  int klimit;         // last iteration whose basis vector exists (t breakdown)
  int stopped;        // stop test fired
  int breakdown;      // bits: 1 t_{k+1,k+1} = 0, 2 h_{k+1,k} = 0, 4 zero sketched column
  int k_done;         // iterations whose LS has completed
  int happy;          // iteration k with h_{k+1,k} = 0 (0: none)
  int err;            // device-detected error code
  int pad;
};

struct Dev {
  // sizes and parameters
  int m, n, s, ell, maxit, method, tau, sketch, zeta;
  int d_sk;           // length of sketched vectors (m or n)
  int N;              // SRHT padded length
  int log2L;          // SRHT block length log2
  int nblk;           // SRHT blocks
  int nws;            // SpMV workgroups of this instance (row ranges)
  int nwv;            // vector-stage workgroups of this instance
  int nwmax;          // stride of the per-stage partial-sum buffers
  int nsg;            // sparse-sign sketch gather workgroups of this instance
  int vwA, vwB;       // SpMV lanes per row
  double eps;
  double sk_scale;    // 1/sqrt(zeta) or 1/sqrt(s)
  // operators
  const int *Arp, *Aci; const double *Ava;
  const int *Brp, *Bci; const double *Bva;
  const double *b;
  const int *Apart, *Bpart;    // nnz-balanced row ranges, nws + 1 entries each
  // vectors
  double *W;          // (ell + 2) * m, unnormalised w~_j
  double *P;          // (ell + 1) * n, unnormalised p~_j (unused when tau = I)
  double *Z;          // (maxit + 1) * n, z~_j (column j-1)
  double *wraw;       // 2 * m, A z_k in slot k & 1
  double *zraw;       // 2 * n, B w_{k+1} in slot k & 1
  double *x;          // n, current iterate (reweighting) / scratch
  // sketch
  int *sk_rp;         // s + 1   (sparse-sign, transposed: entries per sketch row)
  int *sk_ent;        // zeta * d: column | (negative << 31)
  int *sk_code;       // zeta * d: (row << 1) | negative, per column in draw order
  int *srht_rows;     // s
  unsigned long long *srht_d;  // N / 64 sign words
  double *srht_part;  // nblk * s
  double *SK;         // s * (maxit + 1), sketched columns
  double *skrhs;      // s
  // stage reductions
  double *part;       // kNumPart * kMaxQ * nwmax
  Scal *sc;
  double *sigw;       // maxit + 2: 1 / ||w~_j||
  double *sigp;       // maxit + 2: 1 / ||p~_j||
  double *H;          // (maxit + 1) * maxit, column-major
  double *T;          // (maxit + 1) * (maxit + 1), column-major
  double *rho;        // maxit
  // small least-squares state (Householder QR of the sketched matrix)
  double *V;          // s * maxit reflectors (v_j[j] = 1, zeros above)
  double *tauv;       // maxit
  double *R;          // maxit * maxit, column-major
  double *c;          // s: Q^T rhs
  double *y;          // maxit: y_k (kept current for the reweighting)
};

// Launch geometry of a batch of instances: the device array of instance
// descriptors and, per stage type, a block -> (instance, workgroup) map.
struct Launch {
  const Dev *devs;
  const int2 *map_spmv, *map_vec, *map_sg, *map_sb, *map_sc;
  int nspmv, nvec, nsg, nsb, nsc;   // grid sizes
  int ninst, smax, maxitmax, tau, vwA, vwB;
};

__device__ __forceinline__ int wslot(const Dev &D, int j) { return j % (D.ell + 2); }
__device__ __forceinline__ int pslot(const Dev &D, int j) { return j % (D.ell + 1); }
__device__ __forceinline__ double *wrawk(const Dev &D, int k) { return D.wraw + (size_t)(k & 1) * D.m; }
__device__ __forceinline__ double *zrawk(const Dev &D, int k) { return D.zraw + (size_t)(k & 1) * D.n; }
__device__ __forceinline__ double *wvec(const Dev &D, int j) { return D.W + (size_t)wslot(D, j) * D.m; }
__device__ __forceinline__ double *pvec(const Dev &D, int j) {
  // with tau = I the stored basis column z~_j is p~_j itself
  return D.tau == 0 ? D.Z + (size_t)(j - 1) * D.n : D.P + (size_t)pslot(D, j) * D.n;
}

}  // namespace sfk
