// Rank-r truncation tau_r of a basis vector viewed as an nr x nc image (eq.
// (def:lowr-trc)) and its randomized-SVD variant: randomized subspace
// iteration with a re-basing after every product, a Rayleigh-Ritz step, and
// the rank-r product of the Ritz vectors (see sfk_lowrank.h).
//
// Kernels.  A product launch splits the inner dimension into kLrSplit ranges
// (workgroup (b, s): 32 rows, range s); a reduce launch adds the ranges in
// order for 32 rows per workgroup and forms the Gram matrix of its rows (upper
// triangle, one slice); an apply workgroup solves x R = y for 32 rows with the
// triangular R and forms their Gram slice the same way.  The last workgroup of
// a reduce or apply launch to finish (an arrival counter: release fence,
// device-scope atomic, acquire fence) sums the slices in slice order and
// computes the Cholesky factor the next launch needs; it then resets the
// counter.  The Rayleigh-Ritz step's eigen-decomposition runs in a workgroup
// of its own.  Every sum runs in a fixed order, so results are reproducible
// run to run.  The kernels of one call share a status word: stat[0] = 0 (the
// solver iteration is not live) turns every later kernel of the call into a
// no-op.
//
// Orthonormalisation: shifted Cholesky QR followed by two plain Cholesky QR
// passes (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa, "Shifted
// Cholesky QR for computing the QR factorization of ill-conditioned
// matrices", SIAM J. Sci. Comput. 2020): the shift 11 (M l + l (l + 1)) u
// ||Y||_F^2 keeps the first Cholesky factorisation defined for any Y, the two
// later passes restore orthonormality to working precision.  Between the
// products of the iteration only the range matters: the shifted pass alone
// re-bases C C^T Q once per iteration (its condition number is at most
// (sigma_1 / sigma_l)^2, within what the shifted pass handles).
//
// Small symmetric eigenproblem: cyclic two-sided Jacobi with the round-robin
// ordering of disjoint pairs (Golub and Van Loan, Sec. 8.5) in LDS; a rotation
// is skipped when |a_pq| is below u sqrt(|a_pp a_qq|) or 1e-3 u ||A||_F
// (u the unit roundoff), the rotated entry is set to zero, and the sweeps stop
// when a sweep rotates nothing.  The truncated-SVD
// variant continues its iteration from the Ritz basis, so that the next
// Rayleigh-Ritz matrix is nearly diagonal and takes few sweeps.
#include <float.h>

#include "sfk_common.h"
#include "sfk_lowrank.h"

namespace sfk {

namespace {

constexpr int kLrWG = 256;
constexpr int kLd = kLrMaxL + 1;      // LDS row stride (odd: no bank conflicts)
constexpr int kSmem = 2 * kLrMaxL * kLd;   // doubles of LDS per workgroup

__device__ __forceinline__ bool lr_live(const int *stat) { return ld_flag(stat) != 0; }

int lr_slices(int M) { return (M + kLrTM - 1) / kLrTM; }
__host__ __device__ __forceinline__ int packed_len(int l) { return l * (l + 1) / 2; }

// stat[0] = 1 when the stage of iteration k runs (same tests as the stage
// kernels: the sketched path's D(k), or the full path's tau step); mode 2
// always runs (a direct application of the operator)
__global__ void k_lr_begin(const Scal *sc, int maxit, int mode, int k, int *stat) {
  if (threadIdx.x != 0) return;
  bool live;
  if (mode == 2) live = true;
  else if (k >= maxit) live = false;
  else if (mode == 1)
    live = k == 0 || (ld_flag(&sc->halt) == 0 && k <= ld_flag(&sc->klimit) && ld_flag(&sc->k_done) == k);
  else
    live = ld_flag(&sc->halt) == 0 && k <= ld_flag(&sc->klimit);
  stat[0] = live ? 1 : 0;
  if (live) {            // the counters keep the last live call's values
    stat[1] = 0;
    stat[2] = 0;
  }
}

// Gaussian test matrix Omega (nc x l, column-major): entry e = j nc + i is
// normal (e mod 4) of the Philox4x64-10 block with counter (call, e >> 2, 0, 0);
// words (w0, w1) and (w2, w3) give two normals each (Box-Muller with
// u1 = ((w_even >> 11) + 1/2) 2^-53 in (0, 1) and u2 = (w_odd >> 11) 2^-53)
__global__ void __launch_bounds__(kLrWG) k_lr_omega(const int *stat, double *__restrict__ Om,
                                                   int total, uint64_t key0, uint64_t key1,
                                                   uint64_t call) {
#pragma clang fp contract(off)
  if (!lr_live(stat)) return;
  const int64_t blk = (int64_t)blockIdx.x * kLrWG + threadIdx.x;
  if (blk * 4 >= total) return;
  uint64_t c[4] = {call, (uint64_t)blk, 0, 0};
  philox4x64_10(c, key0, key1);
  const double two53 = 0x1p-53;
  double nv[4];
#pragma unroll
  for (int pr = 0; pr < 2; ++pr) {
    const double u1 = ((double)(c[2 * pr] >> 11) + 0.5) * two53;
    const double u2 = (double)(c[2 * pr + 1] >> 11) * two53;
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 2.0 * M_PI * u2;
    nv[2 * pr] = rad * cos(ang);
    nv[2 * pr + 1] = rad * sin(ang);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if (blk * 4 + t < total) Om[blk * 4 + t] = nv[t];
}

// ---------------------------------------------------------------------------
// small dense steps of the last workgroup (256 threads, matrices in LDS)
// ---------------------------------------------------------------------------

// Gram slice of rows ys[0..rows) (ncol columns, stride kLd), upper triangle
// packed by rows
__device__ __forceinline__ void unpack(int e, int l, int &a, int &b) {
  int rem = e;
  a = 0;
  while (rem >= l - a) { rem -= l - a; ++a; }
  b = a + rem;
}

__device__ void gram_slice(const double *ys, int rows, int ncol, double *W) {
  const gptr<double> Wg = gmem(W);
  const int P = packed_len(ncol);
  for (int e = threadIdx.x; e < P; e += kLrWG) {
    int a, b;
    unpack(e, ncol, a, b);
    double g = 0.0;
    for (int ii = 0; ii < rows; ++ii) g = fma(ys[ii * kLd + a], ys[ii * kLd + b], g);
    Wg[e] = g;
  }
}

// The arrival counter: true in the last workgroup of the launch to get here,
// after every workgroup's global writes are visible to it.
__device__ bool last_arrival(int *cnt) {
  __shared__ int s_last;
  __threadfence();       // this thread's stores (the Gram slice) reach device scope
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const int prev = atomicAdd(cnt, 1);
    s_last = prev == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  return true;
}

// A (l x l, LDS, stride kLd) = sum over the nsl packed Gram slices, in slice
// order (NT threads)
template <int NT>
__device__ void sum_slices(const double *Wp, int nsl, int l, double *A) {
  const int P = packed_len(l);
  const gptr<const double> wg = gmem(Wp);
  for (int e = threadIdx.x; e < P; e += NT) {
    double v = 0.0;
    int s = 0;
    for (; s + 4 <= nsl; s += 4) {
      const double v0 = wg[(size_t)s * P + e], v1 = wg[(size_t)(s + 1) * P + e];
      const double v2 = wg[(size_t)(s + 2) * P + e], v3 = wg[(size_t)(s + 3) * P + e];
      v += v0;
      v += v1;
      v += v2;
      v += v3;
    }
    for (; s < nsl; ++s) v += wg[(size_t)s * P + e];
    int a, b;
    unpack(e, l, a, b);
    A[a * kLd + b] = v;
    A[b * kLd + a] = v;
  }
  __syncthreads();
}

// Cholesky factor R of W (+ the shift when shift != 0, relative to M rows):
// W = R^T R, R upper triangular, into Rg (l x l, column-major); a zero or
// non-finite trace gives R = I.  Right-looking LDL^T on the upper triangle of
// W (LDS, stride kLd; overwritten): step j subtracts W[j][a] W[j][b] / d_j from
// the trailing block, one barrier per step; then R = D^(1/2) U.
__device__ void chol_factor(double *W, int l, int M, int shift, double *Rg) {
  __shared__ double dg[kLrMaxL];
  __shared__ double s_tr;
  const int t = threadIdx.x;
  if (t == 0) {
    double tr = 0.0;
    for (int a = 0; a < l; ++a) tr += W[a * kLd + a];
    s_tr = tr;
  }
  __syncthreads();
  const double tr = s_tr;
  const gptr<double> rg = gmem(Rg);
  if (!(tr > 0.0) || !isfinite(tr)) {
    for (int e = t; e < l * l; e += kLrWG) rg[e] = (e / l == e % l) ? 1.0 : 0.0;
    return;
  }
  if (shift) {
    const double sh = 11.0 * ((double)M * l + (double)l * (l + 1)) * DBL_EPSILON * tr;
    if (t < l) W[t * kLd + t] += sh;
    __syncthreads();
  }
  const double floor_ = tr * 1e-30;
  // thread t: trailing rows j + 1 + (t >> 4) + 16 i, columns a + (t & 15) + 16 i'
  const int tr16 = t >> 4, tc16 = t & 15;
  for (int j = 0; j < l; ++j) {
    const double d = fmax(W[j * kLd + j], floor_);
    const double inv = 1.0 / d;
    if (t == 0) dg[j] = d;
    for (int a = j + 1 + tr16; a < l; a += 16) {
      const double wja = W[j * kLd + a] * inv;
      for (int b = a + tc16; b < l; b += 16) W[a * kLd + b] -= wja * W[j * kLd + b];
    }
    __syncthreads();
  }
  for (int e = t; e < l * l; e += kLrWG) {
    const int col = e / l, row = e % l;
    const double sd = sqrt(dg[row]);
    rg[e] = row == col ? sd : row < col ? W[row * kLd + col] / sd : 0.0;
  }
}

// Eigen-decomposition of the symmetric A (LDS, l x l): E (global, column-major,
// columns by descending eigenvalue) and th (descending).  V: LDS scratch.  NT
// threads; each round rotates the np disjoint pairs of the round-robin ordering
// (columns, then rows), and sets the rotated a_pq to zero.
template <int NT>
__device__ void jacobi_eig(double *A, double *V, int l, double *E, double *th) {
  __shared__ int pp[kLrMaxL / 2], qq[kLrMaxL / 2];
  __shared__ double cs[kLrMaxL / 2], sn[kLrMaxL / 2];
  __shared__ double red[NT / 64];
  __shared__ int s_rot, s_round;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int e = t; e < l * l; e += NT) V[(e / l) * kLd + e % l] = (e / l == e % l) ? 1.0 : 0.0;
  double f = 0.0;
  for (int e = t; e < l * l; e += NT) {
    const double v = A[(e / l) * kLd + e % l];
    f += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) f += __shfl_xor(f, o);
  if (lane == 0) red[wv] = f;
  if (t == 0) {
    s_rot = 0;
    s_round = 0;
  }
  __syncthreads();
  double fro2 = 0.0;
  for (int w = 0; w < NT / 64; ++w) fro2 += red[w];
  const double absfloor = 1e-3 * DBL_EPSILON * sqrt(fro2);
  const int L2 = l + (l & 1), np = L2 / 2;
  // work items e = slot * l + index of the row / column updates: lane t takes
  // e = t, t + 64, ...
  const int slot0 = t / l, idx0 = t - slot0 * l;
  for (int sweep = 0; sweep < 30; ++sweep) {
    for (int rd = 0; rd < L2 - 1; ++rd) {
      if (t < np) {
        const int pa = t, pb = L2 - 1 - t;
        int p = pa == 0 ? 0 : 1 + (pa - 1 + rd) % (L2 - 1);
        int q = 1 + (pb - 1 + rd) % (L2 - 1);
        if (p > q) { const int x = p; p = q; q = x; }
        double c = 1.0, s = 0.0;
        if (q < l) {
          const double apq = A[p * kLd + q], app = A[p * kLd + p], aqq = A[q * kLd + q];
          const double aa = fabs(apq);
          if (aa > absfloor && aa > DBL_EPSILON * sqrt(fabs(app * aqq))) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = tau >= 0.0 ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                         : -1.0 / (-tau + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
            s_rot = 1;
          }
        }
        pp[t] = p;
        qq[t] = q;
        cs[t] = c;
        sn[t] = s;
        if (s != 0.0) s_round = sweep * L2 + rd + 1;
      }
      __syncthreads();
      if (s_round != sweep * L2 + rd + 1) continue;   // no rotation in this round
      for (int slot = slot0, i = idx0; slot < np;) {   // A <- A J, V <- V J (columns p, q)
        const double s = sn[slot];
        if (s != 0.0) {
          const double c = cs[slot];
          const int p = pp[slot], q = qq[slot];
          const double aip = A[i * kLd + p], aiq = A[i * kLd + q];
          const double vip = V[i * kLd + p], viq = V[i * kLd + q];
          A[i * kLd + p] = c * aip - s * aiq;
          A[i * kLd + q] = s * aip + c * aiq;
          V[i * kLd + p] = c * vip - s * viq;
          V[i * kLd + q] = s * vip + c * viq;
        }
        i += NT;
        while (i >= l) { i -= l; ++slot; }
      }
      __syncthreads();
      for (int slot = slot0, j = idx0; slot < np;) {   // A <- J^T A (rows p, q); a_pq = 0
        const double s = sn[slot];
        if (s != 0.0) {
          const double c = cs[slot];
          const int p = pp[slot], q = qq[slot];
          const double apj = A[p * kLd + j], aqj = A[q * kLd + j];
          A[p * kLd + j] = j == q ? 0.0 : c * apj - s * aqj;
          A[q * kLd + j] = j == p ? 0.0 : s * apj + c * aqj;
        }
        j += NT;
        while (j >= l) { j -= l; ++slot; }
      }
      __syncthreads();
    }
    const int rotated = s_rot;
    __syncthreads();                 // every thread has read s_rot
    if (rotated == 0) break;
    if (t == 0) s_rot = 0;
    __syncthreads();
  }
  const gptr<double> eg = gmem(E), tg = gmem(th);
  for (int i = t; i < l; i += NT) {
    const double di = A[i * kLd + i];
    int rank = 0;
    for (int j = 0; j < l; ++j) {
      const double dj = A[j * kLd + j];
      rank += (dj > di || (dj == di && j < i)) ? 1 : 0;
    }
    tg[rank] = di;
    for (int row = 0; row < l; ++row) eg[(size_t)rank * l + row] = V[row * kLd + i];
  }
}

constexpr int kEigWG = 1024;

// Eigen-decomposition of the Gram matrix summed from the nsl slices in Wp
__global__ void __launch_bounds__(kEigWG) k_lr_eig(const int *stat, const double *__restrict__ Wp,
                                                  int nsl, int l, double *__restrict__ E,
                                                  double *__restrict__ th) {
  if (!lr_live(stat)) return;
  __shared__ double smem[kSmem];
  sum_slices<kEigWG>(Wp, nsl, l, smem);
  jacobi_eig<kEigWG>(smem, smem + kLrMaxL * kLd, l, E, th);
}

enum LastStep { kNone = 0, kChol = 1, kCholShift = 2, kGram = 3 };

struct LrArgs {
  int nr, nc, l;
  int *stat;
  double *Wp, *R, *E, *th, *part;
};

__device__ void last_step(const LrArgs &a, int step, int ncol, int M, double *smem) {
  if (step == kGram || !last_arrival(a.stat + 4)) return;
  sum_slices<kLrWG>(a.Wp, (int)gridDim.x, ncol, smem);
  chol_factor(smem, ncol, M, step == kCholShift, a.R);
  if (threadIdx.x == 0) a.stat[4] = 0;
}

// Split product: part[s] (M x ncol, column-major) = op(C) X over the s-th of
// kLrSplit ranges of the inner dimension, op(C) = C (M = nr, inner nc) or C^T
// (M = nc, inner nr); X is inner x ncol column-major, ncol <= 64.  Workgroup
// (b, s): rows [32 b, 32 b + 32); thread t: rows 4 (t & 7) .. + 3, columns
// t >> 3 and (t >> 3) + 32.  Each chunk of 64 inner indices is staged whole,
// so a workgroup waits for its loads once per chunk.
template <bool TR>
__global__ void __launch_bounds__(kLrWG) k_lr_prod(LrArgs a, const double *__restrict__ C,
                                                  const double *__restrict__ X, int ncol) {
  if (!lr_live(a.stat)) return;
  constexpr int KC = 64;
  __shared__ double As[KC * (kLrTM + 1)];
  __shared__ double Xs[KC * kLd];
  const int nr = a.nr, nc = a.nc;
  const int M = TR ? nc : nr, K = TR ? nr : nc;
  const int i0 = blockIdx.x * kLrTM, rows = min(kLrTM, M - i0);
  const int sp = blockIdx.y;
  const int kper = (K + kLrSplit - 1) / kLrSplit;
  const int k0 = min(K, sp * kper), k1 = min(K, k0 + kper);
  const int t = threadIdx.x, rg = t & 7, cg = t >> 3;
  const gptr<const double> Cg = gmem(C), Xg = gmem(X);
  double acc[4][2];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q][0] = acc[q][1] = 0.0;
  for (int kk = k0; kk < k1; kk += KC) {
    for (int e = t; e < KC * kLrTM; e += kLrWG) {
      int row, kc;
      if (TR) { kc = e / kLrTM; row = e % kLrTM; } else { row = e / KC; kc = e % KC; }
      const int k = kk + kc;
      double v = 0.0;
      if (row < rows && k < k1) v = TR ? Cg[(size_t)k * nc + i0 + row] : Cg[(size_t)(i0 + row) * nc + k];
      As[kc * (kLrTM + 1) + row] = v;
    }
    for (int e = t; e < KC * kLrMaxL; e += kLrWG) {
      const int j = e / KC, kc = e % KC, k = kk + kc;
      Xs[kc * kLd + j] = (j < ncol && k < k1) ? Xg[(size_t)j * K + k] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kc = 0; kc < KC; ++kc) {
      const double x0 = Xs[kc * kLd + cg], x1 = Xs[kc * kLd + cg + 32];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double av = As[kc * (kLrTM + 1) + rg * 4 + q];
        acc[q][0] = fma(av, x0, acc[q][0]);
        acc[q][1] = fma(av, x1, acc[q][1]);
      }
    }
    __syncthreads();
  }
  const gptr<double> pg = gmem(a.part + (size_t)sp * ncol * M);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = rg * 4 + q;
    if (row >= rows) continue;
    if (cg < ncol) pg[(size_t)cg * M + i0 + row] = acc[q][0];
    if (cg + 32 < ncol) pg[(size_t)(cg + 32) * M + i0 + row] = acc[q][1];
  }
}

// out (M x ncol) = the sum of the kLrSplit partial products, split by split;
// with step != kNone, the Gram slice of the workgroup's 32 rows and the last
// workgroup's step
__global__ void __launch_bounds__(kLrWG) k_lr_reduce(LrArgs a, int M, int ncol,
                                                    double *__restrict__ out, int step) {
  if (!lr_live(a.stat)) return;
  __shared__ double smem[kSmem];
  const int i0 = blockIdx.x * kLrTM, rows = min(kLrTM, M - i0);
  const gptr<const double> pg = gmem(a.part);
  const gptr<double> og = gmem(out);
  for (int e = threadIdx.x; e < kLrTM * ncol; e += kLrWG) {
    const int j = e / kLrTM, ii = e % kLrTM;
    double v = 0.0;
    if (ii < rows) {
      const size_t off = (size_t)j * M + i0 + ii;
      double pv[kLrSplit];
#pragma unroll
      for (int sp = 0; sp < kLrSplit; ++sp) pv[sp] = pg[(size_t)sp * ncol * M + off];
#pragma unroll
      for (int sp = 0; sp < kLrSplit; ++sp) v += pv[sp];
      og[off] = v;
    }
    smem[ii * kLd + j] = v;
  }
  if (step == kNone) return;
  __syncthreads();
  gram_slice(smem, rows, ncol, a.Wp + (size_t)blockIdx.x * packed_len(ncol));
  last_step(a, step, ncol, M, smem);
}

// Y <- Y R^{-1} in place: row y of the workgroup's 32 rows becomes the x with
// x R = y (forward substitution over the columns, 8 lanes per row: lane u
// keeps x_c for c = u mod 8 and sums those terms, the group adds its 8 sums);
// with step != kNone, the Gram slice of the new rows and the last workgroup's
// step.
__global__ void __launch_bounds__(kLrWG) k_lr_apply(LrArgs a, double *__restrict__ Y, int M,
                                                   int step) {
  if (!lr_live(a.stat)) return;
  __shared__ double smem[kSmem];
  double *rs = smem;                          // R (l x l, stride kLd), rs[t][c] = R(t, c)
  double *os = smem + kLrMaxL * kLd;          // kLrTM x kLd: the new rows
  __shared__ double rdi[kLrMaxL];             // 1 / R(c, c)
  const int l = a.l;
  const int i0 = blockIdx.x * kLrTM, rows = min(kLrTM, M - i0);
  const gptr<const double> rg = gmem(a.R);
  const gptr<double> yg = gmem(Y);
  for (int e = threadIdx.x; e < l * l; e += kLrWG) rs[(e % l) * kLd + e / l] = rg[e];
  for (int c = threadIdx.x; c < l; c += kLrWG) rdi[c] = 1.0 / rg[c * l + c];
  const int row = threadIdx.x >> 3, u = threadIdx.x & 7;
  const bool has = row < rows;
  // this lane's entries of y: columns c = u + 8 m
  double yv[kLrMaxL / 8], xv[kLrMaxL / 8];
#pragma unroll
  for (int m = 0; m < kLrMaxL / 8; ++m) {
    const int c = u + 8 * m;
    yv[m] = (has && c < l) ? yg[(size_t)c * M + i0 + row] : 0.0;
    xv[m] = 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kLrMaxL; ++c) {
    if (c >= l) break;
    double part = 0.0;
#pragma unroll
    for (int m = 0; m < kLrMaxL / 8; ++m)
      if (u + 8 * m < c) part = fma(xv[m], rs[(u + 8 * m) * kLd + c], part);
    part += __shfl_xor(part, 1, 8);
    part += __shfl_xor(part, 2, 8);
    part += __shfl_xor(part, 4, 8);
    const double yc = __shfl(yv[c >> 3], (threadIdx.x & ~7) | (c & 7), 64);
    const double xc = (yc - part) * rdi[c];
    if (u == (c & 7)) xv[c >> 3] = xc;
  }
#pragma unroll
  for (int m = 0; m < kLrMaxL / 8; ++m) {
    const int c = u + 8 * m;
    if (c < l) {
      os[row * kLd + c] = xv[m];
      if (has) yg[(size_t)c * M + i0 + row] = xv[m];
    }
  }
  if (step == kNone) return;
  __syncthreads();
  gram_slice(os, rows, l, a.Wp + (size_t)blockIdx.x * packed_len(l));
  last_step(a, step, l, M, smem);
}

// Ritz vectors of all l columns: XE = Q E (nr x l), ZE = Z E (nc x l)
__global__ void __launch_bounds__(kLrWG) k_lr_ritz(const int *stat, const double *__restrict__ Q,
                                                  const double *__restrict__ Z,
                                                  const double *__restrict__ E, int nr, int nc,
                                                  int l, double *__restrict__ XE,
                                                  double *__restrict__ ZE) {
  if (!lr_live(stat)) return;
  __shared__ double es[kLrMaxL * kLd];
  const gptr<const double> Eg = gmem(E), Qg = gmem(Q), Zg = gmem(Z);
  for (int e = threadIdx.x; e < l * l; e += kLrWG) es[(e % l) * kLd + e / l] = Eg[e];
  __syncthreads();
  const int64_t rows = (int64_t)nr + nc, total = rows * l;
  for (int64_t e = (int64_t)blockIdx.x * kLrWG + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kLrWG) {
    const int tcol = (int)(e / rows);
    const int64_t i = e % rows;
    double v = 0.0;
    if (i < nr) {
      for (int q = 0; q < l; ++q) v = fma(Qg[(size_t)q * nr + i], es[q * kLd + tcol], v);
      gmem(XE)[(size_t)tcol * nr + i] = v;
    } else {
      const int64_t j = i - nr;
      for (int q = 0; q < l; ++q) v = fma(Zg[(size_t)q * nc + j], es[q * kLd + tcol], v);
      gmem(ZE)[(size_t)tcol * nc + j] = v;
    }
  }
}

// Ritz residuals ||C v_t - theta_t x_t||, t < r (C v_t in CV): stat[1] = 1 when
// their maximum is at most tol * theta_1; rb = (that maximum / theta_1,
// theta_r, theta_l) for the host
__global__ void __launch_bounds__(kLrWG) k_lr_resid(int *stat, const double *__restrict__ CV,
                                                   const double *__restrict__ Xr,
                                                   const double *__restrict__ th, int nr, int r,
                                                   int l, double tol, double *__restrict__ rb) {
  if (!lr_live(stat)) return;
  __shared__ double red[kLrWG / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const gptr<const double> cg = gmem(CV), xg = gmem(Xr);
  double worst = 0.0;
  for (int col = 0; col < r; ++col) {
    const double thc = th[col];
    double acc = 0.0;
    for (int i = t; i < nr; i += kLrWG) {
      const double d = cg[(size_t)col * nr + i] - thc * xg[(size_t)col * nr + i];
      acc = fma(d, d, acc);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kLrWG / 64; ++w) s += red[w];
    worst = fmax(worst, sqrt(s));
    __syncthreads();
  }
  if (t == 0) {
    const double top = th[0];
    const double rel = top > 0.0 ? worst / top : 0.0;
    rb[0] = rel;
    rb[1] = th[r - 1];
    rb[2] = th[l - 1];
    stat[1] = rel <= tol ? 1 : 0;
  }
}

// out[i nc + j] = sum_{t < r} Xr(i, t) Vr(j, t)
__global__ void __launch_bounds__(kLrWG) k_lr_out(const int *stat, const double *__restrict__ Xr,
                                                 const double *__restrict__ Vr, int nr, int nc,
                                                 int r, double *__restrict__ out) {
  if (!lr_live(stat)) return;
  const int64_t total = (int64_t)nr * nc;
  const gptr<const double> xg = gmem(Xr), vg = gmem(Vr);
  const gptr<double> og = gmem(out);
  for (int64_t e = (int64_t)blockIdx.x * kLrWG + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kLrWG) {
    const int64_t i = e / nc, j = e % nc;
    double v = 0.0;
    for (int tcol = 0; tcol < r; ++tcol)
      v = fma(xg[(size_t)tcol * nr + i], vg[(size_t)tcol * nc + j], v);
    og[e] = v;
  }
}

// bookkeeping of a finished call: iterations, and the count of calls of the
// truncated-SVD variant that reached the iteration limit unconverged
__global__ void k_lr_finish(int *stat, int iters, int count_unconverged) {
  if (threadIdx.x != 0 || !lr_live(stat)) return;
  stat[2] = iters;
  if (count_unconverged && stat[1] == 0) stat[3] += 1;
}

int grid_for(int64_t items, int cap) {
  const int64_t g = (items + kLrWG - 1) / kLrWG;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

LrArgs args_of(const LrBufs &L) {
  LrArgs a;
  a.nr = L.nr;
  a.nc = L.nc;
  a.l = L.l;
  a.stat = L.stat;
  a.Wp = L.Wp;
  a.R = L.R;
  a.part = L.part;
  a.E = L.E;
  a.th = L.th;
  return a;
}

// out (M x ncol) = op(C) X; step: what the last workgroup computes from the
// Gram matrix of out (kNone: no Gram matrix)
void lr_product(const LrBufs &L, bool tr, const double *C, const double *X, int ncol, double *out,
                int step, hipStream_t st) {
  const int M = tr ? L.nc : L.nr;
  const LrArgs a = args_of(L);
  const dim3 g(lr_slices(M), kLrSplit);
  if (tr)
    hipLaunchKernelGGL(k_lr_prod<true>, g, dim3(kLrWG), 0, st, a, C, X, ncol);
  else
    hipLaunchKernelGGL(k_lr_prod<false>, g, dim3(kLrWG), 0, st, a, C, X, ncol);
  hipLaunchKernelGGL(k_lr_reduce, dim3(lr_slices(M)), dim3(kLrWG), 0, st, a, M, ncol, out, step);
}

// Y (M x l) <- a basis of its range, the Cholesky factor of its shifted Gram
// matrix being in L.R on entry.  full: orthonormal to working
// precision (two more plain passes), as the Rayleigh-Ritz step needs;
// otherwise the shifted pass alone, which keeps the range and bounds the
// condition number by ~1 / sqrt(shift): enough between the products of the
// iteration, where only the range matters.
void lr_orth(const LrBufs &L, double *Y, int M, bool full, hipStream_t st) {
  const LrArgs a = args_of(L);
  const dim3 g(lr_slices(M)), b(kLrWG);
  if (full) {
    hipLaunchKernelGGL(k_lr_apply, g, b, 0, st, a, Y, M, (int)kChol);
    hipLaunchKernelGGL(k_lr_apply, g, b, 0, st, a, Y, M, (int)kChol);
  }
  hipLaunchKernelGGL(k_lr_apply, g, b, 0, st, a, Y, M, (int)kNone);
}

void lr_eig(const LrBufs &L, hipStream_t st) {
  hipLaunchKernelGGL(k_lr_eig, dim3(1), dim3(kEigWG), 0, st, L.stat, L.Wp, lr_slices(L.nc), L.l,
                     L.E, L.th);
}

}  // namespace

size_t lr_doubles(int nr, int nc, int r, int l) {
  auto up = [](size_t d) { return (d + 31) / 32 * 32; };
  const size_t ns = (size_t)lr_slices(std::max(nr, nc));
  return 3 * up((size_t)nr * l) + 2 * up((size_t)nc * l) + up((size_t)nr * r) +
         up((size_t)kLrSplit * std::max(nr, nc) * l) + up(ns * packed_len(l)) +
         2 * up((size_t)l * l) + up(l) + up(4) + up(8);
}

void lr_carve(LrBufs &L, double *base) {
  auto up = [](size_t d) { return (d + 31) / 32 * 32; };
  const size_t ns = (size_t)lr_slices(std::max(L.nr, L.nc));
  double *p = base;
  auto take = [&](size_t d) { double *q = p; p += up(d); return q; };
  L.Q = take((size_t)L.nr * L.l);
  L.Y = take((size_t)L.nr * L.l);
  L.XE = take((size_t)L.nr * L.l);
  L.Z = take((size_t)L.nc * L.l);
  L.ZE = take((size_t)L.nc * L.l);
  L.CV = take((size_t)L.nr * L.r);
  L.part = take((size_t)kLrSplit * std::max(L.nr, L.nc) * L.l);
  L.Wp = take(ns * packed_len(L.l));
  L.R = take((size_t)L.l * L.l);
  L.E = take((size_t)L.l * L.l);
  L.th = take(L.l);
  L.rb = take(4);
  L.stat = reinterpret_cast<int *>(take(8));
}

hipError_t lr_apply(const LrBufs &L, const Scal *sc, int maxit, int mode, int k, const double *pin,
                    double *zout, hipStream_t st) {
  hipLaunchKernelGGL(k_lr_begin, dim3(1), dim3(64), 0, st, sc, maxit, mode, k, L.stat);
  const int total = L.nc * L.l;
  const uint64_t key1 = (uint64_t)2 + ((uint64_t)(uint32_t)L.instance << 32);
  double *Z = L.Z, *ZE = L.ZE;
  hipLaunchKernelGGL(k_lr_omega, dim3(grid_for((total + 3) / 4, 1 << 20)), dim3(kLrWG), 0, st,
                     L.stat, Z, total, (uint64_t)L.seed, key1, (uint64_t)(k + 1));
  double *Q = L.Q, *Yn = L.Y;
  const int64_t outn = (int64_t)L.nr * L.nc;
  const int ritz_grid = grid_for(((int64_t)L.nr + L.nc) * L.l, 4096);
  // range finder C Omega; the Rayleigh-Ritz steps need an orthonormal Q (after
  // the randomized variant's last product, and before every residual check)
  int next_check = L.check;
  auto check_at = [&](int it) { return it == next_check || it == L.maxit; };
  lr_product(L, false, pin, Z, L.l, Q, kCholShift, st);
  lr_orth(L, Q, L.nr, L.rnd ? L.q == 0 : check_at(1), st);
  if (L.rnd) {
    for (int it = 0; it < L.q; ++it) {
      lr_product(L, true, pin, Q, L.l, Z, kNone, st);
      lr_product(L, false, pin, Z, L.l, Yn, kCholShift, st);
      lr_orth(L, Yn, L.nr, it + 1 == L.q, st);
      std::swap(Q, Yn);
    }
    lr_product(L, true, pin, Q, L.l, Z, kGram, st);     // Z = C^T Q = B^T
    lr_eig(L, st);                                      // eig of B B^T = Z^T Z
    hipLaunchKernelGGL(k_lr_ritz, dim3(ritz_grid), dim3(kLrWG), 0, st, L.stat, Q, Z, L.E, L.nr,
                       L.nc, L.l, L.XE, ZE);
    hipLaunchKernelGGL(k_lr_out, dim3(grid_for(outn, 8192)), dim3(kLrWG), 0, st, L.stat, L.XE, ZE,
                       L.nr, L.nc, L.r, zout);
    hipLaunchKernelGGL(k_lr_finish, dim3(1), dim3(64), 0, st, L.stat, L.q, 0);
    return hipGetLastError();
  }
  for (int it = 1; it <= L.maxit; ++it) {
    if (check_at(it)) {
      lr_product(L, true, pin, Q, L.l, Z, kGram, st);   // Z = C^T Q
      lr_eig(L, st);                                    // eig of Z^T Z
      hipLaunchKernelGGL(k_lr_ritz, dim3(ritz_grid), dim3(kLrWG), 0, st, L.stat, Q, Z, L.E, L.nr,
                         L.nc, L.l, L.XE, ZE);
      lr_product(L, false, pin, ZE, L.r, L.CV, kNone, st);       // C v_t
      hipLaunchKernelGGL(k_lr_resid, dim3(1), dim3(kLrWG), 0, st, L.stat, L.CV, L.XE, L.th, L.nr,
                         L.r, L.l, L.tol, L.rb);
      int h[2] = {0, 0};
      double rb[3] = {0.0, 0.0, 0.0};
      hipError_t e = hipMemcpyAsync(h, L.stat, sizeof h, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipMemcpyAsync(rb, L.rb, sizeof rb, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return e;
      if (h[0] == 0 || h[1] != 0 || it == L.maxit) {
        hipLaunchKernelGGL(k_lr_out, dim3(grid_for(outn, 8192)), dim3(kLrWG), 0, st, L.stat, L.XE,
                           ZE, L.nr, L.nc, L.r, zout);
        hipLaunchKernelGGL(k_lr_finish, dim3(1), dim3(64), 0, st, L.stat, it, 1);
        return hipGetLastError();
      }
      // next check: the residual falls by ~theta_l / theta_r per iteration
      int wait = 4;
      const double rho = rb[1] > 0.0 ? rb[2] / rb[1] : 1.0;
      if (rb[0] > 0.0 && rho > 0.0 && rho < 0.999) {
        const double need = std::log(L.tol / rb[0]) / std::log(rho);
        wait = (int)std::min(32.0, std::max(2.0, std::ceil(need)));
      }
      next_check = it + wait;
      // continue from the Ritz basis: Z E = C^T (Q E), columns ordered by theta
      std::swap(Z, ZE);
    } else {
      lr_product(L, true, pin, Q, L.l, Z, kNone, st);           // Z = C^T Q
    }
    lr_product(L, false, pin, Z, L.l, Yn, kCholShift, st);
    lr_orth(L, Yn, L.nr, check_at(it + 1), st);
    std::swap(Q, Yn);
  }
  return hipGetLastError();
}

}  // namespace sfk
