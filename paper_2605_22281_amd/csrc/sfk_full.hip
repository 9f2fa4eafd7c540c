// FLSQR and FLSMR with full orthogonalisation (the flexible Golub-Kahan
// process of Sec. 2.2, eq. (flsqr-relations), before any sketching): every
// new w is orthogonalised against all of W_k and every new z against all of
// P_k, so W_{k+1} and P_{k+1} have orthonormal columns and the projected
// problems are small and exact:
//   FLSQR (eq. (FLSQR)): y_k = argmin || beta e_1 - H_{k+1,k} y ||
//   FLSMR:               y_k = argmin || T_{k+1} (beta e_1 - H_{k+1,k} y) ||
// The orthogonalisation is classical Gram-Schmidt applied twice (one pass of
// dot products with all earlier vectors, one update, repeated once): equal to
// modified Gram-Schmidt in exact arithmetic, and the two passes keep the basis
// orthonormal to working precision, with every pass a parallel sweep over the
// stored basis (8 bytes per stored entry per pass) instead of k dependent
// steps.  The small problems are upper Hessenberg (H, and T H since T is upper
// triangular), updated by one Givens rotation per step.
#include <hip/hip_runtime.h>

#include "sfk_common.h"

namespace sfk {

constexpr int kFullWG = 256;
constexpr int kFullNB = 512;      // row blocks of the basis sweeps

__device__ __forceinline__ void rows_of(int len, int b, int &i0, int &i1) {
  i0 = (int)((long long)len * b / kFullNB);
  i1 = (int)((long long)len * (b + 1) / kFullNB);
}

// part[b * ldp + j] = sum over block b's rows of V[:, j] . w (j < ncols), and
// part[b * ldp + ncols] = w . w when with_self.  Waves take columns in turn.
__global__ void __launch_bounds__(kFullWG) k_f_dots(const double *__restrict__ V, int ld, int ncols,
                                                   const double *__restrict__ w, int len,
                                                   double *part, int ldp, int with_self) {
  extern __shared__ double ws[];
  int i0, i1;
  rows_of(len, blockIdx.x, i0, i1);
  const int nr = i1 - i0;
  for (int i = threadIdx.x; i < nr; i += kFullWG) ws[i] = w[i0 + i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nc = ncols + (with_self ? 1 : 0);
  const gptr<const double> Vg = gmem(V);
  for (int j = wv; j < nc; j += kFullWG / 64) {
    double s = 0.0;
    if (j < ncols) {
      const gptr<const double> col = Vg + (size_t)j * ld + i0;
      for (int i = lane; i < nr; i += 64) s += col[i] * ws[i];
    } else {
      for (int i = lane; i < nr; i += 64) s += ws[i] * ws[i];
    }
    s = wave_sum(s);
    if (lane == 0) part[(size_t)blockIdx.x * ldp + j] = s;
  }
}

// out[j] (+)= sum_b part[b * ldp + j], b in order (one workgroup per column)
__global__ void __launch_bounds__(kFullWG) k_f_reduce(const double *part, int ldp, double *out,
                                                     int accumulate) {
  __shared__ double lds_w[kMaxQ * (kFullWG / 64)];
  __shared__ double tot[kMaxQ];
  const int j = blockIdx.x;
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  for (int b = threadIdx.x; b < kFullNB; b += kFullWG) acc[0] += part[(size_t)b * ldp + j];
  block_sum<kFullWG>(acc, 1, lds_w, tot);
  if (threadIdx.x == 0) out[j] = accumulate ? out[j] + tot[0] : tot[0];
}

// w -= V[:, 0:ncols] h over block b's rows; norm partial of the result in
// npart[b] when npart is given
__global__ void __launch_bounds__(kFullWG) k_f_update(const double *__restrict__ V, int ld, int ncols,
                                                     const double *__restrict__ h, double *w,
                                                     int len, double *npart) {
  extern __shared__ double hs[];
  __shared__ double lds_w[kMaxQ * (kFullWG / 64)];
  __shared__ double tot[kMaxQ];
  for (int j = threadIdx.x; j < ncols; j += kFullWG) hs[j] = h[j];
  __syncthreads();
  int i0, i1;
  rows_of(len, blockIdx.x, i0, i1);
  const gptr<const double> Vg = gmem(V);
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kFullWG) {
    double v = w[i];
    for (int j = 0; j < ncols; ++j) v -= Vg[(size_t)j * ld + i] * hs[j];
    w[i] = v;
    acc[0] += v * v;
  }
  if (npart) {
    block_sum<kFullWG>(acc, 1, lds_w, tot);
    if (threadIdx.x == 0) npart[blockIdx.x] = tot[0];
  }
}

// The new unit vector: every block reduces the norm partials in the same
// order, writes out[:] = w / ||w|| for its rows; block 0 stores the
// coefficients coef[0:ncols] = h1 + h2 (the two passes) and coef[ncols] =
// ||w||.  pre: ||w|| before orthogonalisation (breakdown test), flag bit
// `bit` of sc->breakdown when the vector vanishes.
__global__ void __launch_bounds__(kFullWG) k_f_normalize(const double *w, int len,
                                                        const double *npart, double *out,
                                                        const double *h1, const double *h2,
                                                        int ncols, double *coef, double pre2,
                                                        const double *pre2p, Scal *sc, int bit,
                                                        int klim) {
  __shared__ double lds_w[kMaxQ * (kFullWG / 64)];
  __shared__ double tot[kMaxQ];
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  for (int b = threadIdx.x; b < kFullNB; b += kFullWG) acc[0] += npart[b];
  block_sum<kFullWG>(acc, 1, lds_w, tot);
  const double nrm = sqrt(tot[0]);
  const double pre = sqrt(pre2p ? *pre2p : pre2);
  const bool dead = nrm <= kBreakdownTol * pre || nrm == 0.0;
  const double sc_inv = dead ? 0.0 : 1.0 / nrm;
  int i0, i1;
  rows_of(len, blockIdx.x, i0, i1);
  for (int i = i0 + threadIdx.x; i < i1; i += kFullWG) out[i] = w[i] * sc_inv;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int j = 0; j < ncols; ++j) coef[j] = h1[j] + h2[j];
    coef[ncols] = dead ? 0.0 : nrm;
    // a vanished p_{k+1}: the basis cannot grow past k (klim); a vanished
    // w_{k+1} (happy breakdown) ends the run after the least squares of k
    if (dead) {
      atomicOr(&sc->breakdown, bit);
      if (klim >= 0) atomicMin(&sc->klimit, klim);
    }
  }
}

// Givens update of the projected problem after iteration k (one wave).
//   FLSQR: new column c = H[0:k+1, k-1]; FLSMR: c = T_{k+1} H[0:k+1, k-1].
// The k-1 earlier rotations act on c in order, a new rotation zeroes c[k];
// R gets column k-1, g (= Q^T rhs) entries k-1 and k; rho_k = |g[k]|.  Then
// y_k = R^{-1} g[0:k] (column-oriented back-substitution).
__global__ void __launch_bounds__(64) k_f_ls(Dev D, int k, double *gc, double *gs, double *gR,
                                            double *gg) {
  Scal *sc = D.sc;
  if (k > D.maxit || ld_flag(&sc->halt) != 0 || k > ld_flag(&sc->klimit)) return;
  __shared__ double c[1025];
  __shared__ double gy[1024];
  const int lane = threadIdx.x;
  const int ldh = D.maxit + 1, ldr = D.maxit;
  const double *hk = D.H + (size_t)(k - 1) * ldh;
  for (int i = lane; i <= k; i += 64) {
    double v;
    if (D.method == 2) {
      v = hk[i];
    } else {
      v = 0.0;
      for (int j = i; j <= k; ++j) v += D.T[(size_t)j * ldh + i] * hk[j];
    }
    c[i] = v;
  }
  __syncthreads();
  if (lane == 0) {
    for (int j = 0; j < k - 1; ++j) {       // rotation j acts on rows j, j + 1
      const double a = c[j], b = c[j + 1];
      c[j] = gc[j] * a + gs[j] * b;
      c[j + 1] = -gs[j] * a + gc[j] * b;
    }
    const double a = c[k - 1], b = c[k];
    double cs, sn, r;
    if (b == 0.0) { cs = 1.0; sn = 0.0; r = a; }
    else {
      r = hypot(a, b);
      cs = a / r;
      sn = b / r;
    }
    gc[k - 1] = cs;
    gs[k - 1] = sn;
    c[k - 1] = r;
    const double g0 = gg[k - 1];
    gg[k - 1] = cs * g0;
    gg[k] = -sn * g0;
    D.rho[k - 1] = fabs(gg[k]);
  }
  __syncthreads();
  double *Rc = gR + (size_t)(k - 1) * ldr;
  for (int i = lane; i < k; i += 64) Rc[i] = c[i];
  for (int i = lane; i < k; i += 64) gy[i] = gg[i];
  __syncthreads();
  // y = R^{-1} g[0:k]
  for (int j = k - 1; j >= 0; --j) {
    const double yj = gy[j] / gR[(size_t)j * ldr + j];
    __syncthreads();
    if (lane == 0) D.y[j] = yj;
    for (int i = lane; i < j; i += 64) gy[i] -= gR[(size_t)j * ldr + i] * yj;
    __syncthreads();
  }
  if (lane == 0) {
    sc->k_done = k;
    const double rho = fabs(gg[k]);
    if (sc->breakdown & 2) sc->halt = 1;          // w_{k+1} vanished: x_k is final
    if (sc->ttol > 0.0 && D.method == 2 && rho <= sc->ttol) { sc->stopped = 1; sc->halt = 1; }
    if (sc->tol > 0.0 && rho < sc->tol * sc->rhsnorm) { sc->stopped = 1; sc->halt = 1; }
  }
}

// y_j = R_j^{-1} g[0:j] for an earlier iterate (one wave)
__global__ void __launch_bounds__(64) k_f_backsub(Dev D, int jj, const double *gR, const double *gg,
                                                 double *yout) {
  __shared__ double gy[1024];
  const int lane = threadIdx.x, ldr = D.maxit;
  for (int i = lane; i < jj; i += 64) gy[i] = gg[i];
  __syncthreads();
  for (int j = jj - 1; j >= 0; --j) {
    const double yj = gy[j] / gR[(size_t)j * ldr + j];
    __syncthreads();
    if (lane == 0) yout[j] = yj;
    for (int i = lane; i < j; i += 64) gy[i] -= gR[(size_t)j * ldr + i] * yj;
    __syncthreads();
  }
}

// z_{k+1} = tau(p_{k+1}) into Z column k: identity, or the l1 reweighting with
// x_k = Z_k y_k assembled here (also kept in D.x)
__global__ void __launch_bounds__(kFullWG) k_f_tau(Dev D, int k, const double *Pf) {
  if (D.tau >= 2) return;   // the low-rank operators run as a stage of their own
  Scal *sc = D.sc;
  if (k > 0 && (ld_flag(&sc->halt) != 0 || k > ld_flag(&sc->klimit) || ld_flag(&sc->k_done) != k))
    return;
  extern __shared__ double ys[];
  for (int j = threadIdx.x; j < k; j += kFullWG) ys[j] = D.y[j];
  __syncthreads();
  const int n = D.n;
  const gptr<const double> Zg = gmem(D.Z);
  const double *p = Pf + (size_t)k * n;
  double *zo = D.Z + (size_t)k * n;
  const double eps2 = D.eps * D.eps;
  for (int i = blockIdx.x * kFullWG + threadIdx.x; i < n; i += gridDim.x * kFullWG) {
    if (D.tau == 1) {
      double xi = 0.0;
      for (int j = 0; j < k; ++j) xi += ys[j] * Zg[(size_t)j * n + i];
      D.x[i] = xi;
      zo[i] = sqrt(sqrt(xi * xi + eps2)) * p[i];
    } else {
      zo[i] = p[i];
    }
  }
}

// initial scalars: g[0] = beta (FLSQR) or beta t_11 (FLSMR); rhs norm; unit
// scale factors (the stored basis is normalised)
__global__ void k_f_init(Dev D, double *gg) {
  Scal *sc = D.sc;
  const int ldh = D.maxit + 1;
  const double g0 = D.method == 2 ? sc->beta : sc->beta * D.T[0];
  for (int j = threadIdx.x; j < D.maxit + 2; j += blockDim.x) { D.sigw[j] = 1.0; D.sigp[j] = 1.0; }
  if (threadIdx.x == 0) {
    gg[0] = g0;
    sc->rhsnorm = fabs(g0);
    (void)ldh;
  }
}

// w_1 = b / beta (beta from k_init_b)
__global__ void k_f_w1(Dev D, double *Wf) {
  const double inv = 1.0 / D.sc->beta;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < D.m; i += gridDim.x * blockDim.x)
    Wf[i] = D.b[i] * inv;
}

// ----------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------
void launch_spmv_core(const Dev &D, bool isa, int vw, const double *x, double *y, hipStream_t st);

// Orthonormalises w (length len) against V[:, 0:ncols] (leading dimension
// len) by two passes of classical Gram-Schmidt and stores the unit vector in
// V[:, ncols]; coef[0:ncols] = the projections, coef[ncols] = the norm.
// scratch: kFullNB * (ncols + 2) partials, then 2 (ncols + 1) doubles.
static void orthonormalise(double *V, int len, int ncols, double *w, double *coef, double *scratch,
                           Scal *sc, int bit, int klim, hipStream_t st) {
  const int ldp = ncols + 1;
  double *part = scratch;
  double *h1 = part + (size_t)kFullNB * (ncols + 2);
  double *h2 = h1 + (ncols + 1);
  const size_t rows_max = (size_t)len / kFullNB + 2;
  const size_t shd = sizeof(double) * rows_max;
  const size_t shh = sizeof(double) * (size_t)std::max(ncols, 1);
  // pass 1 (with ||w||^2 before orthogonalisation in h1[ncols])
  hipLaunchKernelGGL(k_f_dots, dim3(kFullNB), dim3(kFullWG), shd, st, V, len, ncols, w, len, part,
                     ldp, 1);
  hipLaunchKernelGGL(k_f_reduce, dim3(ncols + 1), dim3(kFullWG), 0, st, part, ldp, h1, 0);
  if (ncols > 0) {
    hipLaunchKernelGGL(k_f_update, dim3(kFullNB), dim3(kFullWG), shh, st, V, len, ncols, h1, w,
                       len, nullptr);
    hipLaunchKernelGGL(k_f_dots, dim3(kFullNB), dim3(kFullWG), shd, st, V, len, ncols, w, len,
                       part, ldp, 0);
    hipLaunchKernelGGL(k_f_reduce, dim3(ncols), dim3(kFullWG), 0, st, part, ldp, h2, 0);
  } else {
    hipMemsetAsync(h2, 0, sizeof(double), st);
  }
  // second update (or, without earlier vectors, a zero update) with the norm partials
  double *npart = part;     // pass-2 partials are consumed: reuse their space
  hipLaunchKernelGGL(k_f_update, dim3(kFullNB), dim3(kFullWG), shh, st, V, len, ncols, h2, w, len,
                     npart);
  hipLaunchKernelGGL(k_f_normalize, dim3(kFullNB), dim3(kFullWG), 0, st, w, len, npart,
                     V + (size_t)ncols * len, h1, h2, ncols, coef, 0.0, h1 + ncols, sc, bit, klim);
}

size_t full_scratch_doubles(int maxit) {
  return (size_t)kFullNB * (maxit + 3) + 2 * (size_t)(maxit + 2) + 64;
}

// Algorithm start of FLSQR / FLSMR after k_init_b: w_1, p_1 (t_11), z_1, g
void launch_full_init(const Dev &D, int vwB, hipStream_t st) {
  hipLaunchKernelGGL(k_f_w1, dim3((D.m + 255) / 256), dim3(256), 0, st, D, D.Wf);
  double *zr = D.zraw;
  launch_spmv_core(D, false, vwB, D.Wf, zr, st);
  const int ldh = D.maxit + 1;
  orthonormalise(D.Pf, D.n, 0, zr, D.T, D.fscr, D.sc, 1, 0, st);
  (void)ldh;
  hipLaunchKernelGGL(k_f_init, dim3(1), dim3(256), 0, st, D, D.gg);
  hipLaunchKernelGGL(k_f_tau, dim3(std::min((D.n + kFullWG - 1) / kFullWG, 2048)), dim3(kFullWG),
                     sizeof(double), st, D, 0, D.Pf);
}

// One iteration k of FLSQR / FLSMR: w = A z_k, full orthogonalisation (H
// column k), z = B w_{k+1}, full orthogonalisation (T column k + 1), Givens
// update and y_k, then z_{k+1} = tau(p_{k+1}).  stage(i) brackets each part
// for the optional stage timing (0 A, 1 w-side, 4 B, 5 z-side, 3 LS).
void launch_full_iteration(const Dev &D, int k, int vwA, int vwB, hipStream_t st,
                           void (*mark)(void *, int, int), void *ctx) {
  const int ldh = D.maxit + 1;
  double *wr = D.wraw, *zr = D.zraw;
  if (mark) mark(ctx, 0, 1);
  launch_spmv_core(D, true, vwA, D.Z + (size_t)(k - 1) * D.n, wr, st);
  if (mark) mark(ctx, 0, 0);
  if (mark) mark(ctx, 1, 1);
  orthonormalise(D.Wf, D.m, k, wr, D.H + (size_t)(k - 1) * ldh, D.fscr, D.sc, 2, -1, st);
  if (mark) mark(ctx, 1, 0);
  if (mark) mark(ctx, 4, 1);
  launch_spmv_core(D, false, vwB, D.Wf + (size_t)k * D.m, zr, st);
  if (mark) mark(ctx, 4, 0);
  if (mark) mark(ctx, 5, 1);
  orthonormalise(D.Pf, D.n, k, zr, D.T + (size_t)k * ldh, D.fscr, D.sc, 1, k, st);
  if (mark) mark(ctx, 5, 0);
  if (mark) mark(ctx, 3, 1);
  hipLaunchKernelGGL(k_f_ls, dim3(1), dim3(64), 0, st, D, k, D.gc, D.gs, D.gR, D.gg);
  if (mark) mark(ctx, 3, 0);
  if (mark) mark(ctx, 5, 1);
  hipLaunchKernelGGL(k_f_tau, dim3(std::min((D.n + kFullWG - 1) / kFullWG, 2048)), dim3(kFullWG),
                     sizeof(double) * (size_t)k, st, D, k, D.Pf);
  if (mark) mark(ctx, 5, 0);
}

void launch_full_backsub(const Dev &D, int j, double *yout, hipStream_t st) {
  hipLaunchKernelGGL(k_f_backsub, dim3(1), dim3(64), 0, st, D, j, D.gR, D.gg, yout);
}

}  // namespace sfk
