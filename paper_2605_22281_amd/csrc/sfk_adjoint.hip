// Reverse-mode derivative (adjoint) of the sFLSQR iterate x_K with respect to
// the right-hand side b and the reweighting parameter eps of the flexible
// operator z_k = (x_{k-1}^2 + eps^2)^(1/4) p_k (eq. (modbasis), the l1 IRLS
// weights of Sec. 1.2).  Given xbar = dL/dx_K it returns bbar = dL/db and
// epsbar = dL/deps for the map defined by K steps of eq. (FGK) with window
// ell and the sketched least-squares problems of eq. (sFLSQR), B = A^T.
//
// The reverse sweep visits k = K .. 1 and undoes, in reverse order, the
// steps of iteration k: x_k = Z_k y_k; y_k = argmin ||S b - C_k y|| with C_k =
// S A Z_k; the normalisation w_{k+1} = v' / h_{k+1,k}; the w-side Gram-Schmidt
// v' = v - sum_j h_jk w_j; v = A z_k and c_k = S v; z_k = tau(p_k); the
// normalisation p_k = u / t_kk; the z-side Gram-Schmidt u = z - sum_j t_jk p_j
// with z = B w_k.  The rules are those of the chain rule for each operation:
// for y = argmin ||s - C y|| with r = s - C y and u = (C^T C)^{-1} ybar,
// sbar += C u and Cbar += r u^T - (C u) y^T; for a unit vector q = v / ||v||,
// vbar = (qbar - q <q, qbar>) / ||v||; for v_new = v - h w with h = <w, v>,
// hbar = -<w, vbar_new>, wbar += -h vbar_new + hbar v, vbar = vbar_new + hbar w.
//
// What the sweep needs of the forward run: Z, H, T, the sketched columns and
// the R factor and rotated right-hand side of the least-squares state are
// kept by the forward anyway; the w_j are regenerated segment by segment from
// checkpoints of the w window taken every `tape` iterations (the forward keeps
// only a window), through eq. (FGK): w_{j+1} = (A z_j - sum_i h_ij w_i) /
// h_{j+1,j}; p_j = z_j / (x_{j-1}^2 + eps^2)^(1/4) and x_{j-1} = Z_{j-1} y_{j-1}.
#include <hip/hip_runtime.h>

#include "sfk_adjoint_layout.h"
#include "sfk_common.h"

namespace sfk {

constexpr int kAdjWG = 256;
constexpr int kAdjNB = kAdjBlocks;

__device__ __forceinline__ void adj_rows(int len, int b, int &i0, int &i1) {
  i0 = (int)((long long)len * b / kAdjNB);
  i1 = (int)((long long)len * (b + 1) / kAdjNB);
}

// part[b] = sum over block b's rows of a[i] * b[i]
__global__ void __launch_bounds__(kAdjWG) k_a_dot(const double *a, const double *b, int len,
                                                 double *part) {
  __shared__ double lds_w[kMaxQ * (kAdjWG / 64)];
  __shared__ double tot[kMaxQ];
  int i0, i1;
  adj_rows(len, blockIdx.x, i0, i1);
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kAdjWG) acc[0] += a[i] * b[i];
  block_sum<kAdjWG>(acc, 1, lds_w, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot[0];
}

// out = sum_b part[b] in block order
__global__ void __launch_bounds__(kAdjWG) k_a_sum(const double *part, int np, double *out) {
  __shared__ double lds_w[kMaxQ * (kAdjWG / 64)];
  __shared__ double tot[kMaxQ];
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  for (int b = threadIdx.x; b < np; b += kAdjWG) acc[0] += part[b];
  block_sum<kAdjWG>(acc, 1, lds_w, tot);
  if (threadIdx.x == 0) *out = tot[0];
}

// y = alpha y + beta x, the coefficients from device scalars:
// alpha = (a0 + a1 sa[0]) / sda[0], beta = (b0 + b1 sb[0]) / sdb[0] (a NULL
// scalar pointer drops its term or divisor); x may be NULL (beta unused)
__global__ void k_a_comb(double *y, const double *x, int len, double a0, double a1,
                         const double *sa, const double *sda, double b0, double b1,
                         const double *sb, const double *sdb) {
  double al = a0 + (sa ? a1 * sa[0] : 0.0);
  if (sda) al /= sda[0];
  double be = b0 + (sb ? b1 * sb[0] : 0.0);
  if (sdb) be /= sdb[0];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x)
    y[i] = al * y[i] + (x ? be * x[i] : 0.0);
}

// Zbar[:, j] += x * y[j], j < k (rank-one update of the basis adjoints)
__global__ void k_a_rank1(double *Zb, int ld, int k, const double *x, const double *y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ld; i += gridDim.x * blockDim.x) {
    const double xi = x[i];
    for (int j = 0; j < k; ++j) Zb[(size_t)j * ld + i] += xi * y[j];
  }
}

// ybar_j = sigp_{j+1} <z~_{j+1}, xbar> from the column partials (one block per j)
__global__ void k_a_ybar(const double *part, int ldp, const double *sigp, double *ybar) {
  __shared__ double lds_w[kMaxQ * (kAdjWG / 64)];
  __shared__ double tot[kMaxQ];
  const int j = blockIdx.x;
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  for (int b = threadIdx.x; b < kAdjNB; b += kAdjWG) acc[0] += part[(size_t)b * ldp + j];
  block_sum<kAdjWG>(acc, 1, lds_w, tot);
  if (threadIdx.x == 0) ybar[j] = sigp[j + 1] * tot[0];
}

// part[b * ldp + j] = sum over block b's rows of Z~[:, j] * x (j < k)
__global__ void __launch_bounds__(kAdjWG) k_a_coldots(const double *Z, int ld, int k,
                                                     const double *x, double *part, int ldp) {
  int i0, i1;
  adj_rows(ld, blockIdx.x, i0, i1);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = wv; j < k; j += kAdjWG / 64) {
    const double *col = Z + (size_t)j * ld;
    double s = 0.0;
    for (int i = i0 + lane; i < i1; i += 64) s += col[i] * x[i];
    s = wave_sum(s);
    if (lane == 0) part[(size_t)blockIdx.x * ldp + j] = s;
  }
}

// Adjoint of the small problem of step k (one workgroup): with y = y_k,
// C = C_k (s x k), R the leading k x k block of the R factor:
// g = R^{-T} ybar, u = R^{-1} g, q = C u, r = s_b - C y;
// Cbar[:, j] += r u_j - q y_j (j < k), sbar += q.
__global__ void __launch_bounds__(kAdjWG) k_a_ls(Dev D, int k, const double *y, const double *ybar,
                                                double *Cbar, double *sbar) {
  __shared__ double g[1024];
  __shared__ double u[1024];
  const int s = D.s, ldr = D.maxit;
  const double *R = D.R;
  for (int j = threadIdx.x; j < k; j += kAdjWG) g[j] = ybar[j];
  __syncthreads();
  // R^T g' = ybar: forward substitution, row j of R^T is column j of R
  for (int j = 0; j < k; ++j) {
    if (threadIdx.x == 0) g[j] /= R[(size_t)j * ldr + j];
    __syncthreads();
    const double gj = g[j];
    for (int i = j + 1 + threadIdx.x; i < k; i += kAdjWG) g[i] -= R[(size_t)i * ldr + j] * gj;
    __syncthreads();
  }
  for (int j = threadIdx.x; j < k; j += kAdjWG) u[j] = g[j];
  __syncthreads();
  // R u = g: back substitution
  for (int j = k - 1; j >= 0; --j) {
    if (threadIdx.x == 0) u[j] /= R[(size_t)j * ldr + j];
    __syncthreads();
    const double uj = u[j];
    for (int i = threadIdx.x; i < j; i += kAdjWG) u[i] -= R[(size_t)j * ldr + i] * uj;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < s; i += kAdjWG) {
    double qi = 0.0, ri = D.skrhs[i];
    for (int j = 0; j < k; ++j) {
      const double c = D.SK[(size_t)j * s + i];
      qi += c * u[j];
      ri -= c * y[j];
    }
    for (int j = 0; j < k; ++j) Cbar[(size_t)j * s + i] += ri * u[j] - qi * y[j];
    sbar[i] += qi;
  }
}

// v += S^T c for the instance's sketch of m-vectors (sparse-sign: the zeta
// codes of column i; SRHT: (1 / sqrt(s)) D_i sum_r (-1)^{popcount(row_r & i)} c_r)
__global__ void k_a_sketch_t(Dev D, const double *c, double *v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.d_sk) return;
  double acc = 0.0;
  if (D.sketch == 0) {
    for (int q = 0; q < D.zeta; ++q) {
      const int code = D.sk_code[(size_t)i * D.zeta + q];
      const double cv = c[code >> 1];
      acc += (code & 1) ? -cv : cv;
    }
    acc *= D.sk_scale;
  } else if (D.sketch == 1) {
    for (int r = 0; r < D.s; ++r) {
      const double cv = c[r];
      acc += (__popc((unsigned)(D.srht_rows[r] & i)) & 1) ? -cv : cv;
    }
    const bool neg = (D.srht_d[i >> 6] >> (i & 63)) & 1ull;
    acc *= neg ? -D.sk_scale : D.sk_scale;
  } else {
    acc = c[i];
  }
  v[i] += acc;
}

// x = Z_k y (x_k, or x_{k-1} with the first k - 1 columns)
__global__ void k_a_x(Dev D, int k, const double *y, double *x) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < D.n; i += gridDim.x * blockDim.x) {
    double xi = 0.0;
    for (int j = 0; j < k; ++j) xi += D.sigp[j + 1] * y[j] * D.Z[(size_t)j * D.n + i];
    x[i] = xi;
  }
}

// z_k = sigp_k z~_k and p_k = z_k / d(x_{k-1}) (identity: p_k = z_k)
__global__ void k_a_zp(Dev D, int k, const double *x, double *z, double *p) {
  const double sg = D.sigp[k];
  const double eps2 = D.eps * D.eps;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < D.n; i += gridDim.x * blockDim.x) {
    const double zi = sg * D.Z[(size_t)(k - 1) * D.n + i];
    z[i] = zi;
    p[i] = D.tau == 1 ? zi / sqrt(sqrt(x[i] * x[i] + eps2)) : zi;
  }
}

// Adjoint of z_k = d(x_{k-1}, eps) * p_k: pbar += d zbar; with the
// reweighting xbar_{k-1} += (p zbar) x d / (2 q) and eps partials
// (p zbar) eps d / (2 q), q = x^2 + eps^2, d = q^(1/4)
__global__ void __launch_bounds__(kAdjWG) k_a_tau(Dev D, const double *x, const double *p,
                                                 const double *zbar, double *pbar, double *xbar,
                                                 double *epart) {
  __shared__ double lds_w[kMaxQ * (kAdjWG / 64)];
  __shared__ double tot[kMaxQ];
  int i0, i1;
  adj_rows(D.n, blockIdx.x, i0, i1);
  const double eps = D.eps, eps2 = eps * eps;
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kAdjWG) {
    if (D.tau == 1) {
      const double q = x[i] * x[i] + eps2, d = sqrt(sqrt(q));
      const double db = p[i] * zbar[i];
      pbar[i] += d * zbar[i];
      const double f = db * d / (2.0 * q);
      xbar[i] += f * x[i];
      acc[0] += f * eps;
    } else {
      pbar[i] += zbar[i];
    }
  }
  block_sum<kAdjWG>(acc, 1, lds_w, tot);
  if (threadIdx.x == 0) epart[blockIdx.x] = tot[0];
}

// w_j of the checkpoint window: the ring vector times its scale
__global__ void k_a_unit(const double *src, const double *scale, int len, double *out) {
  const double sc = scale[0];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x)
    out[i] = src[i] * sc;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void launch_spmv_core(const Dev &D, bool isa, int vw, const double *x, double *y, hipStream_t st);
void launch_backsub(const Dev &D, int j, double *yout, hipStream_t st);

// checkpoint of the w window after iteration k: w_{k-ell} .. w_{k+1} (unit),
// slot (j - (k - ell)) of the checkpoint, zero for j < 1
void launch_checkpoint_w(const Dev &D, int k, double *ck, hipStream_t st) {
  const int m = D.m;
  for (int q = 0; q < D.ell + 2; ++q) {
    const int j = k - D.ell + q;
    double *dst = ck + (size_t)q * m;
    if (j < 1) continue;
    const double *src = D.W + (size_t)(j % (D.ell + 2)) * m;
    hipLaunchKernelGGL(k_a_unit, dim3((m + 255) / 256), dim3(256), 0, st, src, D.sigw + j, m, dst);
  }
}

size_t adjoint_checkpoint_doubles(int maxit, int tape, int ell, int m) {
  if (tape <= 0) return 1;
  return (size_t)(maxit / tape + 1) * (ell + 2) * m;
}

namespace {
// Vector helpers of the sweep (one stream; every reduction in fixed order).
struct Ops {
  hipStream_t st;
  double *part;                   // kAdjNB partials
  int grid(int len) const { return std::max(1, std::min((len + 255) / 256, 4096)); }
  void dot(const double *a, const double *b, int len, double *out) const {
    hipLaunchKernelGGL(k_a_dot, dim3(kAdjNB), dim3(kAdjWG), 0, st, a, b, len, part);
    hipLaunchKernelGGL(k_a_sum, dim3(1), dim3(kAdjWG), 0, st, part, kAdjNB, out);
  }
  // y += mult * coef[0] * x (y += mult * x without coef)
  void axpy(double *y, const double *x, int len, double mult, const double *coef) const {
    hipLaunchKernelGGL(k_a_comb, dim3(grid(len)), dim3(256), 0, st, y, x, len, 1.0, 0.0,
                       (const double *)nullptr, (const double *)nullptr, coef ? 0.0 : mult,
                       coef ? mult : 0.0, coef, (const double *)nullptr);
  }
  // y = x * coef[0] (or x / coef[0] with divide)
  void scaled(double *y, const double *x, int len, const double *coef, bool divide) const {
    hipLaunchKernelGGL(k_a_comb, dim3(grid(len)), dim3(256), 0, st, y, x, len, 0.0, 0.0,
                       (const double *)nullptr, (const double *)nullptr, divide ? 1.0 : 0.0,
                       divide ? 0.0 : 1.0, divide ? nullptr : coef, divide ? coef : nullptr);
  }
  void zero(double *y, int len) const {
    hipLaunchKernelGGL(k_a_comb, dim3(grid(len)), dim3(256), 0, st, y, (const double *)nullptr, len,
                       0.0, 0.0, (const double *)nullptr, (const double *)nullptr, 0.0, 0.0,
                       (const double *)nullptr, (const double *)nullptr);
  }
  void copy(double *y, const double *x, int len) const {
    hipLaunchKernelGGL(k_a_comb, dim3(grid(len)), dim3(256), 0, st, y, x, len, 0.0, 0.0,
                       (const double *)nullptr, (const double *)nullptr, 1.0, 0.0,
                       (const double *)nullptr, (const double *)nullptr);
  }
  // qbar <- (qbar - q <q, qbar>) / nrm: the adjoint of q = v / ||v|| (nrm = ||v||)
  void unit_adjoint(double *qbar, const double *q, int len, const double *nrm, double *t) const {
    dot(q, qbar, len, t);
    hipLaunchKernelGGL(k_a_comb, dim3(grid(len)), dim3(256), 0, st, qbar, q, len, 1.0, 0.0,
                       (const double *)nullptr, nrm, 0.0, -1.0, (const double *)t, nrm);
  }
};
}  // namespace

// The sweep.  ck: the forward's checkpoints of the w window (slot q of
// checkpoint a / tape holds w_{a - ell + q}).  xbar_in: dL/dx_K (library
// order); bbar: dL/db; epsbar_host: dL/deps.
void run_adjoint(const Dev &D, int K, int tape, const double *ck, const double *xbar_in,
                 double *bbar, double *eacc_host, const AdjBufs &B, hipStream_t st) {
  const int m = D.m, n = D.n, s = D.s, ell = D.ell, ldh = D.maxit + 1, ldy = D.maxit;
  const Ops op{st, B.part};
  double *t0 = B.scal, *t1 = B.scal + 1;
  const int gm = op.grid(m), gn = op.grid(n);
  (void)gm;
  // y_j for every j, the accumulators
  for (int j = 1; j <= K; ++j) launch_backsub(D, j, B.Y + (size_t)(j - 1) * ldy, st);
  op.zero(B.Wbar, (ell + 2) * m);
  op.zero(B.Pbar, (ell + 1) * n);
  op.zero(B.Zbar, n * K);
  op.zero(B.Cbar, s * K);
  op.zero(B.sbar, s);
  op.zero(B.xnew, n);
  op.copy(B.xbar, xbar_in, n);
  auto wbar = [&](int j) { return B.Wbar + (size_t)(j % (ell + 2)) * m; };
  auto pbar = [&](int j) { return B.Pbar + (size_t)(j % (ell + 1)) * n; };
  const int nseg = (K + tape - 1) / tape;
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int a = sg * tape, kend = std::min(a + tape, K);
    const int w0 = a - ell;                       // Wseg slot 0 holds w_{a - ell}
    auto wseg = [&](int j) { return B.Wseg + (size_t)(j - w0) * m; };
    const int p0 = a + 1 - ell;                   // Pseg slot 0 holds p_{a + 1 - ell}
    auto pseg = [&](int j) { return B.Pseg + (size_t)(j - p0) * n; };
    auto xseg = [&](int j) { return B.Xseg + (size_t)(j - (a + 1)) * n; };   // x_{j-1}
    // the checkpoint window, then w_{a+2} .. w_{kend+1} by eq. (FGK)
    for (int q = 0; q < ell + 2; ++q)
      if (a - ell + q >= 1)
        op.copy(wseg(a - ell + q), ck + ((size_t)sg * (ell + 2) + q) * m, m);
    for (int j = a + 1; j <= kend; ++j) {
      // x_{j-1}, z_j and p_j
      if (j > 1) hipLaunchKernelGGL(k_a_x, dim3(gn), dim3(256), 0, st, D, j - 1,
                                    B.Y + (size_t)(j - 2) * ldy, xseg(j));
      else op.zero(xseg(j), n);
      hipLaunchKernelGGL(k_a_zp, dim3(gn), dim3(256), 0, st, D, j, xseg(j), B.zk, pseg(j));
      launch_spmv_core(D, true, D.vwA, B.zk, B.tmpm, st);
      for (int i = std::max(1, j - ell); i <= j; ++i)
        op.axpy(B.tmpm, wseg(i), m, -1.0, D.H + (size_t)(j - 1) * ldh + (i - 1));
      op.scaled(wseg(j + 1), B.tmpm, m, D.H + (size_t)(j - 1) * ldh + j, true);
    }
    // p_j of the window before the segment
    for (int j = std::max(1, p0); j <= a; ++j) {
      if (j > 1) hipLaunchKernelGGL(k_a_x, dim3(gn), dim3(256), 0, st, D, j - 1,
                                    B.Y + (size_t)(j - 2) * ldy, B.tmpn);
      else op.zero(B.tmpn, n);
      hipLaunchKernelGGL(k_a_zp, dim3(gn), dim3(256), 0, st, D, j, B.tmpn, B.zk, pseg(j));
    }
    for (int k = kend; k > a; --k) {
      const double *yk = B.Y + (size_t)(k - 1) * ldy;
      // x_k = Z_k y_k: ybar_k and the basis adjoints
      hipLaunchKernelGGL(k_a_coldots, dim3(kAdjNB), dim3(kAdjWG), 0, st, D.Z, n, k, B.xbar, B.cpart,
                         k);
      hipLaunchKernelGGL(k_a_ybar, dim3(k), dim3(kAdjWG), 0, st, B.cpart, k, D.sigp, B.ybar);
      hipLaunchKernelGGL(k_a_rank1, dim3(gn), dim3(256), 0, st, B.Zbar, n, k, B.xbar, yk);
      // the small sketched problem
      hipLaunchKernelGGL(k_a_ls, dim3(1), dim3(kAdjWG), 0, st, D, k, yk, B.ybar, B.Cbar, B.sbar);
      // w_{k+1} = v' / h_{k+1,k}
      const double *hk1 = D.H + (size_t)(k - 1) * ldh + k;
      op.copy(B.vbar, wbar(k + 1), m);
      op.zero(wbar(k + 1), m);
      op.unit_adjoint(B.vbar, wseg(k + 1), m, hk1, t0);
      // w-side Gram-Schmidt, j = k .. max(1, k - ell)
      op.scaled(B.vint, wseg(k + 1), m, hk1, false);
      for (int j = k; j >= std::max(1, k - ell); --j) {
        const double *hj = D.H + (size_t)(k - 1) * ldh + (j - 1);
        op.dot(wseg(j), B.vbar, m, t1);
        op.axpy(wbar(j), B.vbar, m, -1.0, hj);
        op.axpy(B.vint, wseg(j), m, 1.0, hj);
        op.axpy(B.vbar, wseg(j), m, -1.0, t1);
        op.axpy(wbar(j), B.vint, m, -1.0, t1);
      }
      // c_k = S v and v = A z_k
      hipLaunchKernelGGL(k_a_sketch_t, dim3((m + 255) / 256), dim3(256), 0, st, D,
                         B.Cbar + (size_t)(k - 1) * s, B.vbar);
      launch_spmv_core(D, false, D.vwB, B.vbar, B.zbar, st);
      op.axpy(B.zbar, B.Zbar + (size_t)(k - 1) * n, n, 1.0, nullptr);
      // z_k = tau(p_k)
      hipLaunchKernelGGL(k_a_tau, dim3(kAdjNB), dim3(kAdjWG), 0, st, D, xseg(k), pseg(k), B.zbar,
                         pbar(k), B.xnew, B.epart);
      hipLaunchKernelGGL(k_a_sum, dim3(1), dim3(kAdjWG), 0, st, B.epart, kAdjNB, B.eacc + (k - 1));
      // p_k = u / t_kk
      const double *tkk = D.T + (size_t)(k - 1) * ldh + (k - 1);
      op.copy(B.ubar, pbar(k), n);
      op.zero(pbar(k), n);
      op.unit_adjoint(B.ubar, pseg(k), n, tkk, t0);
      // z-side Gram-Schmidt, j = k - 1 .. max(1, k - ell)
      op.scaled(B.zint, pseg(k), n, tkk, false);
      for (int j = k - 1; j >= std::max(1, k - ell); --j) {
        const double *tj = D.T + (size_t)(k - 1) * ldh + (j - 1);
        op.dot(pseg(j), B.ubar, n, t1);
        op.axpy(pbar(j), B.ubar, n, -1.0, tj);
        op.axpy(B.zint, pseg(j), n, 1.0, tj);
        op.axpy(B.ubar, pseg(j), n, -1.0, t1);
        op.axpy(pbar(j), B.zint, n, -1.0, t1);
      }
      // z = B w_k (B = A^T): wbar_k += A ubar
      launch_spmv_core(D, true, D.vwA, B.ubar, B.tmpm, st);
      op.axpy(wbar(k), B.tmpm, m, 1.0, nullptr);
      // x_{k-1}: its adjoint is what tau left in xnew
      op.copy(B.xbar, B.xnew, n);
      op.zero(B.xnew, n);
    }
  }
  // w_1 = b / beta and s_b = S b
  op.copy(bbar, wbar(1), m);
  hipLaunchKernelGGL(k_a_unit, dim3((m + 255) / 256), dim3(256), 0, st, D.b, D.sigw + 1, m, B.tmpm);
  const double *beta = reinterpret_cast<const double *>(D.sc);   // Scal::beta, the first field
  op.unit_adjoint(bbar, B.tmpm, m, beta, t0);
  hipLaunchKernelGGL(k_a_sketch_t, dim3((m + 255) / 256), dim3(256), 0, st, D, B.sbar, bbar);
  hipMemcpyAsync(eacc_host, B.eacc, sizeof(double) * K, hipMemcpyDeviceToHost, st);
}

}  // namespace sfk
