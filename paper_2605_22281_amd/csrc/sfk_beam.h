// Matrix-free parallel-beam projector and back-projectors (device functions),
// the operators of the CT workloads computed on the fly instead of read from
// a stored matrix.
//
// Geometry: an N x N image of unit pixels on [-N/2, N/2]^2, row-major (row =
// y index); nz independent slices (parallel beam rotating about z: detector
// row z sees slice z); n_angles directions u_a = (cos_a, sin_a) given by the
// caller; n_det unit bins centred at t_d = d - (n_det - 1)/2.  Ray (z, a, d)
// is the line {t_d u_a + lambda v_a}, v_a = (-sin_a, cos_a); its index is
// (z n_angles + a) n_det + d, pixel (z, row, col) has index z N^2 + row N + col.
//
// The forward projection is exact (Siddon): the ray's parameter interval
// inside the square is cut at every crossing with a grid line, each piece
// belongs to the pixel holding its midpoint and contributes its length;
// pieces of length <= 1e-9 are dropped.  The crossing parameters are
// (grid - origin) / direction with the same operations as the host generator
// of the explicit matrices, so the entries agree with them.  The exact
// back-projection (the transpose) visits, for each pixel and angle, the rays
// whose line meets the pixel and recomputes the same piece; the unmatched
// back-projector interpolates linearly between the two nearest bins.
#pragma once

#include "sfk_dev.h"

namespace sfk {

struct BeamRay {
  double ox, oy, vx, vy, lmin, lmax;
  bool okx, oky, valid;
};

__device__ __forceinline__ BeamRay beam_ray(const Dev &D, int a, int d) {
#pragma clang fp contract(off)
  BeamRay R;
  const int N = D.bN;
  const double half = 0.5 * N;
  const double ux = D.bCos[a], uy = D.bSin[a];
  R.vx = -uy;
  R.vy = ux;
  const double t = (double)d - (D.bNd - 1) / 2.0;
  R.ox = t * ux;
  R.oy = t * uy;
  const double big = 4.0 * N;
  R.okx = fabs(R.vx) > 1e-15;
  R.oky = fabs(R.vy) > 1e-15;
  double lxmin = -big, lxmax = big, lymin = -big, lymax = big;
  if (R.okx) {
    const double l0 = (-half - R.ox) / R.vx, l1 = (half - R.ox) / R.vx;
    lxmin = fmin(l0, l1);
    lxmax = fmax(l0, l1);
  }
  if (R.oky) {
    const double l0 = (-half - R.oy) / R.vy, l1 = (half - R.oy) / R.vy;
    lymin = fmin(l0, l1);
    lymax = fmax(l0, l1);
  }
  const bool inx = R.okx || (R.ox >= -half && R.ox <= half);
  const bool iny = R.oky || (R.oy >= -half && R.oy <= half);
  R.lmin = fmax(lxmin, lymin);
  R.lmax = fmin(lxmax, lymax);
  R.valid = inx && iny && (R.lmax > R.lmin);
  return R;
}

// crossing parameters of one family of grid lines, in increasing lambda:
// entry k is grid line i = k (direction component > 0) or i = N - k
struct BeamLines {
  double o, v, half;
  int N;
  bool pos;
  __device__ __forceinline__ double lam(int k) const {
#pragma clang fp contract(off)
    const int i = pos ? k : N - k;
    return ((double)i - half - o) / v;
  }
  // first k in [0, N] with lam(k) >= a (N + 1 if none)
  __device__ __forceinline__ int first_at_least(double a) const {
#pragma clang fp contract(off)
    // lam(k) >= a  <=>  i >= o + a v + half (pos) or i <= o + a v + half
    const double q = o + a * v + half;
    int k = pos ? (int)ceil(q) : N - (int)floor(q);
    k = max(0, min(N + 1, k));
    while (k > 0 && lam(k - 1) >= a) --k;
    while (k <= N && lam(k) < a) ++k;
    return k;
  }
};

// Sum of len * x[pixel] over the pieces of ray (a, d) of slice z whose start
// lies in [lmin + (lmax - lmin) g / G, lmin + (lmax - lmin) (g + 1) / G): the
// share of lane g of a group of G lanes.
__device__ __forceinline__ double beam_ray_part(const Dev &D, const BeamRay &R, const double *x,
                                                int z, int g, int G) {
#pragma clang fp contract(off)
  if (!R.valid) return 0.0;
  const int N = D.bN;
  const double half = 0.5 * N;
  const double span = R.lmax - R.lmin;
  const double a0 = g == 0 ? R.lmin : R.lmin + span * g / G;
  const double a1 = g == G - 1 ? R.lmax : R.lmin + span * (g + 1) / G;
  const BeamLines X{R.ox, R.vx, half, N, R.vx > 0};
  const BeamLines Y{R.oy, R.vy, half, N, R.vy > 0};
  const double INF = 1e300;
  int kx = N + 1, ky = N + 1, kxe = -1, kye = -1;
  // the crossings inside [lmin, lmax]: k in [first >= lmin, last <= lmax]
  if (R.okx) {
    kx = X.first_at_least(R.lmin);
    kxe = X.first_at_least(R.lmax);
    if (kxe <= N && X.lam(kxe) == R.lmax) ++kxe;   // lmax itself is inside
  }
  if (R.oky) {
    ky = Y.first_at_least(R.lmin);
    kye = Y.first_at_least(R.lmax);
    if (kye <= N && Y.lam(kye) == R.lmax) ++kye;
  }
  // breakpoints of this lane start at the first one >= a0
  if (g > 0) {
    if (R.okx) kx = max(kx, X.first_at_least(a0));
    if (R.oky) ky = max(ky, Y.first_at_least(a0));
  }
  double cx = (R.okx && kx < kxe) ? X.lam(kx) : INF;
  double cy = (R.oky && ky < kye) ? Y.lam(ky) : INF;
  bool lmax_left = true;
  double beta;
  if (g == 0) {
    beta = R.lmin;
  } else {
    // consume the first breakpoint >= a0
    if (cx <= cy && cx <= R.lmax) { beta = cx; ++kx; cx = (kx < kxe) ? X.lam(kx) : INF; }
    else if (cy <= R.lmax) { beta = cy; ++ky; cy = (ky < kye) ? Y.lam(ky) : INF; }
    else { beta = R.lmax; lmax_left = false; }
  }
  const double *xs = x + (size_t)z * N * N;
  double acc = 0.0;
  while (lmax_left && beta < a1) {
    double nb;
    if (cx <= cy && cx <= R.lmax) { nb = cx; ++kx; cx = (kx < kxe) ? X.lam(kx) : INF; }
    else if (cy <= R.lmax) { nb = cy; ++ky; cy = (ky < kye) ? Y.lam(ky) : INF; }
    else { nb = R.lmax; lmax_left = false; }
    const double seg = nb - beta;
    if (seg > 1e-9) {
      const double mid = 0.5 * (nb + beta);
      const double xm = R.ox + mid * R.vx, ym = R.oy + mid * R.vy;
      const double ci = floor(xm + half), ri = floor(ym + half);
      if (ci >= 0.0 && ci < N && ri >= 0.0 && ri < N) acc += seg * xs[(int)ri * N + (int)ci];
    }
    beta = nb;
  }
  return acc;
}

// The piece of ray (a, d) inside pixel (row, col), 0 if the ray's piece
// there is dropped or belongs to another pixel (the forward's midpoint rule).
__device__ __forceinline__ double beam_piece(const Dev &D, const BeamRay &R, int row, int col) {
#pragma clang fp contract(off)
  if (!R.valid) return 0.0;
  const int N = D.bN;
  const double half = 0.5 * N;
  double lo = R.lmin, hi = R.lmax;
  if (R.okx) {
    const double l0 = ((double)col - half - R.ox) / R.vx, l1 = ((double)(col + 1) - half - R.ox) / R.vx;
    lo = fmax(lo, fmin(l0, l1));
    hi = fmin(hi, fmax(l0, l1));
  }
  if (R.oky) {
    const double l0 = ((double)row - half - R.oy) / R.vy, l1 = ((double)(row + 1) - half - R.oy) / R.vy;
    lo = fmax(lo, fmin(l0, l1));
    hi = fmin(hi, fmax(l0, l1));
  }
  const double seg = hi - lo;
  if (!(seg > 1e-9)) return 0.0;
  const double mid = 0.5 * (hi + lo);
  const double xm = R.ox + mid * R.vx, ym = R.oy + mid * R.vy;
  if (floor(xm + half) != (double)col || floor(ym + half) != (double)row) return 0.0;
  return seg;
}

// ray (a, d) with its interval read from the per-ray table
__device__ __forceinline__ BeamRay beam_ray_tab(const Dev &D, int a, int d, int ray) {
#pragma clang fp contract(off)
  BeamRay R;
  const double ux = D.bCos[a], uy = D.bSin[a];
  R.vx = -uy;
  R.vy = ux;
  const double t = (double)d - (D.bNd - 1) / 2.0;
  R.ox = t * ux;
  R.oy = t * uy;
  R.okx = fabs(R.vx) > 1e-15;
  R.oky = fabs(R.vy) > 1e-15;
  R.lmin = D.brl[2 * (size_t)ray];
  R.lmax = D.brl[2 * (size_t)ray + 1];
  R.valid = R.lmax > R.lmin;
  return R;
}

constexpr int kBeamLanes = 8;     // lanes sharing one ray of the forward projection

// y[r] = scale (A x)_r for rays r in [r0, r1): kBeamLanes lanes per ray, each
// summing the pieces that start in its share of the ray's interval; the
// shares are added in lane order.
__device__ __forceinline__ void beam_forward_rows(const Dev &D, const double *x, double *yout,
                                                  double *ybuf, int r0, int r1, double scale,
                                                  int nthreads) {
  const int G = kBeamLanes;
  const int g = threadIdx.x % G;
  const int per_ang = D.bNd, per_slice = D.bNa * D.bNd;
  // the lanes of a group share r, so they run the same trips and shuffle together
  for (int r = r0 + (int)threadIdx.x / G; r < r1; r += nthreads / G) {
    const int z = r / per_slice, rem = r - z * per_slice;
    const int a = rem / per_ang, d = rem - a * per_ang;
    const BeamRay R = beam_ray_tab(D, a, d, r);
    double part = beam_ray_part(D, R, x, z, g, G);
#pragma unroll
    for (int o = 1; o < G; o <<= 1) part += __shfl_xor(part, o, G);
    if (g == 0) {
      const double yr = part * scale;
      yout[r] = yr;
      if (r - r0 < kRowsLDS) ybuf[r - r0] = yr;
    }
  }
}

// y[p] = scale (B w)_p for pixels p in [p0, p1): B the exact transpose of
// the projector (every ray whose line meets the pixel, its piece there) or
// the linear interpolation between the two nearest bins of each angle.
__device__ __forceinline__ void beam_back_rows(const Dev &D, const double *w, double *yout,
                                               double *ybuf, int p0, int p1, double scale,
                                               int nthreads) {
#pragma clang fp contract(off)
  const int N = D.bN, na = D.bNa, nd = D.bNd;
  const double half = 0.5 * N, c0 = (nd - 1) / 2.0;
  for (int p = p0 + (int)threadIdx.x; p < p1; p += nthreads) {
    const int z = p / (N * N), rem = p - z * N * N;
    const int row = rem / N, col = rem - row * N;
    const double xc = (double)col - half + 0.5, yc = (double)row - half + 0.5;
    const double *ws = w + (size_t)z * na * nd;
    double acc = 0.0;
    for (int a = 0; a < na; ++a) {
      const double ux = D.bCos[a], uy = D.bSin[a];
      if (D.bBack == 1) {
        const double u = xc * ux + yc * uy + c0;
        const double lo = floor(u), f = u - lo;
        const int b0 = (int)lo;
        if (b0 >= 0 && b0 < nd && 1.0 - f > 0.0) acc += (1.0 - f) * ws[a * nd + b0];
        if (b0 + 1 >= 0 && b0 + 1 < nd && f > 0.0) acc += f * ws[a * nd + b0 + 1];
      } else {
        // bins whose line can meet the pixel: |t_d - t_centre| <= (|ux| + |uy|) / 2
        const double tc = xc * ux + yc * uy;
        const double hw = 0.5 * (fabs(ux) + fabs(uy));
        const int d0 = max(0, (int)floor(tc - hw + c0) - 1);
        const int d1 = min(nd - 1, (int)ceil(tc + hw + c0) + 1);
        for (int d = d0; d <= d1; ++d) {
          const int ray = (z * na + a) * nd + d;
          const BeamRay R = beam_ray_tab(D, a, d, ray);
          const double len = beam_piece(D, R, row, col);
          if (len != 0.0) acc += len * ws[a * nd + d];
        }
      }
    }
    const double yr = acc * scale;
    yout[p] = yr;
    if (p - p0 < kRowsLDS) ybuf[p - p0] = yr;
  }
}

}  // namespace sfk
