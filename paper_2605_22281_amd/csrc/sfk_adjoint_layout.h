// Layout of the adjoint sweep's device scratch (host code, shared by the
// library and a host test that checks every buffer lies inside the
// allocation for the workload sizes).
#pragma once

#include <stddef.h>

namespace sfk {

constexpr int kAdjBlocks = 512;      // blocks of the adjoint's fixed-order reductions

// Device buffers of the sweep (carved from one allocation by carve_adjoint).
struct AdjBufs {
  double *Wseg, *Pseg, *Xseg;     // segment: unit w_j, unit p_j, x_{j-1}
  double *Wbar, *Pbar;            // adjoint rings (ell + 2 m-vectors, ell + 1 n-vectors)
  double *Zbar, *Cbar, *sbar;     // n x K, s x K, s
  double *xbar, *xnew, *vbar, *vint, *zbar, *zint, *ubar, *tmpn, *tmpm, *zk;
  double *Y, *ybar, *cpart, *part, *scal, *eacc, *epart;
};

// Carves the sweep's buffers from base and returns the doubles used; with
// base NULL it only counts (the allocation is sized by the same walk).
inline size_t carve_adjoint(double *base, int m, int n, int s, int K, int maxit, int tape, int ell,
                            AdjBufs &B) {
  size_t used = 0;
  auto take = [&](size_t cnt) {
    double *r = base ? base + used : nullptr;
    used += (cnt + 31) / 32 * 32;
    return r;
  };
  B.Wseg = take((size_t)(tape + ell + 2) * m);
  B.Pseg = take((size_t)(tape + ell + 1) * n);
  B.Xseg = take((size_t)tape * n);
  B.Wbar = take((size_t)(ell + 2) * m);
  B.Pbar = take((size_t)(ell + 1) * n);
  B.Zbar = take((size_t)n * K);
  B.Cbar = take((size_t)s * K);
  B.sbar = take(s);
  B.xbar = take(n); B.xnew = take(n); B.zbar = take(n); B.zint = take(n); B.ubar = take(n);
  B.tmpn = take(n); B.zk = take(n);
  B.vbar = take(m); B.vint = take(m); B.tmpm = take(m);
  B.Y = take((size_t)maxit * K);
  B.ybar = take(maxit);
  B.cpart = take((size_t)kAdjBlocks * (maxit + 1));
  B.part = take(kAdjBlocks);
  B.scal = take(16);
  B.eacc = take(K);
  B.epart = take(kAdjBlocks);
  return used;
}


}  // namespace sfk
