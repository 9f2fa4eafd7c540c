// SELL-64 layout of a CSR operator (the copy the SELL-64 product reads), as
// inline functions shared by the device kernels and a g++-compiled host test:
// slice s holds rows 64 s .. 64 s + 63 stored column-major, entry j of row
// 64 s + i at soff[s] + 64 j + i; every row of a slice is padded to the
// slice's length slen[s] (its longest row rounded up to a multiple of
// kSellPad) with value 0 and column 0, and so are the lanes of the last slice
// past the final row.
#pragma once

#include <stddef.h>

#if defined(__HIPCC__)
#define SFK_HD __host__ __device__
#else
#define SFK_HD
#endif

namespace sfk {

constexpr int kSellC = 64;                 // rows per slice (one per lane)
constexpr int kSellPad = 4;                // slice lengths padded to a multiple of this

SFK_HD inline int sell_slices(int rows) { return (rows + kSellC - 1) / kSellC; }

// slen of slice sl: its longest row, padded
SFK_HD inline int sell_len(const int *rp, int rows, int sl) {
  int mx = 0;
  const int r1 = (sl + 1) * kSellC < rows ? (sl + 1) * kSellC : rows;
  for (int r = sl * kSellC; r < r1; ++r) mx = rp[r + 1] - rp[r] > mx ? rp[r + 1] - rp[r] : mx;
  return (mx + kSellPad - 1) / kSellPad * kSellPad;
}

// Position of entry j of lane i of the slice starting at base.
SFK_HD inline size_t sell_at(int base, int j, int lane) {
  return (size_t)base + (size_t)j * kSellC + lane;
}

// Fills lane t = 64 s + i of the copy (t < nsl * 64, the lanes past the last
// row included): the row's entries, then (value 0, column 0) up to slen[s].
SFK_HD inline void sell_fill_lane(int t, int rows, const int *rp, const int *ci, const double *va,
                                  const int *soff, const int *slen, int *scol, double *sval) {
  const int sl = t / kSellC, i = t % kSellC;
  const int e0 = t < rows ? rp[t] : 0, len = t < rows ? rp[t + 1] - e0 : 0, L = slen[sl];
  for (int j = 0; j < L; ++j) {
    const bool in = j < len;
    const size_t at = sell_at(soff[sl], j, i);
    scol[at] = in ? ci[e0 + j] : 0;
    sval[at] = in ? va[e0 + j] : 0.0;
  }
}

// Steps [j0, j1) of a slice of length len taken by wave wv of nwv (a multiple
// of kSellPad each, the last waves possibly empty).
SFK_HD inline void sell_wave_steps(int len, int nwv, int wv, int &j0, int &j1) {
  const int per = ((len + nwv - 1) / nwv + kSellPad - 1) / kSellPad * kSellPad;
  j0 = wv * per < len ? wv * per : len;
  j1 = j0 + per < len ? j0 + per : len;
}

}  // namespace sfk
