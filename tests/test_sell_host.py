"""Host check of the SELL-64 copy (csrc/sfk_sell.h), compiled with g++.

The device fill (k_sell_fill) and the SELL-64 product (spmv_sell) call the
header's functions; here the same functions fill a copy on the host, for row
counts that are not multiples of 64, and a replay of the product's loads (16
waves splitting each slice's steps, lane i on row 64 s + i, every lane of a
slice loaded, also past the last row) checks that

  * every entry the product reads was written by the fill (the arrays start
    out holding a sentinel),
  * every gathered column index lies in [0, cols),
  * padding entries and the lanes past the last row hold (column 0, value 0),
  * the replayed product equals A x.

The lanes past the last row once held whatever the allocation held and sent
the gathers out of bounds; this pins the fill's indexing.
"""
import ctypes
import pathlib
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

ROOT = pathlib.Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2605_22281_amd" / "csrc"

WRAPPER = r"""
#include "sfk_sell.h"
#include <vector>
using namespace sfk;
extern "C" long long sell_total(int rows, const int *rp, int *slen, int *soff) {
  const int nsl = sell_slices(rows);
  long long tot = 0;
  for (int s = 0; s < nsl; ++s) {
    slen[s] = sell_len(rp, rows, s);
    soff[s] = (int)tot;
    tot += (long long)slen[s] * kSellC;
  }
  soff[nsl] = (int)tot;
  return tot;
}
extern "C" void sell_fill(int rows, const int *rp, const int *ci, const double *va,
                          const int *soff, const int *slen, int *scol, double *sval) {
  const int nsl = sell_slices(rows);
  for (int t = 0; t < nsl * kSellC; ++t) sell_fill_lane(t, rows, rp, ci, va, soff, slen, scol, sval);
}
// Replays the loads of the SELL-64 product with nwv waves per workgroup.
// Returns the number of gathers outside [0, cols) (those are not performed).
extern "C" long long sell_replay(int rows, int cols, int nwv, const int *soff, const int *slen,
                                 const int *scol, const double *sval, const double *x, double *y,
                                 long long *reads) {
  const int nsl = sell_slices(rows);
  long long bad = 0;
  *reads = 0;
  std::vector<double> part((size_t)nwv * kSellC);
  for (int sl = 0; sl < nsl; ++sl) {
    for (int wv = 0; wv < nwv; ++wv) {
      int j0, j1;
      sell_wave_steps(slen[sl], nwv, wv, j0, j1);
      for (int lane = 0; lane < kSellC; ++lane) {
        double a0 = 0.0, a1 = 0.0;
        for (int j = j0; j < j1; j += kSellPad) {
          double v[kSellPad];
          int c[kSellPad];
          for (int u = 0; u < kSellPad; ++u) {
            const size_t e = sell_at(soff[sl], j + u, lane);
            v[u] = sval[e];
            c[u] = scol[e];
            ++*reads;
          }
          double xv[kSellPad];
          for (int u = 0; u < kSellPad; ++u) {
            if (c[u] < 0 || c[u] >= cols) { ++bad; xv[u] = 0.0; }
            else xv[u] = x[c[u]];
          }
          for (int u = 0; u < kSellPad; u += 2) {
            a0 += v[u] * xv[u];
            a1 += v[u + 1] * xv[u + 1];
          }
        }
        part[(size_t)wv * kSellC + lane] = a0 + a1;
      }
    }
    for (int lane = 0; lane < kSellC; ++lane) {
      double s = 0.0;
      for (int w = 0; w < nwv; ++w) s += part[(size_t)w * kSellC + lane];
      const int r = sl * kSellC + lane;
      if (r < rows) y[r] = s;
    }
  }
  return bad;
}
"""

SENTINEL_COL = -0x2A2A2A2B


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("sell")
    src = d / "sell.cpp"
    src.write_text(WRAPPER)
    so = d / "sell.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-I", str(CSRC), str(src),
                    "-o", str(so)], check=True)
    L = ctypes.CDLL(str(so))
    L.sell_total.restype = ctypes.c_longlong
    L.sell_replay.restype = ctypes.c_longlong
    return L


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _matrix(rows, cols, seed, empty_tail):
    rng = np.random.default_rng(seed)
    M = sp.random(rows, cols, density=min(1.0, 9.0 / cols), random_state=rng, format="lil")
    # a few long rows (uneven slice lengths) and a few empty ones
    for r in rng.choice(rows, size=max(1, rows // 20), replace=False):
        M[r, rng.choice(cols, size=min(cols, 40), replace=False)] = 1.0
    M = sp.csr_matrix(M)
    if empty_tail:
        keep = np.ones(rows)
        keep[-3:] = 0.0
        M = sp.csr_matrix(sp.diags(keep) @ M)
        M.eliminate_zeros()
    M.data = rng.uniform(0.1, 2.0, size=M.nnz)
    M.sort_indices()
    return M


@pytest.mark.parametrize("rows,cols,nwv", [(612, 300, 16), (65, 40, 16), (1, 7, 16),
                                          (129, 1000, 16), (700, 64, 4), (64 * 5 + 63, 257, 16)])
def test_fill_covers_every_loaded_lane(lib, rows, cols, nwv):
    M = _matrix(rows, cols, seed=rows * 7 + cols, empty_tail=rows > 8)
    rp = np.ascontiguousarray(M.indptr, dtype=np.int32)
    ci = np.ascontiguousarray(M.indices, dtype=np.int32)
    va = np.ascontiguousarray(M.data, dtype=np.float64)
    nsl = (rows + 63) // 64
    slen = np.zeros(nsl, dtype=np.int32)
    soff = np.zeros(nsl + 1, dtype=np.int32)
    tot = lib.sell_total(rows, _ptr(rp, ctypes.c_int), _ptr(slen, ctypes.c_int),
                         _ptr(soff, ctypes.c_int))
    assert tot == soff[-1] and tot % 64 == 0
    assert np.all(slen % 4 == 0)
    scol = np.full(tot, SENTINEL_COL, dtype=np.int32)
    sval = np.full(tot, np.nan, dtype=np.float64)
    lib.sell_fill(rows, _ptr(rp, ctypes.c_int), _ptr(ci, ctypes.c_int), _ptr(va, ctypes.c_double),
                  _ptr(soff, ctypes.c_int), _ptr(slen, ctypes.c_int), _ptr(scol, ctypes.c_int),
                  _ptr(sval, ctypes.c_double))
    # nothing left unwritten
    assert not np.any(scol == SENTINEL_COL)
    assert not np.any(np.isnan(sval))
    # padding: (0, 0.0) after each row's entries and in the lanes past the last row
    for t in range(nsl * 64):
        s, i = divmod(t, 64)
        n_in = rp[t + 1] - rp[t] if t < rows else 0
        at = soff[s] + 64 * np.arange(slen[s]) + i
        np.testing.assert_array_equal(scol[at[:n_in]], ci[rp[t]:rp[t] + n_in] if n_in else [])
        assert np.all(scol[at[n_in:]] == 0) and np.all(sval[at[n_in:]] == 0.0)
    x = np.random.default_rng(1).standard_normal(cols)
    y = np.full(rows, np.nan)
    reads = ctypes.c_longlong(0)
    bad = lib.sell_replay(rows, cols, nwv, _ptr(soff, ctypes.c_int), _ptr(slen, ctypes.c_int),
                          _ptr(scol, ctypes.c_int), _ptr(sval, ctypes.c_double),
                          _ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double), ctypes.byref(reads))
    assert bad == 0
    assert reads.value == tot            # every stored entry is loaded exactly once
    np.testing.assert_allclose(y, M @ x, rtol=1e-13, atol=1e-13 * np.abs(M @ x).max())
