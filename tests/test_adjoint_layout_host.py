"""Host check of the adjoint sweep's scratch layout (csrc/sfk_adjoint_layout.h),
compiled with g++: for the workload sizes (64^2, 256^2, 512^2, small cases)
and several checkpoint intervals, every buffer the sweep uses lies inside the
allocation sized by the same walk, buffers do not overlap, and each is at
least as long as the largest index the sweep's kernels use in it.

An earlier sizing formula counted one n-vector fewer than the buffers carved;
the overflow (n doubles past the allocation) went unnoticed on small
problems and faulted the device on the 256^2 workload.  The allocation is now
sized by the carving walk itself; this pins it."""
import ctypes
import pathlib
import shutil
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2605_22281_amd" / "csrc"

WRAPPER = r"""
#include "sfk_adjoint_layout.h"
using namespace sfk;
// out: used, then (offset, length) of every buffer in carving order; the
// lengths are the extents the sweep indexes
extern "C" long long layout(int m, int n, int s, int K, int maxit, int tape, int ell,
                            long long *out) {
  AdjBufs B;
  const size_t used = carve_adjoint(nullptr, m, n, s, K, maxit, tape, ell, B);
  double *base = reinterpret_cast<double *>(4096);   // never dereferenced
  carve_adjoint(base, m, n, s, K, maxit, tape, ell, B);
  const double *ptr[] = {B.Wseg, B.Pseg, B.Xseg, B.Wbar, B.Pbar, B.Zbar, B.Cbar, B.sbar,
                         B.xbar, B.xnew, B.zbar, B.zint, B.ubar, B.tmpn, B.zk, B.vbar, B.vint,
                         B.tmpm, B.Y, B.ybar, B.cpart, B.part, B.scal, B.eacc, B.epart};
  const long long len[] = {
      (long long)(tape + ell + 2) * m,         // w_{a-ell} .. w_{a+tape+1}
      (long long)(tape + ell) * n,             // p_{a+1-ell} .. p_{a+tape}
      (long long)tape * n,                     // x_a .. x_{a+tape-1}
      (long long)(ell + 2) * m, (long long)(ell + 1) * n,
      (long long)n * K, (long long)s * K, s,
      n, n, n, n, n, n, n, m, m, m,
      (long long)maxit * K,                    // y_1 .. y_K, leading dimension maxit
      maxit,
      (long long)kAdjBlocks * K,               // column partials, ldp = k <= K
      kAdjBlocks, 2, K, kAdjBlocks};
  const int nb = sizeof(len) / sizeof(len[0]);
  out[0] = (long long)used;
  for (int i = 0; i < nb; ++i) {
    out[1 + 2 * i] = (long long)(ptr[i] - base);
    out[2 + 2 * i] = len[i];
  }
  return nb;
}
"""


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("adjlayout")
    src = d / "w.cpp"
    src.write_text(WRAPPER)
    so = d / "w.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", f"-I{CSRC}", str(src), "-o",
                    str(so)], check=True)
    L = ctypes.CDLL(str(so))
    L.layout.restype = ctypes.c_longlong
    return L


CASES = [
    # m, n, s, K, maxit, tape, ell
    (276, 256, 50, 12, 12, 4, 2),
    (276, 256, 50, 12, 12, 1, 2),
    (8190, 4096, 200, 50, 50, 10, 2),
    (65340, 65536, 400, 50, 50, 10, 2),
    (65340, 65536, 400, 50, 60, 7, 8),
    (261000, 262144, 600, 300, 300, 10, 2),
]


@pytest.mark.parametrize("m,n,s,K,maxit,tape,ell", CASES)
def test_every_buffer_inside_and_disjoint(lib, m, n, s, K, maxit, tape, ell):
    out = (ctypes.c_longlong * 64)()
    nb = lib.layout(m, n, s, K, maxit, tape, ell, out)
    used = out[0]
    spans = sorted((out[1 + 2 * i], out[2 + 2 * i]) for i in range(nb))
    for off, ln in spans:
        assert off >= 0 and off + ln <= used, (off, ln, used)
    for (o1, l1), (o2, _) in zip(spans, spans[1:]):
        assert o1 + l1 <= o2
