// HIP kernels (gfx950, wave64, FP64) of the sketched flexible LSQR / LSMR
// iteration.  The host driver (sfk_capi.hip) runs the data-parallel stages on
// the context's stream and the sketch + small least-squares update on a second
// stream, so that the latency-bound LS overlaps the bandwidth-bound products.
//
// Stages of iteration k (paper Algorithm 1 / Algorithm 2, eq. (FGK)):
//   A(k)  w = A z_k                       + partials <w_j, w> (window), ||w||^2
//   B(k)  w~_{k+1} = w - sum h_jk w_j     + partials ||w~_{k+1}||^2, <w~_{k+1}, w~_j>
//   C(k)  z = B w_{k+1}                   + partials <p_j, z> (window), ||z||^2
//   D(k)  p~_{k+1} = z - sum t_j p_j, z~_{k+1} = tau(p~_{k+1})  + partials
//   S(k)  sketch of w (sFLSQR, after B) or of z (sFLSMR, after C)
//   LS(k) Householder update of the small sketched least-squares problem
// Each stage starts by reducing the partial sums of the stage before it, in a
// fixed order, identically in every workgroup (no atomics): that yields the
// modified Gram-Schmidt coefficients of the paper's loops (one pass of dot
// products corrected with the Gram matrix of the window, equal in exact
// arithmetic), the norms, and the breakdown tests.  Workgroup 0 stores the
// recurrence coefficients.  Vectors stay unnormalised (w~, p~); their inverse
// norms (sigw, sigp) are folded into the consumers.
//
// The stage kernels A-D in this file serve instances with contiguous vectors
// (Dev::vs == 1); right-hand sides that share one operator pair run the
// interleaved stage kernels of sfk_multi.hip.  Sketch, least-squares, solution
// and initialisation kernels here serve both.

#include "sfk_beam.h"
#include "sfk_common.h"

namespace sfk {

// ---------------------------------------------------------------------------
// CSR-stream product of one workgroup's rows [r0, r1) (whole rows, contiguous
// nonzeros).  The nonzeros are streamed in chunks of kChunk: every thread loads
// kPerThread (value, column) pairs at once, gathers x, and leaves the products
// in LDS; then one wave per row sums the row's segment of the chunk.  A row
// that continues into the next chunk carries its partial sum.  The next
// chunk's values and columns are loaded while the current one is reduced,
// with ordinary (temporal) loads when the operator's nonzeros fit the 256 MB
// last-level cache, so that they stay there between iterations (the 256^2
// projector, 150 MB: 48 us per product against 57 us with non-temporal
// loads), and with non-temporal loads (nt) when they do not, so that the
// stream does not evict the gathered vector (the 512^2 projector, 1.4 GB:
// 407 us against 426 us).
// y[r] = scale * sum_e val[e] x[col[e]]; also kept in ybuf for rows < kRowsLDS.
// ---------------------------------------------------------------------------
constexpr int kPerThread = 4;
constexpr int kChunk = kSpmvWG * kPerThread;
constexpr int kRowWin = 1024;   // row pointers staged per pass

template <bool NTL, class T>
__device__ __forceinline__ T stream_load(gptr<const T> p) {
  if constexpr (NTL) return __builtin_nontemporal_load(p);
  else return *p;
}

// LDS of spmv_stream, one allocation for both of its instantiations
struct StreamLds {
  double prod[kChunk];
  int rps[kRowWin + 1];
  double carry;
};
__device__ __forceinline__ StreamLds &stream_lds() {
  __shared__ StreamLds s;
  return s;
}

template <bool NTL>
__device__ void spmv_stream(gptr<const int> rp, gptr<const int> ci, gptr<const uint16_t> c16,
                            gptr<const double> va, gptr<const double> xin, gptr<double> yout,
                            double *ybuf, int r0, int r1, double scale) {
  constexpr int NT = kSpmvWG;
  StreamLds &L = stream_lds();
  double *prod = L.prod;
  int *rps = L.rps;
  double &s_carry = L.carry;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (r0 >= r1) return;
  const int E0 = rp[r0], E1 = rp[r1];
  int rcur = r0;
  double carry = 0.0;
  double vv[kPerThread];
  int cc[kPerThread];
#pragma unroll
  for (int j = 0; j < kPerThread; ++j) {
    const int e = E0 + j * NT + tid;
    if (e < E1) {
      vv[j] = stream_load<NTL>(va + e);
      cc[j] = c16 ? (int)stream_load<NTL>(c16 + e) : stream_load<NTL>(ci + e);
    } else { vv[j] = 0.0; cc[j] = -1; }
  }
  for (int cs = E0; cs < E1; cs += kChunk) {
    const int ce = min(cs + kChunk, E1);
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) prod[j * NT + tid] = cc[j] >= 0 ? vv[j] * xin[cc[j]] : 0.0;
    // prefetch the next chunk while this one is reduced
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) {
      const int e = cs + kChunk + j * NT + tid;
      if (e < E1) {
        vv[j] = stream_load<NTL>(va + e);
        cc[j] = c16 ? (int)stream_load<NTL>(c16 + e) : stream_load<NTL>(ci + e);
      } else { vv[j] = 0.0; cc[j] = -1; }
    }
    for (;;) {
      __syncthreads();
      rps[tid] = (rcur + tid <= r1) ? rp[rcur + tid] : 0x7fffffff;
      if (tid == 0) rps[kRowWin] = (rcur + kRowWin <= r1) ? rp[rcur + kRowWin] : 0x7fffffff;
      __syncthreads();
      const int nr = __syncthreads_count(rcur + tid < r1 && rps[tid] < ce);
      if (nr == 0) break;
      for (int i = wv; i < nr; i += NT / 64) {
        const int a = max(rps[i], cs) - cs, b = min(rps[i + 1], ce) - cs;
        double sum = 0.0;
        for (int q = a + lane; q < b; q += 64) sum += prod[q];
        sum = wave_sum(sum);
        if (lane == 0) {
          if (i == 0) sum += carry;
          if (rps[i + 1] <= ce) {
            const int r = rcur + i;
            const double yr = sum * scale;
            yout[r] = yr;
            if (r - r0 < kRowsLDS) ybuf[r - r0] = yr;
          } else {
            s_carry = sum;
          }
        }
      }
      __syncthreads();
      if (rps[nr] > ce) {             // the last row continues into the next chunk
        carry = s_carry;
        rcur += nr - 1;
        break;
      }
      carry = 0.0;
      rcur += nr;
      if (nr < kRowWin) break;
    }
  }
  // rows after the last nonzero are empty
  for (int r = rcur + tid; r < r1; r += NT) {
    yout[r] = 0.0;
    if (r - r0 < kRowsLDS) ybuf[r - r0] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Wave per row for long rows: a row of up to 64 * kRowSlots nonzeros is read
// in one shot (all value and column loads issued, then all gathers), so a row
// costs two dependent memory round trips and no barriers; longer rows loop.
// ---------------------------------------------------------------------------
constexpr int kRowSlots = 8;

__device__ void spmv_rows64(gptr<const int> __restrict__ rp, gptr<const int> __restrict__ ci,
                            gptr<const double> __restrict__ va, gptr<const double> __restrict__ xin,
                            gptr<double> yout, double *ybuf, int r0, int r1, double scale) {
  constexpr int NWV = kSpmvWG / 64;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int r = r0 + wv; r < r1; r += NWV) {
    const int e0 = rp[r], e1 = rp[r + 1];
    double a0 = 0.0, a1 = 0.0;
    for (int base = e0; base < e1; base += 64 * kRowSlots) {
      double v[kRowSlots];
      int c[kRowSlots];
#pragma unroll
      for (int u = 0; u < kRowSlots; ++u) {
        const int e = base + u * 64 + lane;
        const bool ok = e < e1;
        v[u] = ok ? __builtin_nontemporal_load(va + e) : 0.0;
        c[u] = ok ? __builtin_nontemporal_load(ci + e) : 0;
      }
      double xv[kRowSlots];
#pragma unroll
      for (int u = 0; u < kRowSlots; ++u) xv[u] = (base + u * 64 < e1) ? xin[c[u]] : 0.0;
#pragma unroll
      for (int u = 0; u < kRowSlots; u += 2) {
        a0 += v[u] * xv[u];
        a1 += v[u + 1] * xv[u + 1];
      }
    }
    double sum = wave_sum(a0 + a1);
    if (lane == 0) {
      const double yr = sum * scale;
      yout[r] = yr;
      if (r - r0 < kRowsLDS) ybuf[r - r0] = yr;
    }
  }
}

// ---------------------------------------------------------------------------
// SELL-64: the workgroup takes a contiguous range of slices; for each slice the
// 16 waves split its steps (lane i always on row 64 s + i), so at every step
// the 64 lanes read entry j of 64 neighbouring rows: coalesced value/column
// loads, and gathers that for neighbouring rows of a projection operator fall
// on few cache lines.  The 16 partial sums of a row are added in LDS in wave
// order.  Rows [r0, r1) of the workgroup are returned for the epilogue.
// ---------------------------------------------------------------------------
template <bool C16>
__device__ void spmv_sell(gptr<const int> __restrict__ soff, gptr<const int> __restrict__ slen,
                          gptr<const int> __restrict__ scol, gptr<const uint16_t> __restrict__ scol16,
                          gptr<const double> __restrict__ sval, gptr<const double> __restrict__ xin,
                          gptr<double> yout, double *ybuf, int s0, int s1, int rows, double scale,
                          double *lds_part) {
  constexpr int NWV = kSpmvWG / 64;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r0 = s0 * kSellC;
  for (int sl = s0; sl < s1; ++sl) {
    const int len = slen[sl];
    const int base = soff[sl];
    int j0, j1;   // this wave's steps, a multiple of kSellPad
    sell_wave_steps(len, NWV, wv, j0, j1);
    double a0 = 0.0, a1 = 0.0;
    for (int j = j0; j < j1; j += kSellPad) {
      double v[kSellPad];
      int c[kSellPad];
#pragma unroll
      for (int u = 0; u < kSellPad; ++u) {
        const size_t e = sell_at(base, j + u, lane);
        v[u] = __builtin_nontemporal_load(sval + e);
        if constexpr (C16) c[u] = (int)__builtin_nontemporal_load(scol16 + e);
        else c[u] = __builtin_nontemporal_load(scol + e);
      }
      double xv[kSellPad];
#pragma unroll
      for (int u = 0; u < kSellPad; ++u) xv[u] = xin[c[u]];
#pragma unroll
      for (int u = 0; u < kSellPad; u += 2) {
        a0 += v[u] * xv[u];
        a1 += v[u + 1] * xv[u + 1];
      }
    }
    lds_part[wv * kSellC + lane] = a0 + a1;
    __syncthreads();
    if (wv == 0) {
      double sum = 0.0;
      for (int w = 0; w < NWV; ++w) sum += lds_part[w * kSellC + lane];
      const int r = sl * kSellC + lane;
      if (r < rows) {
        const double yr = sum * scale;
        yout[r] = yr;
        if (r - r0 < kRowsLDS) ybuf[r - r0] = yr;
      }
    }
    __syncthreads();
  }
}

// spmv_sell with 16-bit or 32-bit column indices (a uniform choice: with the
// choice inside the unrolled loop, the 32-bit path waited for every load of a
// step group before issuing its last column load)
__device__ __forceinline__ void spmv_sell_any(gptr<const int> soff, gptr<const int> slen,
                                              gptr<const int> scol, gptr<const uint16_t> scol16,
                                              gptr<const double> sval, gptr<const double> xin,
                                              gptr<double> yout, double *ybuf, int s0, int s1,
                                              int rows, double scale, double *lds_part) {
  if (scol16)
    spmv_sell<true>(soff, slen, scol, scol16, sval, xin, yout, ybuf, s0, s1, rows, scale, lds_part);
  else
    spmv_sell<false>(soff, slen, scol, scol16, sval, xin, yout, ybuf, s0, s1, rows, scale, lds_part);
}

// ---------------------------------------------------------------------------
// A(k) / C(k): CSR SpMV; the window dot products run as a coalesced epilogue
// over the workgroup's rows (results staged in LDS).
//   ISA = true : consumes D(k-1) (||p~_k||, Gram), w = sigp_k * A z~_k
//   ISA = false: consumes B(k) (||w~_{k+1}||, Gram), z = sigw_{k+1} * B w~_{k+1}
// VW = 0: CSR-stream (spmv_stream); VW = 1: SELL-64 copy (spmv_sell); VW = 64:
// a wave per row, the whole row in flight (spmv_rows64); VW = 8..32: VW lanes
// cooperate on a row, four independent loads per lane in flight.
// ---------------------------------------------------------------------------
template <int VW, bool ISA>
__global__ void __launch_bounds__(kSpmvWG, 8) k_spmv(const Dev *__restrict__ devs,
                                                      const int2 *__restrict__ map, int k) {
  constexpr int NT = kSpmvWG;
  const int2 bm = map[blockIdx.x];
  const Dev &D = devs[bm.x];
  if (skip_iter(D, k)) return;
  __shared__ double lds_w[kMaxQ * (NT / 64)];
  __shared__ double tot[kMaxQ];
  __shared__ double s_scale;
  __shared__ int s_quit;
  __shared__ double ybuf[kRowsLDS];
  const int wid = bm.y;

  if (ISA) {
    // ---- finish D(k-1): t_kk = ||p~_k||, Gram entries of p_k
    consume<NT>(D, kStageD, k - wwin0(D, k) + 1, lds_w, tot);
    if (threadIdx.x == 0) {
      const double sg = finish_p_norm(D, k, tot, wid == 0);
      s_quit = sg == 0.0;
      s_scale = sg;
    }
    __syncthreads();
    if (s_quit) return;
  } else {
    if (k >= 1) {
      // ---- finish B(k): h_{k+1,k} = ||w~_{k+1}||, Gram entries of w_{k+1}
      consume<NT>(D, kStageB, k - wwin0(D, k) + 2, lds_w, tot);
      if (threadIdx.x == 0) s_scale = finish_w_norm(D, k, tot, wid == 0);
    } else if (threadIdx.x == 0) {
      s_scale = D.sigw[1];
    }
    __syncthreads();
  }

  const gptr<const int> rp = gmem(ISA ? D.Arp : D.Brp);
  const gptr<const int> ci = gmem(ISA ? D.Aci : D.Bci);
  const gptr<const double> va = gmem(ISA ? D.Ava : D.Bva);
  const gptr<const int> part = gmem(ISA ? D.Apart : D.Bpart);
  const gptr<const double> xin = gmem(ISA ? D.Z + (size_t)(k - 1) * D.n : wvec(D, k + 1));
  const gptr<double> yout = gmem(ISA ? wrawk(D, k) : zrawk(D, k));
  const double scale = s_scale;

  int r0, r1;
  if (VW == 1) {
    // SELL-64: the workgroup's rows are its slice range
    const int nsl = ISA ? D.Ansl : D.Bnsl;
    const int rows = ISA ? D.m : D.n;
    const int s0 = (int)((long long)wid * nsl / D.nws), s1 = (int)((long long)(wid + 1) * nsl / D.nws);
    r0 = min(rows, s0 * kSellC);
    r1 = min(rows, s1 * kSellC);
    __shared__ double lds_part[(kSpmvWG / 64) * kSellC];
    spmv_sell_any(gmem(ISA ? D.Asoff : D.Bsoff), gmem(ISA ? D.Aslen : D.Bslen),
              gmem(ISA ? D.Ascol : D.Bscol), gmem(ISA ? D.Ascol16 : D.Bscol16),
              gmem(ISA ? D.Asval : D.Bsval), xin, yout, ybuf, s0, s1, rows, scale, lds_part);
  } else {
    r0 = part[wid];
    r1 = part[wid + 1];
  }
  if (VW == 1) {
  } else if (VW == 3) {
    // matrix-free parallel-beam operators
    if (ISA) beam_forward_rows(D, (const double *)xin, (double *)yout, ybuf, r0, r1, scale, NT);
    else beam_back_rows(D, (const double *)xin, (double *)yout, ybuf, r0, r1, scale, NT);
  } else if (VW == 0) {
    if (ISA ? D.ntA : D.ntB)
      spmv_stream<true>(rp, ci, gmem(ISA ? D.Aci16 : D.Bci16), va, xin, yout, ybuf, r0, r1, scale);
    else
      spmv_stream<false>(rp, ci, gmem(ISA ? D.Aci16 : D.Bci16), va, xin, yout, ybuf, r0, r1, scale);
  } else if (VW == 64) {
    spmv_rows64(rp, ci, va, xin, yout, ybuf, r0, r1, scale);
  } else {
    constexpr int VWL = VW == 0 ? 64 : VW;
    const int grp = threadIdx.x / VWL, lane = threadIdx.x % VWL;
    constexpr int NG = NT / VWL;
    for (int r = r0 + grp; r < r1; r += NG) {
      const int e0 = rp[r], e1 = rp[r + 1];
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int e = e0 + lane;
      for (; e + 3 * VWL < e1; e += 4 * VWL) {
        const double v0 = __builtin_nontemporal_load(va + e);
        const double v1 = __builtin_nontemporal_load(va + e + VWL);
        const double v2 = __builtin_nontemporal_load(va + e + 2 * VWL);
        const double v3 = __builtin_nontemporal_load(va + e + 3 * VWL);
        const int c0 = __builtin_nontemporal_load(ci + e);
        const int c1 = __builtin_nontemporal_load(ci + e + VWL);
        const int c2 = __builtin_nontemporal_load(ci + e + 2 * VWL);
        const int c3 = __builtin_nontemporal_load(ci + e + 3 * VWL);
        s0 += v0 * xin[c0];
        s1 += v1 * xin[c1];
        s2 += v2 * xin[c2];
        s3 += v3 * xin[c3];
      }
      for (; e < e1; e += VWL)
        s0 += __builtin_nontemporal_load(va + e) * xin[__builtin_nontemporal_load(ci + e)];
      const double yr = group_sum<VWL>((s0 + s1) + (s2 + s3)) * scale;
      if (lane == 0) {
        yout[r] = yr;
        if (r - r0 < kRowsLDS) ybuf[r - r0] = yr;
      }
    }
  }
  __threadfence_block();
  __syncthreads();

  // epilogue: window dots and the norm over this workgroup's rows
  int j0, nwin;
  if (ISA) { j0 = wwin0(D, k); nwin = k - j0 + 1; }
  else { j0 = pwin0(D, k); nwin = k >= j0 ? k - j0 + 1 : 0; }
  gptr<const double> win[kMaxEll + 1];
#pragma unroll
  for (int q = 0; q < kMaxEll + 1; ++q)
    win[q] = (q < nwin) ? gmem(ISA ? wvec(D, j0 + q) : pvec(D, j0 + q)) : yout;
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  if (nwin <= 3) {
    // the window's three loads of a row issued together (slots past the window
    // read this product's own output, same length, value unused)
    for (int r = r0 + threadIdx.x; r < r1; r += NT) {
      const double yr = (r - r0 < kRowsLDS) ? ybuf[r - r0] : yout[r];
      double wq[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) wq[q] = win[q][r];
#pragma unroll
      for (int q = 0; q < 3; ++q)
        if (q < nwin) acc[q] += wq[q] * yr;
      acc[kMaxEll + 1] += yr * yr;
    }
  } else {
    for (int r = r0 + threadIdx.x; r < r1; r += NT) {
      const double yr = (r - r0 < kRowsLDS) ? ybuf[r - r0] : yout[r];
#pragma unroll
      for (int q = 0; q < kMaxEll + 1; ++q)
        if (q < nwin) acc[q] += win[q][r] * yr;
      acc[kMaxEll + 1] += yr * yr;
    }
  }
  double v[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) v[q] = (q < nwin) ? acc[q] : (q == nwin ? acc[kMaxEll + 1] : 0.0);
  __shared__ double blk[kMaxQ];
  produce<NT>(D, ISA ? kStageA : kStageC, wid, nwin + 1, v, lds_w, blk);
}

// ---------------------------------------------------------------------------
// y = Op x with one SpMV kernel's core only (no scaling, reductions or
// epilogue): what the initialisation times to choose the kernel per operator.
// ---------------------------------------------------------------------------
template <int VW, bool ISA>
__global__ void __launch_bounds__(kSpmvWG, 8) k_spmv_core(Dev D, const double *__restrict__ xin,
                                                         double *yout) {
  __shared__ double ybuf[kRowsLDS];
  const int wid = blockIdx.x;
  const gptr<const int> rp = gmem(ISA ? D.Arp : D.Brp);
  const gptr<const int> ci = gmem(ISA ? D.Aci : D.Bci);
  const gptr<const double> va = gmem(ISA ? D.Ava : D.Bva);
  const gptr<const int> part = gmem(ISA ? D.Apart : D.Bpart);
  const gptr<const double> xg = gmem(xin);
  const gptr<double> yg = gmem(yout);
  if (VW == 1) {
    const int nsl = ISA ? D.Ansl : D.Bnsl;
    const int rows = ISA ? D.m : D.n;
    const int s0 = (int)((long long)wid * nsl / D.nws), s1 = (int)((long long)(wid + 1) * nsl / D.nws);
    __shared__ double lds_part[(kSpmvWG / 64) * kSellC];
    spmv_sell_any(gmem(ISA ? D.Asoff : D.Bsoff), gmem(ISA ? D.Aslen : D.Bslen),
              gmem(ISA ? D.Ascol : D.Bscol), gmem(ISA ? D.Ascol16 : D.Bscol16),
              gmem(ISA ? D.Asval : D.Bsval), xg, yg, ybuf, s0, s1, rows, 1.0, lds_part);
  } else if (VW == 64) {
    spmv_rows64(rp, ci, va, xg, yg, ybuf, part[wid], part[wid + 1], 1.0);
  } else if (VW == 3) {
    if (ISA) beam_forward_rows(D, xin, yout, ybuf, part[wid], part[wid + 1], 1.0, kSpmvWG);
    else beam_back_rows(D, xin, yout, ybuf, part[wid], part[wid + 1], 1.0, kSpmvWG);
  } else {
    if (ISA ? D.ntA : D.ntB)
      spmv_stream<true>(rp, ci, gmem(ISA ? D.Aci16 : D.Bci16), va, xg, yg, ybuf, part[wid],
                        part[wid + 1], 1.0);
    else
      spmv_stream<false>(rp, ci, gmem(ISA ? D.Aci16 : D.Bci16), va, xg, yg, ybuf, part[wid],
                         part[wid + 1], 1.0);
  }
}

// ---------------------------------------------------------------------------
// B(k): consumes A(k) (dots, ||w||) -> h_jk; w~_{k+1} = w - sum h_jk w_j
// E: window slots compiled in (3 serves ell <= 2, kMaxEll + 1 any ell).  Every
// load of an element is issued before its arithmetic: the slots past the
// window read the raw product instead (a valid vector of the same length, the
// value unused), so that no load sits in a branch of its own, where the
// compiler waits for each before issuing the next.
// ---------------------------------------------------------------------------
template <int E>
__global__ void __launch_bounds__(kWG) k_wupdate(const Dev *__restrict__ devs,
                                                const int2 *__restrict__ map, int k) {
  const int2 bm = map[blockIdx.x];
  const Dev &D = devs[bm.x];
  const int wid = bm.y;
  if (skip_iter(D, k)) return;
  __shared__ double lds_w[kMaxQ * (kWG / 64)];
  __shared__ double tot[kMaxQ];
  __shared__ double blk[kMaxQ];
  __shared__ double s_cf[kMaxEll + 1];
  const int j0 = wwin0(D, k), nwin = k - j0 + 1;
  consume<kWG>(D, kStageA, nwin + 1, lds_w, tot);
  if (threadIdx.x == 0) finish_w_coeffs<E>(D, k, tot, s_cf, wid == 0);
  __syncthreads();
  const gptr<const double> wr = gmem(wrawk(D, k));
  const gptr<double> out = gmem(wvec(D, k + 1));
  gptr<const double> win[E];
  double cf[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    win[q] = (q < nwin) ? gmem(wvec(D, j0 + q)) : wr;
    cf[q] = (q < nwin) ? s_cf[q] : 0.0;
  }
  int i0, i1;
  chunk_range(D.m, D.nwv, wid, i0, i1);
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kWG) {
    double v = wr[i];
    double wj[E];
#pragma unroll
    for (int q = 0; q < E; ++q) wj[q] = win[q][i];
#pragma unroll
    for (int q = 0; q < E; ++q)
      if (q < nwin) v -= cf[q] * wj[q];
    out[i] = v;
    acc[0] += v * v;
#pragma unroll
    for (int q = 0; q < E; ++q)
      if (q < nwin) acc[1 + q] += v * wj[q];
  }
  produce<kWG>(D, kStageB, wid, nwin + 1, acc, lds_w, blk);
}

// ---------------------------------------------------------------------------
// D(k): consumes C(k) (dots, ||z||) -> t_j,k+1; p~_{k+1} = z - sum t_j p_j;
// z~_{k+1} = tau(p~_{k+1}) for the identity and the reweighting.  k = 0 is the initial step (empty window, x_0 = 0).
// The reweighting assembles x_k = Z_k y_k on the fly (y_k from LS(k)).
// ---------------------------------------------------------------------------
template <int E>
__global__ void __launch_bounds__(kWG) k_pupdate(const Dev *__restrict__ devs,
                                                const int2 *__restrict__ map, int k) {
  const int2 bm = map[blockIdx.x];
  const Dev &D = devs[bm.x];
  const int wid = bm.y;
  if (skip_iter(D, k)) return;
  __shared__ double lds_w[kMaxQ * (kWG / 64)];
  __shared__ double tot[kMaxQ];
  __shared__ double blk[kMaxQ];
  __shared__ double s_cf[kMaxEll + 1];
  extern __shared__ double coefx[];  // k coefficients of x_k (reweighting)
  const int j0 = pwin0(D, k);
  const int nwin = k >= j0 ? k - j0 + 1 : 0;
  consume<kWG>(D, kStageC, nwin + 1, lds_w, tot);
  if (threadIdx.x == 0) finish_p_coeffs<E>(D, k, tot, s_cf, wid == 0);
  const bool rew = D.tau == 1;
  if (rew)
    for (int j = threadIdx.x; j < k; j += kWG) coefx[j] = D.sigp[j + 1] * D.y[j];
  __syncthreads();
  const gptr<const double> zr = gmem(zrawk(D, k));
  gptr<const double> win[E];     // past the window: the raw product (see k_wupdate)
  double cf[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    win[q] = (q < nwin) ? gmem(pvec(D, j0 + q)) : zr;
    cf[q] = (q < nwin) ? s_cf[q] : 0.0;
  }
  const gptr<double> zout = gmem(D.Z + (size_t)k * D.n);
  // tau = I: p~ is stored as the basis column itself; otherwise in the P ring
  // (the low-rank operators then write z~ in a stage of their own)
  const gptr<double> pout = D.tau != 0 ? gmem(D.P + (size_t)pslot(D, k + 1) * D.n) : zout;
  const gptr<const double> Zg = gmem(D.Z);
  const gptr<double> xg = gmem(D.x);
  const double eps2 = D.eps * D.eps;
  int i0, i1;
  chunk_range(D.n, D.nwv, wid, i0, i1);
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kWG) {
    double v = zr[i];
    double pj[E];
#pragma unroll
    for (int q = 0; q < E; ++q) pj[q] = win[q][i];
#pragma unroll
    for (int q = 0; q < E; ++q)
      if (q < nwin) v -= cf[q] * pj[q];
    pout[i] = v;
    if (rew) {
      double xi = 0.0;
      for (int j = 0; j < k; ++j) xi += coefx[j] * Zg[(size_t)j * D.n + i];
      xg[i] = xi;
      zout[i] = sqrt(sqrt(xi * xi + eps2)) * v;
    }
    acc[0] += v * v;
#pragma unroll
    for (int q = 0; q < E; ++q)
      if (q < nwin) acc[1 + q] += v * pj[q];
  }
  produce<kWG>(D, kStageD, wid, nwin + 1, acc, lds_w, blk);
}

// ---------------------------------------------------------------------------
// Sketch application (side stream).  k = 0 is the initial sketch (S b for
// sFLSQR, S B w_1 for sFLSMR); k > 0 sketches the raw product of iteration k
// (skipped once the instance has halted).  map[blockIdx.x] = (instance, tile).
// ---------------------------------------------------------------------------
__device__ __forceinline__ const double *sketch_in(const Dev &D, int k, int &stride) {
  stride = (k == 0 && D.method == 0) ? 1 : D.vs;   // b is always contiguous
  if (k == 0) return D.method == 0 ? D.b : zrawk(D, 0);
  return D.method == 0 ? wrawk(D, k) : zrawk(D, k);
}
__device__ __forceinline__ double *sketch_out(const Dev &D, int k) {
  if (k == 0) return D.method == 0 ? D.skrhs : D.SK;
  return D.method == 0 ? D.SK + (size_t)(k - 1) * D.s : D.SK + (size_t)k * D.s;
}

// sparse-sign: a workgroup per sketch row, over the row's (column, sign) entries
// in increasing column order; identity: copy.
__global__ void __launch_bounds__(kWG) k_sketch_gather(const Dev *__restrict__ devs,
                                                      const int2 *__restrict__ map, int k) {
  const int2 bm = map[blockIdx.x];
  const Dev &D = devs[bm.x];
  if (k > 0 && skip_iter(D, k)) return;
  int vs;
  const gptr<const double> v = gmem(sketch_in(D, k, vs));
  const gptr<double> dst = gmem(sketch_out(D, k));
  if (D.sketch == 2) {
    const int i = bm.y * kWG + threadIdx.x;
    if (i < D.s) dst[i] = v[(size_t)(D.skperm ? D.skperm[i] : i) * vs];
    return;
  }
  // sparse-sign: workgroup bm.y sums sketch row bm.y; its threads split the
  // row's entries (four gathers in flight each), then the wave sums are added
  // in wave order
  __shared__ double s_part[kWG / 64];
  const int r = bm.y;
  if (r >= D.s) return;
  const int e0 = D.sk_rp[r], e1 = D.sk_rp[r + 1];
  const gptr<const int> ent = gmem(D.sk_ent);
  double acc = 0.0;
  for (int e = e0 + threadIdx.x; e < e1; e += 4 * kWG) {
    int code[4];
    double val[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) code[u] = e + u * kWG < e1 ? ent[e + u * kWG] : 0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      val[u] = e + u * kWG < e1 ? v[(size_t)(code[u] & 0x7fffffff) * vs] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += code[u] < 0 ? -val[u] : val[u];
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWG / 64; ++w) t += s_part[w];
    dst[r] = t * D.sk_scale;
  }
}

// SRHT, stage 1: per block of L = 2^log2L entries, u = D pad(v) staged in LDS and
// transformed by the Sylvester-ordered Walsh-Hadamard butterflies; the entries
// that the s selected rows need are kept: part[b][i] = (H_L u_b)[rows_i mod L].
__global__ void __launch_bounds__(kWG) k_srht_blocks(const Dev *__restrict__ devs,
                                                    const int2 *__restrict__ map, int k) {
  const int2 bm = map[blockIdx.x];
  const Dev &D = devs[bm.x];
  if (k > 0 && skip_iter(D, k)) return;
  __shared__ double u[kSrhtL];
  int vs;
  const gptr<const double> v = gmem(sketch_in(D, k, vs));
  const gptr<const unsigned long long> dbits = gmem(D.srht_d);
  const gptr<const int> skperm = gmem(D.skperm);
  const int L = 1 << D.log2L;
  const int b = bm.y;
  const int base = b * L;
  if (L == kSrhtL) {
    // Thread t holds elements t + kWG j: the butterfly stages h = 1..32 pair
    // lanes of one wave (shuffles), h = 64 and 128 pair the four waves (one
    // exchange through LDS), h = 256..1024 pair a thread's own elements.  The
    // stages run in increasing h with the same additions as the loop below.
    constexpr int E = kSrhtL / kWG;
    static_assert(E == 8 && kWG == 256, "block layout");
    const int t = threadIdx.x;
    double x[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int g = base + t + kWG * j;
      double val = 0.0;
      if (g < D.d_sk) {
        const unsigned long long w = dbits[g >> 6];
        const double vg = v[(size_t)(skperm ? skperm[g] : g) * vs];
        val = ((w >> (g & 63)) & 1ull) ? -vg : vg;
      }
      x[j] = val;
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const bool hi = (t & d) != 0;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const double o = __shfl_xor(x[j], d, 64);
        x[j] = hi ? o - x[j] : x[j] + o;
      }
    }
#pragma unroll
    for (int j = 0; j < E; ++j) u[t + kWG * j] = x[j];
    __syncthreads();
    {
      const int q = (t >> 6) & 3, i0 = t & ~192;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int i = i0 + kWG * j;
        const double a0 = u[i], a1 = u[i + 64], a2 = u[i + 128], a3 = u[i + 192];
        const double b0 = a0 + a1, b1 = a0 - a1, b2 = a2 + a3, b3 = a2 - a3;
        x[j] = q == 0 ? b0 + b2 : q == 1 ? b1 + b3 : q == 2 ? b0 - b2 : b1 - b3;
      }
    }
#pragma unroll
    for (int h = 1; h < E; h <<= 1) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        if (j & h) continue;
        const double a = x[j], c = x[j + h];
        x[j] = a + c;
        x[j + h] = a - c;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; ++j) u[t + kWG * j] = x[j];
    __syncthreads();
  } else {
    for (int i = threadIdx.x; i < L; i += kWG) {
      const int g = base + i;
      double val = 0.0;
      if (g < D.d_sk) {
        const unsigned long long w = dbits[g >> 6];
        const double vg = v[(size_t)(skperm ? skperm[g] : g) * vs];
        val = ((w >> (g & 63)) & 1ull) ? -vg : vg;
      }
      u[i] = val;
    }
    __syncthreads();
    for (int h = 1; h < L; h <<= 1) {
      for (int p = threadIdx.x; p < (L >> 1); p += kWG) {
        const int i = (p / h) * 2 * h + (p % h);
        const double a = u[i], c = u[i + h];
        u[i] = a + c;
        u[i + h] = a - c;
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < D.s; i += kWG)
    gmem(D.srht_part)[(size_t)b * D.s + i] = u[gmem(D.srht_rows)[i] & (L - 1)];
}

// SRHT, stage 2: dst_i = (1/sqrt(s)) sum_b (-1)^popcount((rows_i >> log2L) & b) part[b][i]
__global__ void __launch_bounds__(kWG) k_srht_combine(const Dev *__restrict__ devs,
                                                     const int2 *__restrict__ map, int k) {
  const int2 bm = map[blockIdx.x];
  const Dev &D = devs[bm.x];
  if (k > 0 && skip_iter(D, k)) return;
  const int i = bm.y * kWG + threadIdx.x;
  if (i >= D.s) return;
  const gptr<double> dst = gmem(sketch_out(D, k));
  const gptr<const double> part = gmem(D.srht_part);
  const int hi = D.srht_rows[i] >> D.log2L;
  // eight block partials in flight, added in block order
  double acc = 0.0;
  for (int b0 = 0; b0 < D.nblk; b0 += 8) {
    double p[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) p[u] = b0 + u < D.nblk ? part[(size_t)(b0 + u) * D.s + i] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (b0 + u < D.nblk) acc += (__popc(hi & (b0 + u)) & 1) ? -p[u] : p[u];
  }
  dst[i] = acc * D.sk_scale;
}

// ---------------------------------------------------------------------------
// y = R_j^{-1} c[0:j] by column-oriented back-substitution in one wave (R upper
// triangular, column-major, leading dimension maxit).  Columns are prefetched
// kBsPF steps ahead; the running right-hand side lives in LDS (cbuf, j doubles).
// ---------------------------------------------------------------------------
constexpr int kBsPF = 4;

template <int ER>
__device__ void backsub_wave(const Dev &D, int j, double *yout, double *cbuf) {
  const int lane = threadIdx.x;
  const int ld = D.maxit;
  const gptr<const double> R = gmem(D.R);
  for (int t = lane; t < j; t += 64) cbuf[t] = D.c[t];
  __syncthreads();
  double col[kBsPF][ER];
#pragma unroll
  for (int p = 0; p < kBsPF; ++p) {
    const int i = j - 1 - p;
#pragma unroll
    for (int e = 0; e < ER; ++e) {
      const int t = lane + 64 * e;
      col[p][e] = (i >= 0 && t <= i) ? R[(size_t)i * ld + t] : 0.0;
    }
  }
  for (int i0 = j - 1; i0 >= 0; i0 -= kBsPF) {
#pragma unroll
    for (int p = 0; p < kBsPF; ++p) {
      const int i = i0 - p;
      if (i >= 0) {
        double dl = 0.0;
#pragma unroll
        for (int e = 0; e < ER; ++e)
          if (lane + 64 * e == i) dl = col[p][e];
        const double rii = lane_double(dl, i & 63);
        const double yi = cbuf[i] / rii;
        if (lane == 0) yout[i] = yi;
#pragma unroll
        for (int e = 0; e < ER; ++e) {
          const int t = lane + 64 * e;
          if (t < i) cbuf[t] -= col[p][e] * yi;
        }
        const int in = i - kBsPF;
#pragma unroll
        for (int e = 0; e < ER; ++e) {
          const int t = lane + 64 * e;
          col[p][e] = (in >= 0 && t <= in) ? R[(size_t)in * ld + t] : 0.0;
        }
        __syncthreads();
      }
    }
  }
}

// y_j for 1 <= j <= k_done (solution_at, or y_k when it is not kept up to date)
template <int ER>
__global__ void __launch_bounds__(64) k_backsub(Dev D, int j, double *yout) {
  __shared__ double cbuf[kMaxS];
  backsub_wave<ER>(D, j, yout, cbuf);
}

// ---------------------------------------------------------------------------
// LS(k): one wave.  Householder QR of the sketched matrix, grown by one column:
//   sFLSQR column k = S A z_k;  sFLSMR column k = [S B W_{k+1}] H[:, k].
// Keeps c = Q^T rhs and R; rho_k = ||c[k:s]||.  y_k = R^{-1} c[0:k] is formed by
// back-substitution when the flexible operator needs x_k (reweighting), else on
// demand (the leading entries of c never change, so any earlier y_j is available).
// ---------------------------------------------------------------------------
template <int E, int PF, int ER>
__global__ void __launch_bounds__(64) k_ls(const Dev *__restrict__ devs, int k) {
  const Dev &D = devs[blockIdx.x];
  if (skip_iter(D, k)) return;
  __shared__ double s_tau[kMaxS];
  __shared__ double s_r[kMaxS];
  const int lane = threadIdx.x;
  const int s = D.s;
  const int ldr = D.maxit;
  const int ldh = D.maxit + 1;
  const int nsel = k - 1;
  Scal *sc = D.sc;

  double a[E];
#pragma unroll
  for (int e = 0; e < E; ++e) a[e] = 0.0;
  if (D.method == 0) {
    const gptr<const double> col = gmem(D.SK) + (size_t)(k - 1) * s;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = lane + 64 * e;
      if (i < s) a[e] = col[i];
    }
  } else {
    const int j0 = max(1, k - D.ell);
    for (int j = j0; j <= k + 1; ++j) {
      const double hj = D.H[(size_t)(k - 1) * ldh + (j - 1)];
      const gptr<const double> col = gmem(D.SK) + (size_t)(j - 1) * s;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int i = lane + 64 * e;
        if (i < s) a[e] += hj * col[i];
      }
    }
  }
  for (int t = lane; t < nsel; t += 64) s_tau[t] = D.tauv[t];
  __syncthreads();

  // apply H_1 ... H_{k-1}.  The reflectors pass through a register ring PF
  // rows ahead.  Their loads are unconditional (row clamped to the last
  // reflector, entry to the last sketch row), so that no branch join makes the
  // compiler wait for them; entries past s meet a zero coefficient instead
  // (a is zero there, and stays so).
  if (nsel > 0) {
    const gptr<const double> Vg = gmem(D.V);
    double vb[PF][E];
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const gptr<const double> vp = Vg + (size_t)min(p, nsel - 1) * s;
#pragma unroll
      for (int e = 0; e < E; ++e) vb[p][e] = vp[min(lane + 64 * e, s - 1)];
    }
    for (int j = 0; j < nsel; j += PF) {
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int jj = j + p;
        if (jj < nsel) {
          double d = 0.0;
#pragma unroll
          for (int e = 0; e < E; ++e) d += vb[p][e] * a[e];
          const double g = s_tau[jj] * wave_sum(d);
#pragma unroll
          for (int e = 0; e < E; ++e) a[e] -= (lane + 64 * e < s ? g : 0.0) * vb[p][e];
        }
        // keep the refill after the use: hoisted above it, the loads would be
        // counted ahead of the older rows still in flight (in-order counter)
        __builtin_amdgcn_sched_barrier(0);
        const gptr<const double> vp = Vg + (size_t)min(jj + PF, nsel - 1) * s;
#pragma unroll
        for (int e = 0; e < E; ++e) vb[p][e] = vp[min(lane + 64 * e, s - 1)];
      }
    }
  }

  // new reflector from a[nsel:s]
  double alpha_l = 0.0, x2 = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = lane + 64 * e;
    if (i == nsel) alpha_l = a[e];
    if (i > nsel && i < s) x2 += a[e] * a[e];
  }
  const double alpha = lane_double(alpha_l, nsel & 63);
  x2 = wave_sum(x2);
  double beta, tau, scl;
  if (x2 == 0.0) {
    beta = alpha; tau = 0.0; scl = 0.0;
  } else {
    beta = -copysign(sqrt(alpha * alpha + x2), alpha);
    tau = (beta - alpha) / beta;
    scl = 1.0 / (alpha - beta);
  }
  double v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = lane + 64 * e;
    v[e] = (i == nsel) ? 1.0 : ((i > nsel && i < s) ? a[e] * scl : 0.0);
  }
  {
    double *vp = D.V + (size_t)nsel * s;
    double *rc = D.R + (size_t)nsel * ldr;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = lane + 64 * e;
      if (i < s) vp[i] = v[e];
      if (i < nsel) { rc[i] = a[e]; s_r[i] = a[e]; }
    }
    if (lane == 0) { rc[nsel] = beta; D.tauv[nsel] = tau; }
  }
  // c <- H_k c
  double cv[E];
  double d = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = lane + 64 * e;
    cv[e] = i < s ? D.c[i] : 0.0;
    d += v[e] * cv[e];
  }
  d = tau * wave_sum(d);
  double ck_l = 0.0, r2 = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = lane + 64 * e;
    cv[e] -= d * v[e];
    if (i < s) D.c[i] = cv[e];
    if (i == nsel) ck_l = cv[e];
    if (i > nsel && i < s) r2 += cv[e] * cv[e];
  }
  const double ck = lane_double(ck_l, nsel & 63);
  const double rho = sqrt(wave_sum(r2));
  __syncthreads();

  if (beta == 0.0) {  // the new sketched column is zero: the basis cannot grow
    if (lane == 0) { atomicOr(&sc->breakdown, 4); sc->halt = 1; }
    return;
  }
  // the reweighting needs y_k = R_k^{-1} c[0:k] before the next basis vector,
  // the per-iteration true residual for x_k
  if (D.tau == 1 || D.resid) backsub_wave<ER>(D, k, D.y, s_r);
  if (lane == 0) {
    D.rho[k - 1] = rho;
    sc->k_done = k;
    if (ld_flag(&sc->happy) == k) { atomicOr(&sc->breakdown, 2); sc->halt = 1; }
    if (sc->tol > 0.0 && rho < sc->tol * sc->rhsnorm) { sc->stopped = 1; sc->halt = 1; }
  }
  (void)ck;
}

// ---------------------------------------------------------------------------
// solution and residual helpers
// ---------------------------------------------------------------------------
// x = sum_{j<kk} sigp_{j+1} y_j z~_{j+1}
__global__ void __launch_bounds__(kWG) k_solution(Dev D, int kk, const double *yv, double *x) {
  extern __shared__ double cf[];
  for (int j = threadIdx.x; j < kk; j += kWG) cf[j] = D.sigp[j + 1] * yv[j];
  __syncthreads();
  const int i = blockIdx.x * kWG + threadIdx.x;
  if (i >= D.n) return;
  double xi = 0.0;
  for (int j = 0; j < kk; ++j) xi += cf[j] * zcol(D, j)[(size_t)i * D.vs];
  x[D.pinv ? D.pinv[i] : i] = xi;
}

// ||b - A x||^2: partials over the nnz-balanced row ranges, then one workgroup
__global__ void __launch_bounds__(kWG) k_true_residual(Dev D, const double *x) {
  __shared__ double lds_w[kMaxQ * (kWG / 64)];
  __shared__ double blk[kMaxQ];
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  const int r0 = D.Apart[blockIdx.x], r1 = D.Apart[blockIdx.x + 1];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int r = r0 + wv; r < r1; r += kWG / 64) {
    double s = 0.0;
    for (int e = D.Arp[r] + lane; e < D.Arp[r + 1]; e += 64) s += D.Ava[e] * x[D.Aci[e]];
    s = wave_sum(s);
    if (lane == 0) { const double rr = D.b[r] - s; acc[0] += rr * rr; }
  }
  produce<kWG>(D, kStageMisc, blockIdx.x, 1, acc, lds_w, blk);
}

// Per-iteration true residual (resid >= 1, side stream after LS(k)): runs only
// when LS(k) completed (k_done = k); a stop at k makes every later k skip.
__device__ __forceinline__ bool true_iter_off(const Dev &D, int k) {
  return ld_flag(&D.sc->k_done) != k;
}

// x_k = Z_k y_k in the library's order of the unknowns
__global__ void __launch_bounds__(kWG) k_xres(Dev D, int k) {
  if (true_iter_off(D, k)) return;
  extern __shared__ double cf[];
  for (int j = threadIdx.x; j < k; j += kWG) cf[j] = D.sigp[j + 1] * D.y[j];
  __syncthreads();
  const gptr<const double> Zg = gmem(D.Z);
  for (int i = blockIdx.x * kWG + threadIdx.x; i < D.n; i += gridDim.x * kWG) {
    double xi = 0.0;
    for (int j = 0; j < k; ++j) xi += cf[j] * Zg[(size_t)j * D.n + i];
    D.xres[i] = xi;
  }
}

// ||b - A x_k||^2 partials over the nnz-balanced row ranges (operator as the
// products use it, x_k in the same order)
__global__ void __launch_bounds__(kWG) k_true_res_iter(Dev D, int k) {
  if (true_iter_off(D, k)) return;
  __shared__ double lds_w[kMaxQ * (kWG / 64)];
  __shared__ double blk[kMaxQ];
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  const int r0 = D.Apart[blockIdx.x], r1 = D.Apart[blockIdx.x + 1];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const gptr<const double> x = gmem(D.xres);
  for (int r = r0 + wv; r < r1; r += kWG / 64) {
    double s = 0.0;
    for (int e = D.Arp[r] + lane; e < D.Arp[r + 1]; e += 64) s += D.Ava[e] * x[D.Aci[e]];
    s = wave_sum(s);
    if (lane == 0) { const double rr = D.b[r] - s; acc[0] += rr * rr; }
  }
  produce<kWG>(D, kStageTrue, blockIdx.x, 1, acc, lds_w, blk);
}

// ||b - A x||^2 partials from a computed A x (matrix-free operators), over
// the row ranges of the SpMV workgroups, into the partial buffer of `stage`
__global__ void __launch_bounds__(kWG) k_resid_ax(Dev D, const double *ax, int stage, int k) {
  if (stage == kStageTrue && true_iter_off(D, k)) return;
  __shared__ double lds_w[kMaxQ * (kWG / 64)];
  __shared__ double blk[kMaxQ];
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  const int r0 = D.Apart[blockIdx.x], r1 = D.Apart[blockIdx.x + 1];
  for (int r = r0 + threadIdx.x; r < r1; r += kWG) {
    const double rr = D.b[r] - ax[r];
    acc[0] += rr * rr;
  }
  produce<kWG>(D, stage, blockIdx.x, 1, acc, lds_w, blk);
}

// rtrue[k-1] = ||b - A x_k||; with resid = 2 the discrepancy principle stops
// the run at the first k with ||b - A x_k|| <= ttol
__global__ void __launch_bounds__(kWG) k_true_stop(Dev D, int k) {
  if (true_iter_off(D, k)) return;
  __shared__ double lds_w[kMaxQ * (kWG / 64)];
  __shared__ double tot[kMaxQ];
  // the producers of kStageTrue are the nws SpMV row ranges
  const gptr<const double> p = gmem(part_of(D, kStageTrue));
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  for (int i = threadIdx.x; i < D.nws; i += kWG) acc[0] += p[i];
  block_sum<kWG>(acc, 1, lds_w, tot);
  if (threadIdx.x != 0) return;
  const double r = sqrt(tot[0]);
  D.rtrue[k - 1] = r;
  Scal *sc = D.sc;
  if (D.resid == 2 && r <= sc->ttol) { sc->stopped = 1; sc->halt = 1; }
}

__global__ void __launch_bounds__(kWG) k_finish_misc(Dev D, double *out) {
  __shared__ double lds_w[kMaxQ * (kWG / 64)];
  __shared__ double tot[kMaxQ];
  consume<kWG>(D, kStageMisc, 1, lds_w, tot);
  if (threadIdx.x == 0) *out = sqrt(tot[0]);
}

// ---------------------------------------------------------------------------
// initialisation kernels
// ---------------------------------------------------------------------------
// CSR structure check: row pointers monotone from 0 to nnz, columns in range.
// ---------------------------------------------------------------------------
// Caller's order of the unknowns (initialisation only).  perm must hold each
// of 0..n-1 once; pinv is its inverse.
// ---------------------------------------------------------------------------
__global__ void k_perm_check(const int *perm, int n, int *cnt, int *pinv, int *err) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int v = perm[j];
  if (v < 0 || v >= n) {
    atomicOr(err, 8);
    return;
  }
  if (atomicAdd(cnt + v, 1) != 0) atomicOr(err, 8);
  else pinv[v] = j;
}
// A' = A with column j renamed perm[j] (rows keep their entries, re-sorted
// afterwards by k_tr_sort)
__global__ void k_relabel_cols(const int *ci, const double *va, int nnz, const int *perm, int *oci,
                               double *ova) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  oci[e] = perm[ci[e]];
  ova[e] = va[e];
}
// B' = B with row i moved to row perm[i]: lengths (then an exclusive scan of
// [len_0, ..., len_{n-1}, 0]), then one wave copies each row
__global__ void k_perm_rowlen(const int *rp, int rows, const int *perm, int *orp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows) orp[perm[i]] = rp[i + 1] - rp[i];
  if (i == rows) orp[rows] = 0;
}
__global__ void k_perm_rows(const int *rp, const int *ci, const double *va, int rows,
                            const int *perm, const int *orp, int *oci, double *ova) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= rows) return;
  const int e0 = rp[i], len = rp[i + 1] - e0, d0 = orp[perm[i]];
  for (int t = lane; t < len; t += 64) {
    oci[d0 + t] = ci[e0 + t];
    ova[d0 + t] = va[e0 + t];
  }
}

__global__ void k_csr_check(const int *rp, const int *ci, int rows, int cols, long long nnz,
                            int *err) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r > rows) return;
  if (r == 0 && rp[0] != 0) atomicOr(err, 1);
  if (r == rows) { if ((long long)rp[rows] != nnz) atomicOr(err, 1); return; }
  const int e0 = rp[r], e1 = rp[r + 1];
  if (e1 < e0 || e0 < 0 || (long long)e1 > nnz) { atomicOr(err, 1); return; }
  for (int e = e0; e < e1; ++e)
    if (ci[e] < 0 || ci[e] >= cols) { atomicOr(err, 2); return; }
}

// nnz-balanced row ranges: part[w] = first row r with rp[r] >= w * nnz / nw
__global__ void k_partition(const int *rp, int rows, long long nnz, int nw, int *part) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w > nw) return;
  if (w == nw) { part[w] = rows; return; }
  const long long target = (long long)w * nnz / nw;
  int lo = 0, hi = rows;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((long long)rp[mid] < target) lo = mid + 1; else hi = mid;
  }
  part[w] = lo;
}

// device transpose of A (m x n) into B (n x m): counts, then atomic fill, then
// a per-row sort by column so that the row order does not depend on timing.
__global__ void k_tr_count(const int *rp, const int *ci, int rows, int *cnt) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  for (int e = rp[r]; e < rp[r + 1]; ++e) atomicAdd(cnt + ci[e], 1);
}

// exclusive scan of a[0..len) in place by one workgroup
__global__ void __launch_bounds__(1024) k_scan_single(int *a, int len) {
  __shared__ int sums[1024];
  const int t = threadIdx.x;
  const int per = (len + 1023) / 1024;
  const int b0 = min(len, t * per), b1 = min(len, b0 + per);
  int s = 0;
  for (int i = b0; i < b1; ++i) s += a[i];
  sums[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? sums[t - o] : 0;
    __syncthreads();
    sums[t] += v;
    __syncthreads();
  }
  int run = t ? sums[t - 1] : 0;
  for (int i = b0; i < b1; ++i) { const int v = a[i]; a[i] = run; run += v; }
}

__global__ void k_tr_fill(const int *rp, const int *ci, const double *va, int rows, int *cursor,
                          int *bci, double *bva) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  for (int e = rp[r]; e < rp[r + 1]; ++e) {
    const int pos = atomicAdd(cursor + ci[e], 1);
    bci[pos] = r;
    bva[pos] = va[e];
  }
}

// sort each row segment by column (odd-even transposition in LDS, len <= 4096)
__global__ void __launch_bounds__(256) k_tr_sort(const int *brp, int *bci, double *bva, int rows,
                                                 int *err) {
  __shared__ int kc[4096];
  __shared__ double kv[4096];
  const int r = blockIdx.x;
  if (r >= rows) return;
  const int e0 = brp[r], len = brp[r + 1] - e0;
  if (len > 4096) { if (threadIdx.x == 0) atomicOr(err, 4); return; }
  for (int i = threadIdx.x; i < len; i += 256) { kc[i] = bci[e0 + i]; kv[i] = bva[e0 + i]; }
  __syncthreads();
  for (int phase = 0; phase < len; ++phase) {
    for (int i = 2 * threadIdx.x + (phase & 1); i + 1 < len; i += 512) {
      if (kc[i] > kc[i + 1]) {
        const int tc = kc[i]; kc[i] = kc[i + 1]; kc[i + 1] = tc;
        const double tv = kv[i]; kv[i] = kv[i + 1]; kv[i + 1] = tv;
      }
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < len; i += 256) { bci[e0 + i] = kc[i]; bva[e0 + i] = kv[i]; }
}

// sparse-sign generation: column j takes zeta distinct rows from Philox blocks
// (j, t, 0, 0); code = (row << 1) | negative.
__global__ void k_ss_gen(Dev D, uint64_t key0, uint64_t key1, int *err) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= D.d_sk) return;
  const int zeta = D.zeta;
  const uint64_t s = (uint64_t)D.s;
  int rows[64];
  int cnt = 0;
  for (uint64_t t = 0; cnt < zeta; ++t) {
    if (t > 100000) { atomicOr(err, 8); return; }
    uint64_t c[4] = {(uint64_t)j, t, 0ull, 0ull};
    philox4x64_10(c, key0, key1);
    for (int w = 0; w < 4 && cnt < zeta; ++w) {
      const uint64_t u = c[w];
      const int row = (int)(((u >> 32) * s) >> 32);
      bool dup = false;
      for (int q = 0; q < cnt; ++q) dup |= (rows[q] == row);
      if (dup) continue;
      rows[cnt] = row;
      D.sk_code[(size_t)j * zeta + cnt] = (row << 1) | (int)(u & 1ull);
      ++cnt;
    }
  }
}

// per chunk of 256 columns: entries per sketch row
__global__ void __launch_bounds__(256) k_ss_count(Dev D, int *chunk_cnt) {
  extern __shared__ int cnt[];
  for (int r = threadIdx.x; r < D.s; r += 256) cnt[r] = 0;
  __syncthreads();
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < D.d_sk)
    for (int t = 0; t < D.zeta; ++t) atomicAdd(&cnt[D.sk_code[(size_t)j * D.zeta + t] >> 1], 1);
  __syncthreads();
  for (int r = threadIdx.x; r < D.s; r += 256) chunk_cnt[(size_t)blockIdx.x * D.s + r] = cnt[r];
}

// per sketch row: offsets of each chunk within the row; totals into sk_rp[r]
__global__ void k_ss_rowscan(Dev D, int *chunk_cnt, int nchunk) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D.s) return;
  int run = 0;
  for (int c = 0; c < nchunk; ++c) {
    const int v = chunk_cnt[(size_t)c * D.s + r];
    chunk_cnt[(size_t)c * D.s + r] = run;
    run += v;
  }
  D.sk_rp[r] = run;
}

// place entries of each chunk in column order (one thread per chunk)
__global__ void __launch_bounds__(64) k_ss_fill(Dev D, const int *chunk_off) {
  extern __shared__ int cur[];
  for (int r = threadIdx.x; r < D.s; r += 64) cur[r] = D.sk_rp[r] + chunk_off[(size_t)blockIdx.x * D.s + r];
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int j0 = blockIdx.x * 256, j1 = min(D.d_sk, j0 + 256);
  for (int j = j0; j < j1; ++j)
    for (int t = 0; t < D.zeta; ++t) {
      const int code = D.sk_code[(size_t)j * D.zeta + t];
      const int pos = cur[code >> 1]++;
      D.sk_ent[pos] = (int)((unsigned)(D.skperm ? D.skperm[j] : j) | ((unsigned)(code & 1) << 31));
    }
}

// SRHT signs: word w of D is word (w & 3) of the block with counter (w >> 2, 0, 0, 0)
__global__ void k_srht_dbits(Dev D, uint64_t key0, uint64_t key1) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= D.N / 64 + (D.N < 64 ? 1 : 0)) return;
  uint64_t c[4] = {(uint64_t)(w >> 2), 0ull, 0ull, 0ull};
  philox4x64_10(c, key0, key1);
  D.srht_d[w] = c[w & 3];
}

// SRHT rows: partial Fisher-Yates over [0, N) with a permutation in scratch
__global__ void k_srht_rows(Dev D, uint64_t key0, uint64_t key1, int *perm) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const uint64_t N = (uint64_t)D.N;
  uint64_t c[4] = {0, 0, 0, 0};
  for (int t = 0; t < D.s; ++t) {
    if ((t & 3) == 0) { c[0] = (uint64_t)(t >> 2); c[1] = c[2] = c[3] = 0; philox4x64_10(c, key0, key1); }
    const uint64_t u = c[t & 3];
    const int j = t + (int)__umul64hi(u, N - (uint64_t)t);
    const int a = perm[t], b = perm[j];
    perm[t] = b; perm[j] = a;
    D.srht_rows[t] = b;
  }
}

__global__ void k_iota(int *a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = i;
}

// beta = ||b||, w~_1 = b, sigw_1 = 1 / beta, stop tolerance (one workgroup)
__global__ void __launch_bounds__(1024) k_init_b(Dev D, double eta, double noise, double tol_user,
                                                int use_disc) {
  __shared__ double lds_w[kMaxQ * 16];
  __shared__ double tot[kMaxQ];
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  double *w1 = wvec(D, 1);
  for (int i = threadIdx.x; i < D.m; i += 1024) {
    const double v = D.b[i];
    w1[(size_t)i * D.vs] = v;
    acc[0] += v * v;
  }
  block_sum<1024>(acc, 1, lds_w, tot);
  if (threadIdx.x != 0) return;
  Scal *sc = D.sc;
  const double beta = sqrt(tot[0]);
  sc->beta = beta;
  sc->klimit = 0x7fffffff;
  if (!(beta > 0.0) || !isfinite(beta)) { sc->err |= 16; sc->halt = 1; return; }
  D.sigw[1] = 1.0 / beta;
  // with the true-residual stop (resid = 2) the sketched test is off and the
  // discrepancy principle reads ||b - A x_k|| <= eta delta_e (or tol ||b||)
  sc->ttol = noise > 0.0 ? eta * noise : tol_user * beta;
  sc->tol = D.resid == 2 ? 0.0 : (use_disc ? eta * noise / beta : tol_user);
}

// rhs = S b (sFLSQR) or beta * S B w_1 (sFLSMR, in SK column 0); c = rhs
__global__ void __launch_bounds__(64) k_init_rhs(Dev D) {
  Scal *sc = D.sc;
  if (sc->halt) return;
  const int lane = threadIdx.x;
  double r2 = 0.0;
  for (int i = lane; i < D.s; i += 64) {
    double v = D.method == 0 ? D.skrhs[i] : sc->beta * D.SK[i];
    D.skrhs[i] = v;
    D.c[i] = v;
    r2 += v * v;
  }
  r2 = wave_sum(r2);
  if (lane == 0) sc->rhsnorm = sqrt(r2);
}

// SELL-64 build: slen[s] = longest row of slice s, padded to kSellPad
__global__ void k_sell_len(const int *rp, int rows, int nsl, int *slen) {
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= nsl) return;
  slen[sl] = sell_len(rp, rows, sl);
}

// one thread per slice lane, the lanes of the last slice past the final row
// included (the SpMV loads every lane of a slice): row entries at
// soff[s] + 64 j + i, then padding (value 0, column 0) up to the slice length
__global__ void k_sell_fill(const int *rp, const int *ci, const double *va, int rows, int nsl,
                            const int *soff, const int *slen, int *scol, double *sval) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsl * kSellC) return;
  sell_fill_lane(t, rows, rp, ci, va, soff, slen, scol, sval);
}

// run state of every instance after iteration k: 1 if no further iteration can
// change it (stopped, broken down, or past its capacity)
__global__ void k_collect_halt(const Dev *__restrict__ devs, int n, int k, int *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Dev &D = devs[i];
  const Scal *sc = D.sc;
  const int done = ld_flag(&sc->k_done);
  out[i] = (ld_flag(&sc->halt) != 0 || ld_flag(&sc->klimit) <= done || k >= D.maxit) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// launch helpers (host side)
// ---------------------------------------------------------------------------
// Launch geometry of one batch of instances (device arrays built by the host).
template <bool ISA>
static void launch_spmv_vw(const Launch &L, int k, int vw, hipStream_t st) {
  const dim3 g(L.nspmv), b(kSpmvWG);
  const int2 *map = L.map_spmv;
  switch (vw) {
    case 8: hipLaunchKernelGGL((k_spmv<8, ISA>), g, b, 0, st, L.devs, map, k); break;
    case 16: hipLaunchKernelGGL((k_spmv<16, ISA>), g, b, 0, st, L.devs, map, k); break;
    case 32: hipLaunchKernelGGL((k_spmv<32, ISA>), g, b, 0, st, L.devs, map, k); break;
    case 64: hipLaunchKernelGGL((k_spmv<64, ISA>), g, b, 0, st, L.devs, map, k); break;
    case 1: hipLaunchKernelGGL((k_spmv<1, ISA>), g, b, 0, st, L.devs, map, k); break;
    case 3: hipLaunchKernelGGL((k_spmv<3, ISA>), g, b, 0, st, L.devs, map, k); break;
    default: hipLaunchKernelGGL((k_spmv<0, ISA>), g, b, 0, st, L.devs, map, k); break;
  }
}

// resident SpMV workgroups per CU (the grid is sized to one wave of workgroups)
int spmv_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_spmv<0, true>, kSpmvWG, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

void launch_stage_A(const Launch &L, int k, hipStream_t st) { launch_spmv_vw<true>(L, k, L.vwA, st); }
void launch_stage_C(const Launch &L, int k, hipStream_t st) { launch_spmv_vw<false>(L, k, L.vwB, st); }
void launch_stage_B(const Launch &L, int k, hipStream_t st) {
  if (L.ellmax <= 2) hipLaunchKernelGGL((k_wupdate<3>), dim3(L.nvec), dim3(kWG), 0, st, L.devs, L.map_vec, k);
  else hipLaunchKernelGGL((k_wupdate<kMaxEll + 1>), dim3(L.nvec), dim3(kWG), 0, st, L.devs, L.map_vec, k);
}
void launch_stage_D(const Launch &L, int k, hipStream_t st) {
  const size_t sh = L.tau == 1 ? sizeof(double) * (size_t)max(1, k) : 0;
  if (L.ellmax <= 2) hipLaunchKernelGGL((k_pupdate<3>), dim3(L.nvec), dim3(kWG), sh, st, L.devs, L.map_vec, k);
  else hipLaunchKernelGGL((k_pupdate<kMaxEll + 1>), dim3(L.nvec), dim3(kWG), sh, st, L.devs, L.map_vec, k);
}

// sketch of iteration k (k = 0: the initial sketch) for every instance
void launch_sketch(const Launch &L, int k, hipStream_t st) {
  if (L.nsb > 0) {
    hipLaunchKernelGGL(k_srht_blocks, dim3(L.nsb), dim3(kWG), 0, st, L.devs, L.map_sb, k);
    hipLaunchKernelGGL(k_srht_combine, dim3(L.nsc), dim3(kWG), 0, st, L.devs, L.map_sc, k);
  }
  if (L.nsg > 0)
    hipLaunchKernelGGL(k_sketch_gather, dim3(L.nsg), dim3(kWG), 0, st, L.devs, L.map_sg, k);
}

template <int ER>
static void launch_ls_er(const Launch &L, int k, hipStream_t st) {
  const int s = L.smax;
  const dim3 g(L.ninst), b(64);
  if (s <= 128) hipLaunchKernelGGL((k_ls<2, 4, ER>), g, b, 0, st, L.devs, k);
  else if (s <= 256) hipLaunchKernelGGL((k_ls<4, 4, ER>), g, b, 0, st, L.devs, k);
  else if (s <= 512) hipLaunchKernelGGL((k_ls<8, 4, ER>), g, b, 0, st, L.devs, k);
  else if (s <= 1024) hipLaunchKernelGGL((k_ls<16, 2, ER>), g, b, 0, st, L.devs, k);
  else hipLaunchKernelGGL((k_ls<32, 2, ER>), g, b, 0, st, L.devs, k);
}

// ER = elements per lane of an R column (maxit <= 64 * ER)
void launch_ls(const Launch &L, int k, hipStream_t st) {
  if (L.maxitmax <= 128) launch_ls_er<2>(L, k, st);
  else if (L.maxitmax <= 256) launch_ls_er<4>(L, k, st);
  else if (L.maxitmax <= 512) launch_ls_er<8>(L, k, st);
  else if (L.maxitmax <= 1024) launch_ls_er<16>(L, k, st);
  else launch_ls_er<32>(L, k, st);
}

void launch_backsub(const Dev &D, int j, double *yout, hipStream_t st) {
  if (D.maxit <= 128) hipLaunchKernelGGL((k_backsub<2>), dim3(1), dim3(64), 0, st, D, j, yout);
  else if (D.maxit <= 256) hipLaunchKernelGGL((k_backsub<4>), dim3(1), dim3(64), 0, st, D, j, yout);
  else if (D.maxit <= 512) hipLaunchKernelGGL((k_backsub<8>), dim3(1), dim3(64), 0, st, D, j, yout);
  else if (D.maxit <= 1024) hipLaunchKernelGGL((k_backsub<16>), dim3(1), dim3(64), 0, st, D, j, yout);
  else hipLaunchKernelGGL((k_backsub<32>), dim3(1), dim3(64), 0, st, D, j, yout);
}

void launch_init_b(const Dev &D, double eta, double noise, double tol_user, int use_disc,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_init_b, dim3(1), dim3(1024), 0, st, D, eta, noise, tol_user, use_disc);
}
void launch_init_rhs(const Dev &D, hipStream_t st) {
  hipLaunchKernelGGL(k_init_rhs, dim3(1), dim3(64), 0, st, D);
}
void launch_collect_halt(const Launch &L, int k, int *out, hipStream_t st) {
  hipLaunchKernelGGL(k_collect_halt, dim3((L.ninst + 255) / 256), dim3(256), 0, st, L.devs, L.ninst,
                     k, out);
}
// one launch of the core of SpMV kernel vw (0, 1 or 64) for A (isa) or B
void launch_spmv_core(const Dev &D, bool isa, int vw, const double *x, double *y, hipStream_t st) {
  const dim3 g(D.nws), b(kSpmvWG);
  if (vw == 3) {
    if (isa) hipLaunchKernelGGL((k_spmv_core<3, true>), g, b, 0, st, D, x, y);
    else hipLaunchKernelGGL((k_spmv_core<3, false>), g, b, 0, st, D, x, y);
    return;
  }
  if (isa) {
    if (vw == 1) hipLaunchKernelGGL((k_spmv_core<1, true>), g, b, 0, st, D, x, y);
    else if (vw == 64) hipLaunchKernelGGL((k_spmv_core<64, true>), g, b, 0, st, D, x, y);
    else hipLaunchKernelGGL((k_spmv_core<0, true>), g, b, 0, st, D, x, y);
  } else {
    if (vw == 1) hipLaunchKernelGGL((k_spmv_core<1, false>), g, b, 0, st, D, x, y);
    else if (vw == 64) hipLaunchKernelGGL((k_spmv_core<64, false>), g, b, 0, st, D, x, y);
    else hipLaunchKernelGGL((k_spmv_core<0, false>), g, b, 0, st, D, x, y);
  }
}

// 16-bit copy of column indices known to lie in [0, 65536)
__global__ void k_to_u16(const int *in, uint16_t *out, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = (uint16_t)in[i];
}
void launch_to_u16(const int *in, uint16_t *out, long long n, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_to_u16, dim3((unsigned)std::min<long long>((n + 255) / 256, 65536)),
                       dim3(256), 0, st, in, out, n);
}
void launch_sell_len(const int *rp, int rows, int nsl, int *slen, hipStream_t st) {
  hipLaunchKernelGGL(k_sell_len, dim3((nsl + 255) / 256), dim3(256), 0, st, rp, rows, nsl, slen);
}
void launch_sell_fill(const int *rp, const int *ci, const double *va, int rows, const int *soff,
                      const int *slen, int *scol, double *sval, hipStream_t st) {
  const int nsl = (rows + kSellC - 1) / kSellC;
  if (nsl > 0)
    hipLaunchKernelGGL(k_sell_fill, dim3((nsl * kSellC + 255) / 256), dim3(256), 0, st, rp, ci, va,
                       rows, nsl, soff, slen, scol, sval);
}
void launch_scan(int *a, int len, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, st, a, len);
}
void launch_csr_check(const int *rp, const int *ci, int rows, int cols, long long nnz, int *err,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_csr_check, dim3((rows + 1 + 255) / 256), dim3(256), 0, st, rp, ci, rows,
                     cols, nnz, err);
}
void launch_partition(const int *rp, int rows, long long nnz, int nw, int *part, hipStream_t st) {
  hipLaunchKernelGGL(k_partition, dim3((nw + 1 + 255) / 256), dim3(256), 0, st, rp, rows, nnz, nw,
                     part);
}
void launch_transpose(const int *rp, const int *ci, const double *va, int rows, int cols,
                      int *brp, int *bci, double *bva, int *cursor, int *err, hipStream_t st) {
  hipMemsetAsync(brp, 0, sizeof(int) * (cols + 1), st);
  hipLaunchKernelGGL(k_tr_count, dim3((rows + 255) / 256), dim3(256), 0, st, rp, ci, rows, brp);
  // exclusive scan of [cnt_0, ..., cnt_{n-1}, 0]: entry c is the start of row c,
  // entry n the total
  hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, st, brp, cols + 1);
  hipMemcpyAsync(cursor, brp, sizeof(int) * cols, hipMemcpyDeviceToDevice, st);
  hipLaunchKernelGGL(k_tr_fill, dim3((rows + 255) / 256), dim3(256), 0, st, rp, ci, va, rows,
                     cursor, bci, bva);
  hipLaunchKernelGGL(k_tr_sort, dim3(cols), dim3(256), 0, st, brp, bci, bva, cols, err);
}
void launch_perm_check(const int *perm, int n, int *cnt, int *pinv, int *err, hipStream_t st) {
  hipLaunchKernelGGL(k_perm_check, dim3((n + 255) / 256), dim3(256), 0, st, perm, n, cnt, pinv, err);
}
// A' columns renamed and each row re-sorted (err bit 4: a row longer than 4096)
void launch_relabel_cols(const int *rp, const int *ci, const double *va, int rows, int nnz,
                         const int *perm, int *oci, double *ova, int *err, hipStream_t st) {
  if (nnz > 0)
    hipLaunchKernelGGL(k_relabel_cols, dim3((nnz + 255) / 256), dim3(256), 0, st, ci, va, nnz, perm,
                       oci, ova);
  if (rows > 0) hipLaunchKernelGGL(k_tr_sort, dim3(rows), dim3(256), 0, st, rp, oci, ova, rows, err);
}
void launch_perm_rows(const int *rp, const int *ci, const double *va, int rows, const int *perm,
                      int *orp, int *oci, double *ova, hipStream_t st) {
  hipLaunchKernelGGL(k_perm_rowlen, dim3((rows + 1 + 255) / 256), dim3(256), 0, st, rp, rows, perm, orp);
  hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, st, orp, rows + 1);
  if (rows > 0)
    hipLaunchKernelGGL(k_perm_rows, dim3((rows + 3) / 4), dim3(256), 0, st, rp, ci, va, rows, perm, orp,
                       oci, ova);
}
void launch_sketch_build(const Dev &D, uint64_t key0, uint64_t key1, uint64_t key1_rows,
                         int *scratch, int *err, hipStream_t st) {
  if (D.sketch == 0) {
    hipLaunchKernelGGL(k_ss_gen, dim3((D.d_sk + 255) / 256), dim3(256), 0, st, D, key0, key1, err);
    const int nchunk = (D.d_sk + 255) / 256;
    hipLaunchKernelGGL(k_ss_count, dim3(nchunk), dim3(256), sizeof(int) * D.s, st, D, scratch);
    hipLaunchKernelGGL(k_ss_rowscan, dim3((D.s + 255) / 256), dim3(256), 0, st, D, scratch, nchunk);
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, st, D.sk_rp, D.s + 1);
    hipLaunchKernelGGL(k_ss_fill, dim3(nchunk), dim3(64), sizeof(int) * D.s, st, D, scratch);
  } else if (D.sketch == 1) {
    const int nw = D.N / 64 + (D.N < 64 ? 1 : 0);
    hipLaunchKernelGGL(k_srht_dbits, dim3((nw + 255) / 256), dim3(256), 0, st, D, key0, key1);
    hipLaunchKernelGGL(k_iota, dim3((D.N + 255) / 256), dim3(256), 0, st, scratch, D.N);
    hipLaunchKernelGGL(k_srht_rows, dim3(1), dim3(1), 0, st, D, key0, key1_rows, scratch);
  }
}
void launch_solution(const Dev &D, int kk, const double *yv, double *x, hipStream_t st) {
  hipLaunchKernelGGL(k_solution, dim3((D.n + kWG - 1) / kWG), dim3(kWG),
                     sizeof(double) * (size_t)max(1, kk), st, D, kk, yv, x);
}
// per-ray parameter interval inside the image (lmin, lmax; a ray that misses
// the image gets lmin = 1, lmax = 0)
__global__ void k_beam_rays(Dev D) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D.m) return;
  const int per_slice = D.bNa * D.bNd;
  const int rem = r % per_slice, a = rem / D.bNd, d = rem % D.bNd;
  const BeamRay R = beam_ray(D, a, d);
  D.brl[2 * (size_t)r] = R.valid ? R.lmin : 1.0;
  D.brl[2 * (size_t)r + 1] = R.valid ? R.lmax : 0.0;
}
void launch_beam_rays(const Dev &D, hipStream_t st) {
  hipLaunchKernelGGL(k_beam_rays, dim3((D.m + 255) / 256), dim3(256), 0, st, D);
}

// rows split evenly over nw workgroups
__global__ void k_uniform_part(int rows, int nw, int *part) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w <= nw) part[w] = (int)((long long)rows * w / nw);
}
void launch_uniform_part(int rows, int nw, int *part, hipStream_t st) {
  hipLaunchKernelGGL(k_uniform_part, dim3((nw + 1 + 255) / 256), dim3(256), 0, st, rows, nw, part);
}

// byte fill with zero (16-byte stores; the tail byte by byte)
__global__ void k_zero_bytes(unsigned char *p, size_t n) {
  const size_t n16 = n / 16;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += stride)
    reinterpret_cast<int4 *>(p)[i] = make_int4(0, 0, 0, 0);
  for (size_t i = n16 * 16 + blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride)
    p[i] = 0;
}
void launch_zero_bytes(void *p, size_t n, hipStream_t st) {
  if (n == 0) return;
  const size_t blocks = std::min<size_t>((n / 16 + 255) / 256 + 1, 4096);
  hipLaunchKernelGGL(k_zero_bytes, dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<unsigned char *>(p), n);
}

// block map of a single instance: entry w = (0, w)
__global__ void k_iota_map(int2 *map, int count) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < count) map[w] = make_int2(0, w);
}
void launch_iota_map(int2 *map, int count, hipStream_t st) {
  if (count > 0)
    hipLaunchKernelGGL(k_iota_map, dim3((count + 255) / 256), dim3(256), 0, st, map, count);
}

// a stored basis vector times its scale (1 / the norm of the unnormalised
// vector), written in the caller's order when pinv is given
__global__ void k_export_vec(const double *src, int vs, int len, const double *scale,
                             const int *pinv, double *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  out[pinv ? pinv[i] : i] = src[(size_t)i * vs] * scale[0];
}
void launch_export_vec(const double *src, int vs, int len, const double *scale, const int *pinv,
                       double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_export_vec, dim3((len + 255) / 256), dim3(256), 0, st, src, vs, len, scale,
                     pinv, out);
}

void launch_true_iter(const Dev &D, int k, hipStream_t st) {
  const int nb = std::max(1, std::min((D.n + kWG - 1) / kWG, 2048));
  hipLaunchKernelGGL(k_xres, dim3(nb), dim3(kWG), sizeof(double) * (size_t)max(1, k), st, D, k);
  if (D.vwA == 3) {
    launch_spmv_core(D, true, 3, D.xres, D.mscr, st);
    hipLaunchKernelGGL(k_resid_ax, dim3(D.nws), dim3(kWG), 0, st, D, (const double *)D.mscr,
                       (int)kStageTrue, k);
  } else {
    hipLaunchKernelGGL(k_true_res_iter, dim3(D.nws), dim3(kWG), 0, st, D, k);
  }
  hipLaunchKernelGGL(k_true_stop, dim3(1), dim3(kWG), 0, st, D, k);
}
void launch_true_residual(const Dev &D, const double *x, double *out, hipStream_t st) {
  if (D.vwA == 3) {
    launch_spmv_core(D, true, 3, x, D.mscr, st);
    hipLaunchKernelGGL(k_resid_ax, dim3(D.nws), dim3(kWG), 0, st, D, (const double *)D.mscr,
                       (int)kStageMisc, 0);
  } else {
    hipLaunchKernelGGL(k_true_residual, dim3(D.nws), dim3(kWG), 0, st, D, x);
  }
  hipLaunchKernelGGL(k_finish_misc, dim3(1), dim3(kWG), 0, st, D, out);
}

}  // namespace sfk
