// Stage kernels for R right-hand sides that share the operator pair A, B
// (paper Algorithm 1 / Algorithm 2 run R times side by side, eq. (FGK) for
// each).  The long vectors of all right-hand sides are interleaved (element i
// of right-hand side r at [i * RS + r]), so one pass over the CSR arrays of A
// or B serves every right-hand side: a sparse matrix times a block of RS
// vectors, where each nonzero gathers one contiguous row of RS doubles.
//
// Every stage X of iteration k is two launches on the main stream:
//   k_gfinish<X>  one workgroup per right-hand side reduces the partial sums
//                 the previous stage left for it (fixed order), runs the same
//                 scalar step as the single-instance path (Gram-Schmidt
//                 coefficients, norms, breakdown tests), and writes the
//                 coefficients of X and an "active" flag to a small table;
//   stage kernel  streams the interleaved vectors once for all right-hand
//                 sides; a right-hand side that has stopped, broken down or
//                 reached its capacity is inactive, and nothing of it is
//                 written.
// The sketch and least-squares kernels stay per instance (sfk_kernels.hip),
// reading the interleaved raw products with stride RS.

#include "sfk_common.h"

namespace sfk {

constexpr int kGWG = 512;   // threads per SpMM workgroup
constexpr int kStreamU = 2; // elements per thread in flight in the streaming kernels

__device__ __forceinline__ double *gwvec(const Grp &G, int j) {
  return G.W + (size_t)(j % (G.ell + 2)) * G.m * G.RS;
}
__device__ __forceinline__ double *gzcol(const Grp &G, int j) {
  return G.Z + (size_t)j * G.n * G.RS;
}
__device__ __forceinline__ double *gpvec(const Grp &G, int j) {
  return G.tau == 0 ? gzcol(G, j - 1) : G.P + (size_t)(j % (G.ell + 1)) * G.n * G.RS;
}

// ---------------------------------------------------------------------------
// Scalar step of stage ST (kStageA..kStageD) for right-hand side blockIdx.x.
// ---------------------------------------------------------------------------
template <int ST>
__global__ void __launch_bounds__(kWG) k_gfinish(Grp G, int k) {
  const int r = blockIdx.x;
  const Dev &D = G.devs[r];
  __shared__ double lds_w[kMaxQ * (kWG / 64)];
  __shared__ double tot[kMaxQ];
  __shared__ int s_on;
  double *cf = G.coef + (size_t)r * kCoefStride;
  if (threadIdx.x == 0) s_on = skip_iter(D, k) ? 0 : 1;
  __syncthreads();
  if (!s_on) {
    if (threadIdx.x < kCoefStride) cf[threadIdx.x] = 0.0;
    if (threadIdx.x == 0) G.act[r] = 0;
    return;
  }
  if (ST == kStageA) {
    // before A(k): t_kk = ||p~_k|| from D(k-1); a breakdown ends the basis
    consume<kWG>(D, kStageD, k - wwin0(D, k) + 1, lds_w, tot);
    if (threadIdx.x == 0) {
      const double sg = finish_p_norm(D, k, tot, true);
      cf[0] = sg;
      G.act[r] = sg != 0.0;
    }
  } else if (ST == kStageB) {
    // before B(k): h_jk from the dots of A(k)
    consume<kWG>(D, kStageA, k - wwin0(D, k) + 2, lds_w, tot);
    if (threadIdx.x == 0) {
      finish_w_coeffs<kMaxEll + 1>(D, k, tot, cf, true);
      G.act[r] = 1;
    }
  } else if (ST == kStageC) {
    // before C(k): h_{k+1,k} = ||w~_{k+1}|| from B(k); C(0) scales w~_1 by 1/beta
    if (k >= 1) consume<kWG>(D, kStageB, k - wwin0(D, k) + 2, lds_w, tot);
    if (threadIdx.x == 0) {
      cf[0] = k >= 1 ? finish_w_norm(D, k, tot, true) : D.sigw[1];
      G.act[r] = 1;
    }
  } else {
    // before D(k): t_j,k+1 from the dots of C(k); the reweighting also needs
    // the coefficients of x_k = sum_j sigp_{j+1} y_j z~_{j+1}
    const int j0 = pwin0(D, k);
    const int nwin = k >= j0 ? k - j0 + 1 : 0;
    consume<kWG>(D, kStageC, nwin + 1, lds_w, tot);
    if (threadIdx.x == 0) {
      finish_p_coeffs<kMaxEll + 1>(D, k, tot, cf, true);
      G.act[r] = 1;
    }
    if (D.tau == 1)
      for (int j = threadIdx.x; j < k; j += kWG) G.gx[(size_t)j * G.RS + r] = D.sigp[j + 1] * D.y[j];
  }
}

__device__ __forceinline__ bool any_active(const Grp &G, int *s_any) {
  if (threadIdx.x == 0) {
    int a = 0;
    for (int r = 0; r < G.R; ++r) a |= G.act[r];
    *s_any = a;
  }
  __syncthreads();
  return *s_any != 0;
}

// Per-right-hand-side block totals of Q partial sums.  v[q] of a thread
// belongs to right-hand side threadIdx.x % RS (lanes with g > 0 of the SpMM
// pass zeros).  Threads r < R store the totals of right-hand side r at
// workgroup slot wid of its partial-sum buffer for 'stage'.
template <int RS, int NT>
__device__ void produce_rhs(const Grp &G, int stage, int wid, int Q, const double (&v)[kMaxQ],
                            double *red) {
  constexpr int NWV = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) {
    if (q < Q) {
      double t = v[q];
#pragma unroll
      for (int o = RS; o < 64; o <<= 1) t += __shfl_xor(t, o, 64);
      if (lane < RS) red[wv * RS + lane] = t;
      __syncthreads();
      if (threadIdx.x < G.R && G.act[threadIdx.x]) {
        double s = 0.0;
        for (int w = 0; w < NWV; ++w) s += red[w * RS + threadIdx.x];
        const Dev &D = G.devs[threadIdx.x];
        part_of(D, stage)[(size_t)q * D.nwmax + wid] = s;
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// A(k) / C(k): Y = scale * Op X for the block of RS vectors, with the window
// dot products and the norm of each right-hand side's product.
//   ISA = true : Y = A Z~_k,       window w~_j, j = max(1,k-ell)..k
//   ISA = false: Y = B W~_{k+1},   window p~_j, j = max(1,k+1-ell)..k
// A wave handles one row at a time: lane = g * RS + r works on right-hand
// side r and nonzeros g, g + 64/RS, ... of the row; four gathers in flight.
// ---------------------------------------------------------------------------
template <int RS, bool ISA>
__global__ void __launch_bounds__(kGWG) k_gspmm(Grp G, int k) {
  constexpr int NG = 64 / RS;
  constexpr int NWV = kGWG / 64;
  __shared__ int s_any;
  __shared__ double red[NWV * RS];
  if (!any_active(G, &s_any)) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane / RS, j = lane % RS;
  const bool on = j < G.R && G.act[j] != 0;
  const double scale = G.coef[(size_t)j * kCoefStride];
  const int wid = blockIdx.x;

  const int *rp = ISA ? G.Arp : G.Brp;
  const int *ci = ISA ? G.Aci : G.Bci;
  const double *va = ISA ? G.Ava : G.Bva;
  const int *part = ISA ? G.Apart : G.Bpart;
  const double *xin = (ISA ? gzcol(G, k - 1) : gwvec(G, k + 1)) + j;
  double *yout = ISA ? G.wraw + (size_t)(k & (kRawSlots - 1)) * G.m * RS : G.zraw + (size_t)(k & (kRawSlots - 1)) * G.n * RS;
  int j0, nwin;
  if (ISA) { j0 = max(1, k - G.ell); nwin = k - j0 + 1; }
  else { j0 = max(1, k + 1 - G.ell); nwin = k >= j0 ? k - j0 + 1 : 0; }
  const double *win[kMaxEll + 1];
#pragma unroll
  for (int q = 0; q < kMaxEll + 1; ++q)
    win[q] = (q < nwin) ? (ISA ? gwvec(G, j0 + q) : gpvec(G, j0 + q)) : nullptr;
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;

  const int r0 = part[wid], r1 = part[wid + 1];
  for (int row = r0 + wv; row < r1; row += NWV) {
    const int e0 = rp[row], e1 = rp[row + 1];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int e = e0 + g;
    for (; e + 3 * NG < e1; e += 4 * NG) {
      const double v0 = va[e], v1 = va[e + NG], v2 = va[e + 2 * NG], v3 = va[e + 3 * NG];
      const int c0 = ci[e], c1 = ci[e + NG], c2 = ci[e + 2 * NG], c3 = ci[e + 3 * NG];
      a0 += v0 * xin[(size_t)c0 * RS];
      a1 += v1 * xin[(size_t)c1 * RS];
      a2 += v2 * xin[(size_t)c2 * RS];
      a3 += v3 * xin[(size_t)c3 * RS];
    }
    for (; e < e1; e += NG) a0 += va[e] * xin[(size_t)ci[e] * RS];
    double sum = (a0 + a1) + (a2 + a3);
#pragma unroll
    for (int o = RS; o < 64; o <<= 1) sum += __shfl_xor(sum, o, 64);
    if (g == 0) {
      const size_t at = (size_t)row * RS + j;
      const double y = sum * scale;
      if (on) yout[at] = y;
#pragma unroll
      for (int q = 0; q < kMaxEll + 1; ++q)
        if (q < nwin) acc[q] += win[q][at] * y;
      acc[kMaxEll + 1] += y * y;
    }
  }
  double v[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) v[q] = (q < nwin) ? acc[q] : (q == nwin ? acc[kMaxEll + 1] : 0.0);
  produce_rhs<RS, kGWG>(G, ISA ? kStageA : kStageC, wid, nwin + 1, v, red);
}

// ---------------------------------------------------------------------------
// Sliced products.  A(k) / C(k) as two passes:
//   k_gspmm_x   one partial row per segment, sum_e val[e] X[col[e], :], with no
//               scaling; workgroup b works on slice 8 * (b / (8 nbs)) + b % 8,
//               so all workgroups of a slice share one L2 domain.  A lane
//               holds two right-hand sides (16-byte gathers through a buffer
//               resource with 32-bit offsets).  A wave reads the 16-byte
//               records (value, source-row offset) of 64 nonzeros with one
//               load and passes each lane group its record by a cross-lane
//               broadcast, so only the gathers return data per lane;
//   k_gcombine  y = scale * (sum of the row's partials in slice order), the
//               window dot products and the norm, per right-hand side.
// ---------------------------------------------------------------------------
// Hands the lanes of a nonzero group the record another lane holds.
// row_newbcast:I copies lane I of every row of 16 lanes to the whole row (one
// VALU op); ds_bpermute reads any lane (the address is the source lane * 4).
template <int I>
__device__ __forceinline__ int row_bcast(int x) {
  return __builtin_amdgcn_mov_dpp(x, 0x150 + I, 0xf, 0xf, true);
}
__device__ __forceinline__ int row_bcast_i(int x, int i) {
  switch (i) {   // i is a compile-time constant at every call site after unrolling
    case 0: return row_bcast<0>(x);    case 1: return row_bcast<1>(x);
    case 2: return row_bcast<2>(x);    case 3: return row_bcast<3>(x);
    case 4: return row_bcast<4>(x);    case 5: return row_bcast<5>(x);
    case 6: return row_bcast<6>(x);    case 7: return row_bcast<7>(x);
    case 8: return row_bcast<8>(x);    case 9: return row_bcast<9>(x);
    case 10: return row_bcast<10>(x);  case 11: return row_bcast<11>(x);
    case 12: return row_bcast<12>(x);  case 13: return row_bcast<13>(x);
    case 14: return row_bcast<14>(x);  default: return row_bcast<15>(x);
  }
}

template <int LPR>
__device__ __forceinline__ int group_bcast(int x, int i) {
  if (LPR == 16) return row_bcast_i(x, i);
  return __builtin_amdgcn_ds_bpermute(((threadIdx.x & 63) / LPR * LPR + i) * 4, x);
}

// Each lane group (LPR lanes, two right-hand sides per lane) streams its own
// contiguous range of whole segments, one nonzero per wave step: its lanes
// load the group's next LPR records with one load, a cross-lane broadcast
// hands step i the record of lane i of the group, U gathers are in flight at
// once, and when a segment ends the group stores its sums to the segment's
// partial slot (no reduction across lanes).
template <int RS, bool ISA>
__global__ void __launch_bounds__(kGWG) k_gspmm_x(Grp G, const int4 *__restrict__ segs,
                                                 const int *__restrict__ spart,
                                                 const XNz *__restrict__ nz, int k) {
  constexpr int LPR = RS / 2;          // lanes per group = records per chunk
  constexpr int NPS = 64 / LPR;        // groups per wave
  constexpr int NWV = kGWG / 64;
  constexpr int U = 4;                 // gathers in flight per lane
  static_assert(LPR % U == 0 && LPR <= kXPad && U == kSegAlign, "chunk layout");
  __shared__ int s_any;
  if (!any_active(G, &s_any)) return;
  const XOp &X = ISA ? G.xa : G.xb;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane / LPR, li = lane % LPR;
  const int j2 = li * 2;
  const int per_phase = kXcds * X.nbs;
  const int b = blockIdx.x;
  const int sl = kXcds * (b / per_phase) + b % kXcds;
  const int q = (b % per_phase) / kXcds;
  const int* up = spart + (size_t)sl * (X.nbs * X.upb + 1) + (q * NWV + wv) * NPS + g;
  const int sA = up[0], sB = up[1];
  // group state: next record, end of its range, current segment (end, slot)
  // and the following one, prefetched
  int rec = 0, rend = 0, ci = sA, cend = -1, cslot = 0, nend = -1, nslot = 0;
  if (sA < sB) {
    const int4 d0 = segs[sA];
    rec = d0.y;
    cend = d0.z;
    cslot = d0.w;
    rend = segs[sB - 1].z;
    if (sA + 1 < sB) {
      const int4 d1 = segs[sA + 1];
      nend = d1.z;
      nslot = d1.w;
    }
  }
  int steps = rend - rec;
#pragma unroll
  for (int o = LPR; o < 64; o <<= 1) steps = max(steps, __shfl_xor(steps, o, 64));
  steps = __builtin_amdgcn_readfirstlane(steps);
  const double *xbase = ISA ? gzcol(G, k - 1) : gwvec(G, k + 1);
  const int xbytes = X.cols * RS * (int)sizeof(double);
  const __amdgpu_buffer_rsrc_t xr =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(xbase), (short)0, xbytes, 0x00020000);
  const int loff = j2 * (int)sizeof(double);
  double sx = 0.0, sy = 0.0;
  // records of the next chunk are loaded one chunk ahead; a group whose range
  // has ended reads record li (valid, value masked)
  XNz zn = nz[rec < rend ? rec + li : li];             // < rend + LPR <= nnz + kXPad
  for (int c0 = 0; c0 < steps; c0 += LPR) {
    const int cr = rec + c0;
    const XNz z = zn;
    zn = nz[cr + LPR < rend ? cr + LPR + li : li];
    const int zo = z.off;
    const int zl = __double2loint(z.v), zh = __double2hiint(z.v);
#pragma unroll
    for (int i0 = 0; i0 < LPR; i0 += U) {
      if (c0 + i0 < steps) {
        int off[U];
        double v[U];
        double2 xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u;
          off[u] = group_bcast<LPR>(zo, i);
          const double vv = __hiloint2double(group_bcast<LPR>(zh, i), group_bcast<LPR>(zl, i));
          v[u] = cr + i < rend ? vv : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const auto raw = __builtin_amdgcn_raw_buffer_load_b128(xr, off[u] + loff, 0, 0);
          __builtin_memcpy(&xv[u], &raw, sizeof(double2));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          sx += v[u] * xv[u].x;
          sy += v[u] * xv[u].y;
        }
        // segments are padded to whole blocks: at most one ends here, after
        // the block's last step
        if (cr + i0 + U == cend) {
          *reinterpret_cast<double2 *>(X.part + (size_t)cslot * RS + j2) = make_double2(sx, sy);
          sx = sy = 0.0;
          ++ci;
          cend = nend;
          cslot = nslot;
          nend = -1;
          if (ci + 1 < sB) {
            const int4 d = segs[ci + 1];
            nend = d.z;
            nslot = d.w;
          }
        }
      }
    }
  }
}

// LDS-staged variant of k_gspmm_x for operators whose nearby rows read the
// same source rows.  A unit is a run of consecutive segments of one slice
// whose nonzeros read at most kLdsRows bytes of distinct source rows and hold
// at most kLdsRecs records (planned at init).  The workgroup copies the unit's
// source rows, its records and the record range of each lane group into LDS,
// then each lane group streams its range with every read from LDS: all lanes
// of a group read the current records themselves (no cross-lane broadcast), a
// record's offset is into the staged block (padding records: the zero row
// after it), and a segment's last record carries the segment's partial slot.
// The last kSegAlign record slots of a unit hold padding, read by blocks past a
// group's range.  All global reads of the next unit (rows, records, ranges) are issued
// when the current unit's compute starts and land in registers, so the compute
// loop itself reads no global memory.  Partial slots and the summation order
// inside a segment are those of k_gspmm_x.
template <int RS, bool ISA>
__global__ void __launch_bounds__(kGWG, 2) k_gspmm_l(Grp G, int k) {
  constexpr int LPR = RS / 2;          // lanes per group = records per chunk
  constexpr int NPS = 64 / LPR;        // groups per wave
  constexpr int NWV = kGWG / 64;
  constexpr int NG = NWV * NPS;        // groups per workgroup
  constexpr int U = 4;                 // records per block (segments are padded to U)
  constexpr int NB = 2;                // blocks per batch of LDS reads
  constexpr int CAP = kLdsRows / (RS * 8);   // staged rows per unit
  constexpr int XE = kLdsRows / 16;    // double2 slots of the staged block
  constexpr int SPT = (XE + kGWG - 1) / kGWG;
  constexpr int RPT = (kLdsRecs + kGWG - 1) / kGWG;
  static_assert(U == kSegAlign && kLdsRows % (8 * 64) == 0 && NG <= kGWG, "block layout");
  __shared__ double2 xs[XE + LPR];     // staged block, then a row of zeros
  __shared__ XNz zs[kLdsRecs];         // the unit's records
  __shared__ int2 gs[NG];              // record range of each lane group
  __shared__ int s_any;
  if (!any_active(G, &s_any)) return;
  const XOp &X = ISA ? G.xa : G.xb;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane / LPR, li = lane % LPR;
  const int j2 = li * 2;
  const int gid = wv * NPS + g;
  if (tid < LPR) xs[XE + tid] = make_double2(0.0, 0.0);
  const int per_phase = kXcds * X.nbw;
  const int b = blockIdx.x;
  const int sl = kXcds * (b / per_phase) + b % kXcds;
  const int q = (b % per_phase) / kXcds;
  const int *up = X.upart + (size_t)sl * (X.nbw + 1) + q;
  const int u0 = up[0], u1 = up[1];
  if (u0 >= u1) return;
  const double2 *xg = reinterpret_cast<const double2 *>(ISA ? gzcol(G, k - 1) : gwvec(G, k + 1));
  // registers of the unit about to be written to LDS: block slot t = tid +
  // i kGWG (pair t % LPR of staged row t / LPR), record tid + i kGWG, and
  // the range of group tid
  int sidx[SPT];                       // source rows of a later unit's slots, -1 past its rows
  double bx[SPT], by[SPT];
  unsigned vmask = 0;                  // bit i: slot i holds a staged row
  double rv[RPT];                      // records: value, offset, partial slot
  int ro[RPT], rs[RPT];
  int2 gg = make_int2(0, 0);
  auto load_idx = [&](int u) {
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
      const int t = tid + i * kGWG;
      sidx[i] = t < CAP * LPR ? X.stage[(size_t)u * CAP + t / LPR] : -1;
    }
  };
  auto load_unit = [&](int u) {        // uses sidx of unit u
    vmask = 0;
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
      const int t = tid + i * kGWG;
      double2 v = make_double2(0.0, 0.0);
      if (sidx[i] >= 0) {
        v = xg[(size_t)sidx[i] * LPR + t % LPR];
        vmask |= 1u << i;
      }
      bx[i] = v.x;
      by[i] = v.y;
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int t = tid + i * kGWG;
      XNz z{0.0, kLdsRows, -1};
      if (t < kLdsRecs) z = X.urec[(size_t)u * kLdsRecs + t];
      rv[i] = z.v;
      ro[i] = z.off;
      rs[i] = z.pad;
    }
    if (tid < NG) gg = X.ugrp[(size_t)u * NG + tid];
  };
  load_idx(u0);
  load_unit(u0);
  if (u0 + 1 < u1) load_idx(u0 + 1);
  for (int u = u0; u < u1; ++u) {
    __syncthreads();                   // every wave is done with the previous unit
    // every global read issued so far is needed now (vmcnt 0; expcnt and
    // lgkmcnt left alone): stating it here spares the reads of the next unit
    // waits that only the loop's merged counts would ask for
    __builtin_amdgcn_s_waitcnt(0x0F70);
#pragma unroll
    for (int i = 0; i < SPT; ++i)
      if (vmask & (1u << i)) xs[tid + i * kGWG] = make_double2(bx[i], by[i]);
#pragma unroll
    for (int i = 0; i < RPT; ++i)
      if (tid + i * kGWG < kLdsRecs) zs[tid + i * kGWG] = XNz{rv[i], ro[i], rs[i]};
    if (tid < NG) gs[tid] = gg;
    __syncthreads();
    if (u + 1 < u1) {                  // the next unit, and the row list after it
      load_unit(u + 1);
      if (u + 2 < u1) load_idx(u + 2);
    }
    const int2 gr = gs[gid];
    const int rec = gr.x, rend = gr.y;   // a whole number of blocks of U records
    int steps = rend - rec;
#pragma unroll
    for (int o = LPR; o < 64; o <<= 1) steps = max(steps, __shfl_xor(steps, o, 64));
    steps = __builtin_amdgcn_readfirstlane(steps);
    double sx = 0.0, sy = 0.0;
    // batches of NB blocks of U records; every lane of a group reads the
    // block's records itself (one address per group), and a block past the
    // group's range reads the padding records at the end of the unit's block
    for (int c0 = 0; c0 < steps; c0 += NB * U) {
      int base[NB];
#pragma unroll
      for (int h = 0; h < NB; ++h) {
        const int r = rec + c0 + h * U;
        base[h] = r < rend ? r : kLdsRecs - U;
      }
      XNz zz[NB * U];
#pragma unroll
      for (int uu = 0; uu < NB * U; ++uu) zz[uu] = zs[base[uu / U] + uu % U];
      double2 xv[NB * U];
#pragma unroll
      for (int uu = 0; uu < NB * U; ++uu)
        xv[uu] = *reinterpret_cast<const double2 *>(reinterpret_cast<const char *>(xs) +
                                                     min((unsigned)zz[uu].off, (unsigned)kLdsRows) + li * 16);
#pragma unroll
      for (int h = 0; h < NB; ++h) {
#pragma unroll
        for (int uu = h * U; uu < h * U + U; ++uu) {
          sx += zz[uu].v * xv[uu].x;
          sy += zz[uu].v * xv[uu].y;
        }
        const int es = zz[h * U + U - 1].pad;   // slot if a segment ends with this block
        if (es >= 0) {
          *reinterpret_cast<double2 *>(X.part + (size_t)es * RS + j2) = make_double2(sx, sy);
          sx = sy = 0.0;
        }
      }
    }
  }
}

template <int RS, bool ISA, int NW>
__global__ void __launch_bounds__(kWG) k_gcombine(Grp G, int k) {
  __shared__ int s_any;
  __shared__ double red[(kWG / 64) * RS];
  if (!any_active(G, &s_any)) return;
  const XOp &X = ISA ? G.xa : G.xb;
  const int j = threadIdx.x % RS;
  const bool on = j < G.R && G.act[j] != 0;
  const double scale = G.coef[(size_t)j * kCoefStride];
  const int wid = blockIdx.x;
  const int rows = ISA ? G.m : G.n;
  double *yout = ISA ? G.wraw + (size_t)(k & (kRawSlots - 1)) * G.m * RS : G.zraw + (size_t)(k & (kRawSlots - 1)) * G.n * RS;
  int j0, nwin;
  if (ISA) { j0 = max(1, k - G.ell); nwin = k - j0 + 1; }
  else { j0 = max(1, k + 1 - G.ell); nwin = k >= j0 ? k - j0 + 1 : 0; }
  const double *win[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q)
    win[q] = (q < nwin) ? (ISA ? gwvec(G, j0 + q) : gpvec(G, j0 + q)) : nullptr;
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  int i0, i1;
  chunk_range(rows, G.nwv, wid, i0, i1);
  const size_t e1 = (size_t)i1 * RS;
  for (size_t e0 = (size_t)i0 * RS + threadIdx.x; e0 < e1; e0 += kStreamU * kWG) {
    int pb[kStreamU], np[kStreamU];
#pragma unroll
    for (int u = 0; u < kStreamU; ++u) {
      const size_t e = e0 + (size_t)u * kWG;
      pb[u] = 0;
      np[u] = 0;
      if (e < e1) {
        const int i = (int)(e / RS);
        pb[u] = X.crp[i];
        np[u] = X.crp[i + 1] - pb[u];
      }
    }
    int npm = 0;
#pragma unroll
    for (int u = 0; u < kStreamU; ++u) npm = max(npm, np[u]);
    double sum[kStreamU];
#pragma unroll
    for (int u = 0; u < kStreamU; ++u) sum[u] = 0.0;
    for (int t = 0; t < npm; t += 4) {      // the partials of a row, summed in slice order
      double p[kStreamU][4];
#pragma unroll
      for (int u = 0; u < kStreamU; ++u)
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
          p[u][tt] = t + tt < np[u] ? X.part[((size_t)pb[u] + t + tt) * RS + j] : 0.0;
#pragma unroll
      for (int u = 0; u < kStreamU; ++u)
        if (t < np[u]) sum[u] = (((sum[u] + p[u][0]) + p[u][1]) + p[u][2]) + p[u][3];
    }
#pragma unroll
    for (int u = 0; u < kStreamU; ++u) {
      const size_t e = e0 + (size_t)u * kWG;
      if (e < e1) {
        const double y = sum[u] * scale;
        if (on) yout[e] = y;
#pragma unroll
        for (int q = 0; q < NW; ++q)
          if (q < nwin) acc[q] += win[q][e] * y;
        acc[NW] += y * y;
      }
    }
  }
  double v[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) v[q] = (q < nwin) ? acc[q] : (q == nwin ? acc[NW] : 0.0);
  produce_rhs<RS, kWG>(G, ISA ? kStageA : kStageC, wid, nwin + 1, v, red);
}

// ---------------------------------------------------------------------------
// Building the sliced copy (initialisation).  Columns of every row must be in
// increasing order (checked; err bit 32 otherwise).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int slice_of(const int *cb, int NS, int c, int s) {
  while (s + 1 < NS && c >= cb[s + 1]) ++s;
  return s;
}

// touch[s * rows + i] = 1 if row i has nonzeros in slice s; rowcnt[i] = segments of row i
__global__ void k_xs_count(const int *rp, const int *ci, int rows, int NS, const int *cb,
                           int *touch, int *rowcnt, int *err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  int s = -1, cnt = 0, prev = -1;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const int c = ci[e];
    if (c <= prev) { atomicOr(err, 32); return; }
    prev = c;
    const int sc = slice_of(cb, NS, c, s < 0 ? 0 : s);
    if (sc != s) {
      s = sc;
      touch[(size_t)s * rows + i] = 1;
      ++cnt;
    }
  }
  rowcnt[i] = cnt;
}

// per row, with touch and rowcnt scanned: segment id of each of its segments
// and the row-major slot of its partial
__global__ void k_xs_fill1(const int *rp, const int *ci, int rows, int NS, const int *cb,
                           const int *touch, const int *crp, int *slot, int *seglen, int *segsrc,
                           int *segrow, int *segcnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  int s = -1, t = crp[i], beg = 0, id = 0;
  const int e1 = rp[i + 1];
  for (int e = rp[i]; e <= e1; ++e) {
    const int sc = e < e1 ? slice_of(cb, NS, ci[e], s < 0 ? 0 : s) : -2;
    if (sc != s) {
      if (s >= 0) {
        seglen[id] = (e - beg + kSegAlign - 1) / kSegAlign * kSegAlign;
        segcnt[id] = e - beg;
        segsrc[id] = beg;
        segrow[id] = i;
        slot[id] = t++;
      }
      if (sc >= 0) {
        s = sc;
        beg = e;
        id = touch[(size_t)s * rows + i];
      }
    }
  }
}

// per segment: descriptor and the slice-major copy of its nonzeros
__global__ void k_xs_fill2(const int *ci, const double *va, int nseg, const int *pos,
                           const int *segsrc, const int *segrow, const int *segcnt,
                           const int *slot, int RS, int4 *seg, XNz *xnz) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nseg) return;
  const int p0 = pos[id], len = pos[id + 1] - p0, cnt = segcnt[id], src = segsrc[id];
  seg[id] = make_int4(segrow[id], p0, p0 + len, slot[id]);
  for (int e = 0; e < len; ++e) {
    XNz z;
    z.v = e < cnt ? va[src + e] : 0.0;
    z.off = e < cnt ? ci[src + e] * RS * (int)sizeof(double) : kXPadOff;
    z.pad = 0;
    xnz[p0 + e] = z;
  }
}

// nonzero-balanced segment ranges of the nbs work units of each slice
__global__ void k_xs_part(const int *touch, int rows, int NS, int nseg, const int *pos, int nbs,
                          int *spart) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= NS * (nbs + 1)) return;
  const int s = id / (nbs + 1), q = id % (nbs + 1);
  const int a = touch[(size_t)s * rows];
  const int z = s + 1 < NS ? touch[(size_t)(s + 1) * rows] : nseg;
  if (q == nbs) { spart[id] = z; return; }
  const long long lo_nz = pos[a], hi_nz = pos[z];
  const long long target = lo_nz + (hi_nz - lo_nz) * q / nbs;
  int lo = a, hi = z;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((long long)pos[mid] < target) lo = mid + 1; else hi = mid;
  }
  spart[id] = lo;
}

void launch_xs_count(const int *rp, const int *ci, int rows, int NS, const int *cb, int *touch,
                     int *rowcnt, int *err, hipStream_t st) {
  hipLaunchKernelGGL(k_xs_count, dim3((rows + 255) / 256), dim3(256), 0, st, rp, ci, rows, NS, cb,
                     touch, rowcnt, err);
}
void launch_xs_fill1(const int *rp, const int *ci, int rows, int NS, const int *cb,
                     const int *touch, const int *crp, int *slot, int *seglen, int *segsrc,
                     int *segrow, int *segcnt, hipStream_t st) {
  hipLaunchKernelGGL(k_xs_fill1, dim3((rows + 255) / 256), dim3(256), 0, st, rp, ci, rows, NS, cb,
                     touch, crp, slot, seglen, segsrc, segrow, segcnt);
}
void launch_xs_fill2(const int *ci, const double *va, int nseg, const int *pos, const int *segsrc,
                     const int *segrow, const int *segcnt, const int *slot, int RS, int4 *seg,
                     XNz *xnz, hipStream_t st) {
  hipLaunchKernelGGL(k_xs_fill2, dim3((nseg + 255) / 256), dim3(256), 0, st, ci, va, nseg, pos,
                     segsrc, segrow, segcnt, slot, RS, seg, xnz);
}
void launch_xs_part(const int *touch, int rows, int NS, int nseg, const int *pos, int nbs,
                    int *spart, hipStream_t st) {
  const int tot = NS * (nbs + 1);
  hipLaunchKernelGGL(k_xs_part, dim3((tot + 255) / 256), dim3(256), 0, st, touch, rows, NS, nseg,
                     pos, nbs, spart);
}

// ---------------------------------------------------------------------------
// B(k): w~_{k+1} = w - sum_j h_jk w~_j sigw_j for every right-hand side, with
// ||w~_{k+1}||^2 and the Gram entries <w~_{k+1}, w~_j>.  Thread t always works
// on right-hand side t % RS (kWG is a multiple of RS).
// ---------------------------------------------------------------------------
template <int RS, int NW>
__global__ void __launch_bounds__(kWG) k_gwupdate(Grp G, int k) {
  __shared__ int s_any;
  __shared__ double red[(kWG / 64) * RS];
  if (!any_active(G, &s_any)) return;
  const int j = threadIdx.x % RS;
  const bool on = j < G.R && G.act[j] != 0;
  const int wid = blockIdx.x;
  const int j0 = max(1, k - G.ell), nwin = k - j0 + 1;
  const double *win[NW];
  double cf[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    win[q] = (q < nwin) ? gwvec(G, j0 + q) : nullptr;
    cf[q] = (q < nwin) ? G.coef[(size_t)j * kCoefStride + q] : 0.0;
  }
  const double *wr = G.wraw + (size_t)(k & (kRawSlots - 1)) * G.m * RS;
  double *out = gwvec(G, k + 1);
  int i0, i1;
  chunk_range(G.m, G.nwv, wid, i0, i1);
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  // kStreamU elements per thread at a time, all loads issued before use; the
  // sums accumulate in element order
  const size_t e1 = (size_t)i1 * RS;
  for (size_t e0 = (size_t)i0 * RS + threadIdx.x; e0 < e1; e0 += kStreamU * kWG) {
    double v[kStreamU], wj[kStreamU][NW];
#pragma unroll
    for (int u = 0; u < kStreamU; ++u) {
      const size_t e = e0 + (size_t)u * kWG;
      v[u] = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) wj[u][q] = 0.0;
      if (e < e1) {
        v[u] = wr[e];
#pragma unroll
        for (int q = 0; q < NW; ++q)
          if (q < nwin) wj[u][q] = win[q][e];
      }
    }
#pragma unroll
    for (int u = 0; u < kStreamU; ++u) {
      const size_t e = e0 + (size_t)u * kWG;
      if (e < e1) {
        double vv = v[u];
#pragma unroll
        for (int q = 0; q < NW; ++q)
          if (q < nwin) vv -= cf[q] * wj[u][q];
        if (on) out[e] = vv;
        acc[0] += vv * vv;
#pragma unroll
        for (int q = 0; q < NW; ++q)
          if (q < nwin) acc[1 + q] += vv * wj[u][q];
      }
    }
  }
  produce_rhs<RS, kWG>(G, kStageB, wid, nwin + 1, acc, red);
}

// ---------------------------------------------------------------------------
// D(k): p~_{k+1} = z - sum_j t_j,k+1 p~_j sigp_j, z~_{k+1} = tau(p~_{k+1}), with
// ||p~_{k+1}||^2 and the Gram entries.  The reweighting forms x_k on the fly.
// ---------------------------------------------------------------------------
template <int RS, int NW>
__global__ void __launch_bounds__(kWG) k_gpupdate(Grp G, int k) {
  __shared__ int s_any;
  __shared__ double red[(kWG / 64) * RS];
  if (!any_active(G, &s_any)) return;
  const int j = threadIdx.x % RS;
  const bool on = j < G.R && G.act[j] != 0;
  const int wid = blockIdx.x;
  const int j0 = max(1, k + 1 - G.ell);
  const int nwin = k >= j0 ? k - j0 + 1 : 0;
  const double *win[NW];
  double cf[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    win[q] = (q < nwin) ? gpvec(G, j0 + q) : nullptr;
    cf[q] = (q < nwin) ? G.coef[(size_t)j * kCoefStride + q] : 0.0;
  }
  const bool rew = G.tau == 1;
  const double *zr = G.zraw + (size_t)(k & (kRawSlots - 1)) * G.n * RS;
  double *zout = gzcol(G, k);
  double *pout = rew ? G.P + (size_t)((k + 1) % (G.ell + 1)) * G.n * RS : zout;
  const double eps2 = G.eps * G.eps;
  const size_t colstride = (size_t)G.n * RS;
  int i0, i1;
  chunk_range(G.n, G.nwv, wid, i0, i1);
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  const size_t e1 = (size_t)i1 * RS;
  for (size_t e0 = (size_t)i0 * RS + threadIdx.x; e0 < e1; e0 += kStreamU * kWG) {
    double v[kStreamU], pj[kStreamU][NW];
#pragma unroll
    for (int u = 0; u < kStreamU; ++u) {
      const size_t e = e0 + (size_t)u * kWG;
      v[u] = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) pj[u][q] = 0.0;
      if (e < e1) {
        v[u] = zr[e];
#pragma unroll
        for (int q = 0; q < NW; ++q)
          if (q < nwin) pj[u][q] = win[q][e];
      }
    }
#pragma unroll
    for (int u = 0; u < kStreamU; ++u) {
      const size_t e = e0 + (size_t)u * kWG;
      if (e < e1) {
        double vv = v[u];
#pragma unroll
        for (int q = 0; q < NW; ++q)
          if (q < nwin) vv -= cf[q] * pj[u][q];
        if (on) pout[e] = vv;
        if (rew) {
          double xi = 0.0;
          for (int jj = 0; jj < k; ++jj) xi += G.gx[(size_t)jj * RS + j] * G.Z[(size_t)jj * colstride + e];
          if (on) {
            G.x[e] = xi;
            zout[e] = sqrt(sqrt(xi * xi + eps2)) * vv;
          }
        }
        acc[0] += vv * vv;
#pragma unroll
        for (int q = 0; q < NW; ++q)
          if (q < nwin) acc[1 + q] += vv * pj[u][q];
      }
    }
  }
  produce_rhs<RS, kWG>(G, kStageD, wid, nwin + 1, acc, red);
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <int RS, bool ISA>
static void launch_product(const Grp &G, int k, hipStream_t st) {
  if (G.sliced) {
    const XOp &X = ISA ? G.xa : G.xb;
    if (X.urec)
      hipLaunchKernelGGL((k_gspmm_l<RS, ISA>), dim3(X.NS * X.nbw), dim3(kGWG), 0, st, G, k);
    else
      hipLaunchKernelGGL((k_gspmm_x<RS, ISA>), dim3(X.NS * X.nbs), dim3(kGWG), 0, st, G, X.seg,
                         X.spart, X.nz, k);
    if (G.ell <= 2)
      hipLaunchKernelGGL((k_gcombine<RS, ISA, 3>), dim3(G.nwv), dim3(kWG), 0, st, G, k);
    else
      hipLaunchKernelGGL((k_gcombine<RS, ISA, kMaxEll + 1>), dim3(G.nwv), dim3(kWG), 0, st, G, k);
  } else {
    hipLaunchKernelGGL((k_gspmm<RS, ISA>), dim3(G.nws), dim3(kGWG), 0, st, G, k);
  }
}

template <int RS>
static void launch_group_rs(const Grp &G, int stage, int k, hipStream_t st) {
  const dim3 fin(G.R), fb(kWG);
  switch (stage) {
    case kStageA:
      hipLaunchKernelGGL(k_gfinish<kStageA>, fin, fb, 0, st, G, k);
      launch_product<RS, true>(G, k, st);
      break;
    case kStageB:
      hipLaunchKernelGGL(k_gfinish<kStageB>, fin, fb, 0, st, G, k);
      if (G.ell <= 2)
        hipLaunchKernelGGL((k_gwupdate<RS, 3>), dim3(G.nwv), dim3(kWG), 0, st, G, k);
      else
        hipLaunchKernelGGL((k_gwupdate<RS, kMaxEll + 1>), dim3(G.nwv), dim3(kWG), 0, st, G, k);
      break;
    case kStageC:
      hipLaunchKernelGGL(k_gfinish<kStageC>, fin, fb, 0, st, G, k);
      launch_product<RS, false>(G, k, st);
      break;
    default:
      hipLaunchKernelGGL(k_gfinish<kStageD>, fin, fb, 0, st, G, k);
      if (G.ell <= 2)
        hipLaunchKernelGGL((k_gpupdate<RS, 3>), dim3(G.nwv), dim3(kWG), 0, st, G, k);
      else
        hipLaunchKernelGGL((k_gpupdate<RS, kMaxEll + 1>), dim3(G.nwv), dim3(kWG), 0, st, G, k);
      break;
  }
}

// stage kA..kD of iteration k for every right-hand side of the group
void launch_group_stage(const Grp &G, int stage, int k, hipStream_t st) {
  switch (G.RS) {
    case 8: launch_group_rs<8>(G, stage, k, st); break;
    case 16: launch_group_rs<16>(G, stage, k, st); break;
    case 32: launch_group_rs<32>(G, stage, k, st); break;
    default: launch_group_rs<64>(G, stage, k, st); break;
  }
}

// lane groups (work units) of one sliced-SpMM workgroup
int gspmm_x_units_per_block(int RS) { return (kGWG / 64) * (64 / (RS / 2)); }

// resident sliced-SpMM workgroups per CU for interleave width RS
int gspmm_x_blocks_per_cu(int RS) {
  int nb = 0;
  hipError_t e;
  switch (RS) {
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gspmm_x<8, true>, kGWG, 0); break;
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gspmm_x<16, true>, kGWG, 0); break;
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gspmm_x<32, true>, kGWG, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gspmm_x<64, true>, kGWG, 0); break;
  }
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

// resident LDS-staged SpMM workgroups per CU for interleave width RS
int gspmm_l_blocks_per_cu(int RS) {
  int nb = 0;
  hipError_t e;
  switch (RS) {
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gspmm_l<8, true>, kGWG, 0); break;
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gspmm_l<16, true>, kGWG, 0); break;
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gspmm_l<32, true>, kGWG, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gspmm_l<64, true>, kGWG, 0); break;
  }
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

// resident SpMM workgroups per CU for interleave width RS
int gspmm_blocks_per_cu(int RS) {
  int nb = 0;
  hipError_t e;
  switch (RS) {
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gspmm<8, true>, kGWG, 0); break;
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gspmm<16, true>, kGWG, 0); break;
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gspmm<32, true>, kGWG, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gspmm<64, true>, kGWG, 0); break;
  }
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace sfk
