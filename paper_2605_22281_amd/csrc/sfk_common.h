// Device helpers shared by the single-instance, batched and multi-RHS stage
// kernels: workgroup reductions, per-stage partial sums, run flags, and the
// scalar steps that turn a stage's reduced sums into the recurrence
// coefficients of eq. (FGK) (modified Gram-Schmidt via the window's Gram
// matrix, norms, breakdown tests).
#pragma once

#include "sfk_dev.h"

namespace sfk {

// A pointer into device (global) memory.  A plain pointer read out of a Dev
// record may address any memory as far as the compiler knows, so its loads and
// stores become flat instructions, which also count against the LDS/scalar
// wait counter: every wait for an LDS value then waits for all memory loads in
// flight as well.  Through gptr they become global instructions.
template <class T>
using gptr = T __attribute__((address_space(1))) *;

template <class T>
__device__ __forceinline__ gptr<T> gmem(T *p) {
  return (gptr<T>)p;
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11), from the published definition.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0;
    const uint64_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}

// A double moved across lanes by a DPP pattern (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

// The double held by lane `src` (uniform across the wave), in every lane.
__device__ __forceinline__ double lane_double(double v, int src) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), src),
                          __builtin_amdgcn_readlane(__double2loint(v), src));
}

// Sum over the 64 lanes of a wave (every lane active), the same in every lane.
// Within each row of 16 lanes: pairs (xor 1), quads (xor 2), then the mirror
// images in the half row and the row, after which all 16 lanes hold the row's
// sum; the four row sums are read by lane and added as (r0 + r1) + (r2 + r3).
// No LDS traffic (cross-lane permutes through the LDS unit cost a round trip
// per stage).
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_double<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_double<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_double<0x141>(v);   // row_half_mirror
  v += dpp_double<0x140>(v);   // row_mirror
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const double r0 = __hiloint2double(__builtin_amdgcn_readlane(hi, 0), __builtin_amdgcn_readlane(lo, 0));
  const double r1 = __hiloint2double(__builtin_amdgcn_readlane(hi, 16), __builtin_amdgcn_readlane(lo, 16));
  const double r2 = __hiloint2double(__builtin_amdgcn_readlane(hi, 32), __builtin_amdgcn_readlane(lo, 32));
  const double r3 = __hiloint2double(__builtin_amdgcn_readlane(hi, 48), __builtin_amdgcn_readlane(lo, 48));
  return (r0 + r1) + (r2 + r3);
}

// Sum of Q per-thread values over a workgroup of NT threads, result in out[0..Q)
// (LDS, visible to all threads on return).  lds_w holds kMaxQ * NT / 64 doubles.
template <int NT>
__device__ __forceinline__ void block_sum(const double (&v)[kMaxQ], int Q, double *lds_w,
                                          double *out) {
  constexpr int NWV = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) {
    if (q < Q) {
      const double t = wave_sum(v[q]);
      if (lane == 0) lds_w[q * NWV + wv] = t;
    }
  }
  __syncthreads();
  if (threadIdx.x < Q) {
    double t = 0.0;
    for (int w = 0; w < NWV; ++w) t += lds_w[threadIdx.x * NWV + w];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

__device__ __forceinline__ double *part_of(const Dev &D, int stage) {
  return D.part + (size_t)stage * kMaxQ * D.nwmax;
}

// workgroups that produced a stage's partial sums
__device__ __forceinline__ int producers(const Dev &D, int stage) {
  return (stage == kStageB || stage == kStageD) ? D.nwv : D.nws;
}

// Totals of the Q partial sums that the previous stage left, in a fixed order
// (every workgroup obtains identical values).
// Every row is read unconditionally (rows from Q on re-read row Q - 1, cached,
// their values unused), so that the loads of a producer are in flight
// together instead of one branch and one wait each.
template <int NT>
__device__ __forceinline__ void consume(const Dev &D, int stage, int Q, double *lds_w, double *tot) {
  const gptr<const double> p = gmem(part_of(D, stage));
  const int np = producers(D, stage);
  const int qlast = Q > 0 ? Q - 1 : 0;
  double acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = 0.0;
  for (int i = threadIdx.x; i < np; i += NT) {
    double v[kMaxQ];
#pragma unroll
    for (int q = 0; q < kMaxQ; ++q) v[q] = p[(size_t)min(q, qlast) * D.nwmax + i];
#pragma unroll
    for (int q = 0; q < kMaxQ; ++q)
      if (q < Q) acc[q] += v[q];
  }
  block_sum<NT>(acc, Q, lds_w, tot);
}

template <int NT>
__device__ __forceinline__ void produce(const Dev &D, int stage, int wid, int Q, const double (&acc)[kMaxQ],
                        double *lds_w, double *blk) {
  block_sum<NT>(acc, Q, lds_w, blk);
  if (threadIdx.x < Q) gmem(part_of(D, stage))[(size_t)threadIdx.x * D.nwmax + wid] = blk[threadIdx.x];
}

__device__ __forceinline__ int ld_flag(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// stages of iteration k run only while the instance is live, within its
// capacity, and while its basis reaches k
__device__ __forceinline__ bool skip_iter(const Dev &D, int k) {
  const int halt = ld_flag(&D.sc->halt), klimit = ld_flag(&D.sc->klimit);   // both in flight
  return k > D.maxit || halt != 0 || k > klimit;
}

__device__ __forceinline__ void chunk_range(int d, int nw, int wid, int &i0, int &i1) {
  const int per = (d + nw - 1) / nw;
  i0 = min(d, wid * per);
  i1 = min(d, i0 + per);
}

// windows (1-based basis indices)
__device__ __forceinline__ int wwin0(const Dev &D, int k) { return max(1, k - D.ell); }      // A(k), B(k)
__device__ __forceinline__ int pwin0(const Dev &D, int k) { return max(1, k + 1 - D.ell); }  // C(k), D(k)


// ---------------------------------------------------------------------------
// Scalar steps (one thread).  tot[] holds the reduced partial sums of the
// producing stage; 'store' is true in exactly one workgroup per instance, which
// writes the persistent coefficients (H, T, inverse norms, Gram entries, flags).
// ---------------------------------------------------------------------------

// after D(k-1): t_kk = ||p~_k||, sigp_k and the Gram entries of p_k.  Returns
// 1 / t_kk, or 0 when the basis cannot grow (breakdown: klimit = k - 1).
__device__ inline double finish_p_norm(const Dev &D, int k, const double *tot, bool store) {
  Scal *sc = D.sc;
  const int ldh = D.maxit + 1;
  const int j0 = wwin0(D, k);              // D(k-1) window: [max(1,k-ell), k-1]
  const int nwin = k - j0;
  const double t = sqrt(tot[0]);
  const bool quit = (t <= kBreakdownTol * sc->zpre || t == 0.0);
  if (store) {
    D.T[(size_t)(k - 1) * ldh + (k - 1)] = t;
    if (quit) {
      atomicOr(&sc->breakdown, 1);
      atomicMin(&sc->klimit, k - 1);
    } else {
      const double sg = 1.0 / t;
      D.sigp[k] = sg;
      const int ns = D.ell + 1, sk = pslot(D, k);
      sc->Gp[sk * ns + sk] = 1.0;
      for (int q = 0; q < nwin; ++q) {
        const int j = j0 + q;
        if (j < k + 1 - D.ell) continue;
        const double g = sg * D.sigp[j] * tot[1 + q];
        sc->Gp[sk * ns + pslot(D, j)] = g;
        sc->Gp[pslot(D, j) * ns + sk] = g;
      }
    }
  }
  return quit ? 0.0 : 1.0 / t;
}

// after A(k): h_jk by modified Gram-Schmidt over the window j = max(1,k-ell)..k,
// h_q = <w_jq, w> - sum_{i<q} h_i <w_jq, w_ji>.  cf[q] = h_q * sigw_jq multiplies w~_jq.
// E: window slots of the caller (nwin <= E).  With a small E every input is
// loaded first, all at once (indices past the window clamped to its last
// entry, values unused), then combined in the same order as the loop form.
template <int E>
__device__ inline void finish_w_coeffs(const Dev &D, int k, const double *tot, double *cf,
                                       bool store) {
  Scal *sc = D.sc;
  const int j0 = wwin0(D, k), nwin = k - j0 + 1;
  const int ns = D.ell + 2, ldh = D.maxit + 1;
  if constexpr (E <= 3) {
    double sg[E], G[E][E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int jq = j0 + max(0, min(q, nwin - 1));
      sg[q] = D.sigw[jq];
#pragma unroll
      for (int i = 0; i < q; ++i)
        G[q][i] = sc->Gw[wslot(D, jq) * ns + wslot(D, j0 + max(0, min(i, nwin - 1)))];
    }
    double h[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
      if (q < nwin) {
        double t = sg[q] * tot[q];
#pragma unroll
        for (int i = 0; i < q; ++i) t -= h[i] * G[q][i];
        h[q] = t;
        cf[q] = t * sg[q];
        if (store) D.H[(size_t)(k - 1) * ldh + (j0 + q - 1)] = t;
      }
    }
  } else {
    double h[kMaxEll + 1];
    for (int q = 0; q < nwin; ++q) {
      const int jq = j0 + q;
      double t = D.sigw[jq] * tot[q];
      for (int i = 0; i < q; ++i) t -= h[i] * sc->Gw[wslot(D, jq) * ns + wslot(D, j0 + i)];
      h[q] = t;
      cf[q] = t * D.sigw[jq];
      if (store) D.H[(size_t)(k - 1) * ldh + (jq - 1)] = t;
    }
  }
  if (store) sc->wpre = sqrt(tot[nwin]);
}

// after B(k): h_{k+1,k} = ||w~_{k+1}||, sigw_{k+1}, Gram entries of w_{k+1}.
// Returns 1 / h, or 0 at a happy breakdown (h = 0: recorded in sc->happy).
__device__ inline double finish_w_norm(const Dev &D, int k, const double *tot, bool store) {
  Scal *sc = D.sc;
  const int ldh = D.maxit + 1;
  const int j0 = wwin0(D, k);
  const int nwin = k - j0 + 1;
  const double h = sqrt(tot[0]);
  const bool happy = (h <= kBreakdownTol * sc->wpre || h == 0.0);
  const double scale = happy ? 0.0 : 1.0 / h;
  if (store) {
    D.H[(size_t)(k - 1) * ldh + k] = happy ? 0.0 : h;
    D.sigw[k + 1] = scale;
    if (happy) {
      sc->happy = k;
    } else {
      const int ns = D.ell + 2, sk = wslot(D, k + 1);
      sc->Gw[sk * ns + sk] = 1.0;
      for (int q = 0; q < nwin; ++q) {
        const int j = j0 + q;
        if (j < k + 1 - D.ell) continue;
        const double g = scale * D.sigw[j] * tot[1 + q];
        sc->Gw[sk * ns + wslot(D, j)] = g;
        sc->Gw[wslot(D, j) * ns + sk] = g;
      }
    }
  }
  return scale;
}

// after C(k): t_{j,k+1} by modified Gram-Schmidt over j = max(1,k+1-ell)..k;
// cf[q] multiplies p~_jq.  E as in finish_w_coeffs (the window may be empty).
template <int E>
__device__ inline void finish_p_coeffs(const Dev &D, int k, const double *tot, double *cf,
                                       bool store) {
  Scal *sc = D.sc;
  const int j0 = pwin0(D, k);
  const int nwin = k >= j0 ? k - j0 + 1 : 0;
  const int ns = D.ell + 1, ldh = D.maxit + 1;
  if constexpr (E <= 3) {
    double sg[E], G[E][E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int jq = j0 + max(0, min(q, nwin - 1));
      sg[q] = D.sigp[jq];
#pragma unroll
      for (int i = 0; i < q; ++i)
        G[q][i] = sc->Gp[pslot(D, jq) * ns + pslot(D, j0 + max(0, min(i, nwin - 1)))];
    }
    double t[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
      if (q < nwin) {
        double v = sg[q] * tot[q];
#pragma unroll
        for (int i = 0; i < q; ++i) v -= t[i] * G[q][i];
        t[q] = v;
        cf[q] = v * sg[q];
        if (store) D.T[(size_t)k * ldh + (j0 + q - 1)] = v;
      }
    }
  } else {
    double t[kMaxEll + 1];
    for (int q = 0; q < nwin; ++q) {
      const int jq = j0 + q;
      double v = D.sigp[jq] * tot[q];
      for (int i = 0; i < q; ++i) v -= t[i] * sc->Gp[pslot(D, jq) * ns + pslot(D, j0 + i)];
      t[q] = v;
      cf[q] = v * D.sigp[jq];
      if (store) D.T[(size_t)k * ldh + (jq - 1)] = v;
    }
  }
  if (store) sc->zpre = sqrt(tot[nwin]);
}

}  // namespace sfk
