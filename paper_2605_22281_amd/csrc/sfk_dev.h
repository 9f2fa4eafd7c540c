// Internal device-side layout of one solver instance.  Everything here is
// FP64 except indices; all arrays live in one device workspace carved by the
// host (sfk_capi.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sfk_sell.h"

namespace sfk {

constexpr int kMaxEll = 8;                 // orthogonalisation window limit
constexpr int kMaxS = 2048;                // sketch rows limit (LS kept in one wave)
constexpr int kWG = 256;                   // threads per vector-stage workgroup
constexpr int kSpmvWG = 1024;              // threads per SpMV workgroup
constexpr int kRowsLDS = 2048;             // SpMV results kept in LDS for the epilogue
constexpr int kMaxQ = kMaxEll + 2;         // partial sums per workgroup and stage
constexpr int kRawSlots = 8;   // raw products kept (the sketch of iteration k reads
                                // slot k % kRawSlots until iteration k + kRawSlots)
constexpr int kSrhtL = 2048;               // SRHT block length staged in LDS
constexpr double kBreakdownTol = 1e-14;    // relative breakdown threshold

// Partial-sum buffers, one per producing stage.
// kStageMisc: the true residual asked for after the run; kStageTrue: the one
// recorded every iteration (side stream)
enum Stage { kStageA = 0, kStageB = 1, kStageC = 2, kStageD = 3, kStageMisc = 4, kStageTrue = 5,
             kNumPart = 6 };

// Scalar state shared by the stages (device memory).  Slots: w_j lives in
// W ring slot j % (ell + 2), p_j in P ring slot j % (ell + 1).
struct Scal {
  double beta;        // ||b||
  double rhsnorm;     // ||S b|| (sFLSQR) or ||S B b|| (sFLSMR)
  double tol;         // relative tolerance of the sketched stop test (0: none)
  double ttol;        // threshold of the true-residual stop test (Dev::resid = 2)
  double wpre;        // ||A z_k|| before orthogonalisation
  double zpre;        // ||B w_{k+1}|| before orthogonalisation
  double Gw[(kMaxEll + 2) * (kMaxEll + 2)];  // <w_i, w_j> by slot
  double Gp[(kMaxEll + 1) * (kMaxEll + 1)];  // <p_i, p_j> by slot
  int halt;           // 1: no further stage may run (stop test, or after a breakdown's LS)
  int klimit;         // last iteration whose basis vector exists (t breakdown)
  int stopped;        // stop test fired
  int breakdown;      // bits: 1 t_{k+1,k+1} = 0, 2 h_{k+1,k} = 0, 4 zero sketched column
  int k_done;         // iterations whose LS has completed
  int happy;          // iteration k with h_{k+1,k} = 0 (0: none)
  int err;            // device-detected error code
  int pad;
};

struct Dev {
  // sizes and parameters
  int m, n, s, ell, maxit, method, tau, sketch, zeta;
  int d_sk;           // length of sketched vectors (m or n)
  int resid;          // 0: no per-iteration true residual; 1: recorded; 2: recorded
                      // and the stop test
  int N;              // SRHT padded length
  int log2L;          // SRHT block length log2
  int nblk;           // SRHT blocks
  int nws;            // SpMV workgroups of this instance (row ranges)
  int nwv;            // vector-stage workgroups of this instance
  int nwmax;          // stride of the per-stage partial-sum buffers
  int nsg;            // sparse-sign sketch gather workgroups of this instance
  int vwA, vwB;       // SpMV lanes per row
  int ntA, ntB;       // 1: CSR-stream reads the operator with non-temporal loads (it
                      // exceeds the last-level cache)
  int vs;             // element stride of W, P, Z, wraw, zraw, x: 1, or the
                      // interleave width when right-hand sides share A and B
  double eps;
  double sk_scale;    // 1/sqrt(zeta) or 1/sqrt(s)
  // operators
  const int *Arp, *Aci; const double *Ava;
  const int *Brp, *Bci; const double *Bva;
  const double *b;
  const int *Apart, *Bpart;    // nnz-balanced row ranges, nws + 1 entries each
  // caller's order of the unknowns (sfk_params.perm): unknown j at position
  // perm[j]; skperm = perm when the sketched vectors are n-vectors (sFLSMR),
  // pinv the inverse (solutions are written back in the caller's order); both
  // NULL without a perm
  const int *skperm, *pinv;
  // SELL-64 copies (SpMV variant 1): slice s holds rows 64 s .. 64 s + 63
  // column-major, entry j of row 64 s + i at soff[s] + 64 j + i (padding:
  // value 0, column 0); slen[s] is a multiple of kSellPad
  int Ansl, Bnsl;
  const int *Asoff, *Aslen, *Ascol; const double *Asval;
  const int *Bsoff, *Bslen, *Bscol; const double *Bsval;
  // 16-bit copies of the column indices of an operator with at most 65536
  // columns (read by CSR-stream and SELL-64 instead of the 32-bit arrays), or
  // nullptr
  const uint16_t *Aci16, *Bci16, *Ascol16, *Bscol16;
  // vectors
  double *W;          // (ell + 2) * m, unnormalised w~_j
  double *P;          // (ell + 1) * n, unnormalised p~_j (unused when tau = I)
  double *Z;          // (maxit + 1) * n, z~_j (column j-1)
  double *wraw;       // kRawSlots * m, A z_k in slot k % kRawSlots
  double *zraw;       // kRawSlots * n, B w_{k+1} in slot k % kRawSlots
  double *x;          // n, current iterate (reweighting) / scratch
  // sketch
  int *sk_rp;         // s + 1   (sparse-sign, transposed: entries per sketch row)
  int *sk_ent;        // zeta * d: column | (negative << 31)
  int *sk_code;       // zeta * d: (row << 1) | negative, per column in draw order
  int *srht_rows;     // s
  unsigned long long *srht_d;  // N / 64 sign words
  double *srht_part;  // nblk * s
  double *SK;         // s * (maxit + 1), sketched columns
  double *skrhs;      // s
  // stage reductions
  double *part;       // kNumPart * kMaxQ * nwmax
  Scal *sc;
  double *sigw;       // maxit + 2: 1 / ||w~_j||
  double *sigp;       // maxit + 2: 1 / ||p~_j||
  double *H;          // (maxit + 1) * maxit, column-major
  double *T;          // (maxit + 1) * (maxit + 1), column-major
  double *rho;        // maxit
  // small least-squares state (Householder QR of the sketched matrix)
  double *V;          // s * maxit reflectors (v_j[j] = 1, zeros above)
  double *tauv;       // maxit
  double *R;          // maxit * maxit, column-major
  double *c;          // s: Q^T rhs
  double *y;          // maxit: y_k (kept current for the reweighting and resid)
  // per-iteration true residual (resid >= 1)
  double *rtrue;      // maxit: ||b - A x_k||
  double *xres;       // n: x_k in the library's order of the unknowns
  // full orthogonalisation (FLSQR / FLSMR, method 2 / 3): the whole bases,
  // orthonormal columns, and the Givens state of the projected problem
  double *Wf;         // (maxit + 1) * m, w_j in column j - 1
  double *Pf;         // (maxit + 1) * n, p_j in column j - 1
  double *fscr;       // sweep partials and projections
  double *gc, *gs;    // maxit rotations
  double *gR;         // maxit * maxit, column-major upper triangular
  double *gg;         // maxit + 1: Q^T (rhs)
  // derivative tape: checkpoints of the w window every `tape` iterations
  int tape;
  double *ck;         // (maxit / tape + 1) * (ell + 2) * m
  // matrix-free parallel-beam operators (SpMV variant 3; the CSR pointers
  // are then NULL): image side, slices, angles, bins, back-projector (0
  // exact transpose, 1 linear interpolation), directions, and per ray its
  // parameter interval inside the image (lmin, lmax; lmin > lmax: misses it)
  int bN, bNz, bNa, bNd, bBack;
  const double *bCos, *bSin;
  double *brl;        // 2 m
  double *mscr;       // m: scratch of the explicit residual
};

// Launch geometry of a batch of instances: the device array of instance
// descriptors and, per stage type, a block -> (instance, workgroup) map.
struct Launch {
  const Dev *devs;
  const int2 *map_spmv, *map_vec, *map_sg, *map_sb, *map_sc;
  int nspmv, nvec, nsg, nsb, nsc;   // grid sizes
  int ninst, smax, maxitmax, tau, vwA, vwB;
  int ellmax;         // largest orthogonalisation window of the instances
};

// Right-hand sides that share one operator pair A, B (a group): the long
// vectors of all of them are interleaved, element i of right-hand side r at
// [i * RS + r], so that one pass over A or B serves every right-hand side and
// each gathered row of the source block is RS contiguous doubles.  The
// per-right-hand-side state (sketch, least squares, coefficients, flags) stays
// in the R instance descriptors devs[0..R).
constexpr int kCoefStride = 16;            // >= kMaxEll + 2
constexpr int kMaxRhs = 64;
constexpr int kXPad = 256;                 // tail padding of the sliced nonzero copy
constexpr int kXcds = 8;                   // L2 domains; workgroup b runs on domain b % 8
constexpr int kSegAlign = 4;               // segments of the sliced copy padded to this many nonzeros
constexpr int kXPadOff = 0x7fffff00;       // offset of a padding nonzero: past any source block
constexpr int kLdsRows = 98304;            // bytes of staged source rows per unit (LDS)
constexpr int kLdsRecs = 3584;             // records per unit (LDS)

// Column-sliced copy of one operator for the shared-operator products.  The
// columns are cut into NS ranges (a multiple of kXcds, each small enough that
// its rows of the source block stay in one L2), and each row's nonzeros in a
// range form a segment.  The workgroups of slice s all run on L2 domain s % 8,
// so every gather of a slice hits the same L2.  Each segment leaves a partial
// row of RS sums in a row-major slot (the partials of row i are slots
// crp[i] .. crp[i + 1] - 1, in slice order); a combine pass adds them.
// one nonzero of the sliced copy: value and byte offset of its source row in
// the interleaved block (column * RS * 8); for the LDS-staged products the
// offset is into the unit's staged block and `pad` is the segment's partial
// slot on a segment's last record (-1 elsewhere)
struct alignas(16) XNz {
  double v;
  int off;
  int pad;
};

struct XOp {
  int rows, cols, NS, nbs, nseg;
  int upb;              // work units per workgroup (one per lane group of a wave)
  const int4 *seg;      // nseg: (row, first, end, slot) into nz, end - first a multiple of
                        // kSegAlign (padding: value 0, offset kXPadOff); slice-major, rows ascending
  const int *spart;     // NS * (nbs * upb + 1): segment range of each work unit of a slice
  const XNz *nz;        // nnz + kXPad (padding: value 0, offset 0)
  const int *crp;       // rows + 1
  double *part;         // nseg * RS, slot-major
  // LDS-staged units (urec != nullptr; record offsets are byte offsets inside
  // the unit's staged block, kLdsRows for padding)
  int nbw;              // workgroups per slice
  const XNz *urec;      // kLdsRecs per unit: the unit's records, then padding (value 0,
                        // offset kLdsRows, slot -1)
  const int *stage;     // kLdsRows / (8 RS) per unit: source rows of the staged block, -1 after
  const int2 *ugrp;     // per unit and lane group: record range relative to the unit's first
  const int *upart;     // NS * (nbw + 1): unit range of each workgroup of a slice
};

struct Grp {
  int R, RS;          // right-hand sides, interleave width (power of two, 8..64)
  int m, n, ell, maxit, tau, nws, nwv;
  double eps;
  const int *Arp, *Aci; const double *Ava;
  const int *Brp, *Bci; const double *Bva;
  const int *Apart, *Bpart;
  double *W;          // (ell + 2) slots of m * RS
  double *P;          // (ell + 1) slots of n * RS (reweighting only)
  double *Z;          // (maxit + 1) columns of n * RS
  double *wraw;       // kRawSlots * m * RS
  double *zraw;       // kRawSlots * n * RS (at least)
  double *x;          // n * RS, x_k for the reweighting
  double *coef;       // RS * kCoefStride: coefficients of the stage about to run
  int *act;           // RS: 1 if the right-hand side takes part in that stage
  double *gx;         // maxit * RS: sigp_{j+1} y_j per right-hand side, [j * RS + r]
  const Dev *devs;    // R instance descriptors (device memory)
  int sliced;         // 1: products through xa / xb; 0: row kernel on the CSR arrays
  XOp xa, xb;         // sliced A and B
};

__device__ __forceinline__ int wslot(const Dev &D, int j) { return j % (D.ell + 2); }
__device__ __forceinline__ int pslot(const Dev &D, int j) { return j % (D.ell + 1); }
// vectors of one instance; element i of each is at [i * D.vs]
__device__ __forceinline__ double *wrawk(const Dev &D, int k) { return D.wraw + (size_t)(k & (kRawSlots - 1)) * D.m * D.vs; }
__device__ __forceinline__ double *zrawk(const Dev &D, int k) { return D.zraw + (size_t)(k & (kRawSlots - 1)) * D.n * D.vs; }
__device__ __forceinline__ double *wvec(const Dev &D, int j) { return D.W + (size_t)wslot(D, j) * D.m * D.vs; }
__device__ __forceinline__ double *zcol(const Dev &D, int j) { return D.Z + (size_t)j * D.n * D.vs; }
__device__ __forceinline__ double *pvec(const Dev &D, int j) {
  // with tau = I the stored basis column z~_j is p~_j itself
  return D.tau == 0 ? zcol(D, j - 1) : D.P + (size_t)pslot(D, j) * D.n * D.vs;
}

}  // namespace sfk
