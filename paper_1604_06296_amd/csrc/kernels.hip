// HIP kernels for gfx950 (CDNA4): loop expansion, projections, products and
// ODE helpers of the TUfRG flow right-hand side (the loop kernel itself is in
// loops.hip).
//
// Every kernel is driven by a table of work items (point, a, b, c): one launch
// covers any set of points with uneven grids and truncations, a single point
// being a batch of one.  The point's tables are read from a device array of
// DevTables; temperatures are read from a per-point device array (so that a
// captured HIP graph can be replayed with new temperatures), and points whose
// flow has stopped are skipped through a per-point device flag.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <climits>
#include <cstdint>

#include "proj_bodies.h"
#include "transforms.h"
#include "tufrg_internal.h"

namespace tufrg {
namespace {

// chi'_mn(q) = sum_j Ebub_{mn,j} ghat(q, S_j) for every momentum, with
// ghat(q, S_j) = sign ghat(r, S_j') of its representative (pack_sym entry of
// the symmetry map), as one contraction over j: rows (channel, q), columns
// mn.  Item (p, row tile of 32, column tile of 64); the representatives'
// harmonics are the sums of their loop slices, or come from fin
// [nirr][2][nsh] (single point).  Each thread owns 2 rows x 4 columns.  Items
// with w = 1 take the rows (channel, representative slot) instead: chi' at the
// orbit representatives only (symmetric states).
constexpr int kExpRows = 32, kExpCols = 64, kExpK = 36;
struct alignas(16) ExpandShared {
  double As[kExpRows][kExpK];
  double Bs[kExpK][kExpCols];
};
// ONE: the launch covers a single point (p = 0), so its descriptor loads need
// not wait for the item's
template <bool ONE>
__device__ __forceinline__ void expand_body(const Batch& b, const int4 item, const double* __restrict__ fin,
                                            double* __restrict__ dchi, ExpandShared& sh) {
  const int p = ONE ? 0 : item.x;
  if (skip_point(b, p)) return;
  const DevTables& d = point_tables<ONE>(b, p);
  auto& As = sh.As;
  auto& Bs = sh.Bs;
  const int nq = d.nq, nsh = d.nsh, nout = 2 * nsh, nff2 = d.nff * d.nff;
  const int r0 = item.y * kExpRows, c0 = item.z * kExpCols;
  const bool reps = item.w != 0;
  const int nrow = reps ? d.nirr : nq;   // rows per channel
  const int tid = threadIdx.x;
  {
    // the coefficient tile first (its loads need the descriptor only), all of
    // the thread's loads in flight together
    constexpr int kB = kExpK * kExpCols / 256;
    double bv[kB];
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      const int e = tid + 256 * i, j = e / kExpCols, mn = c0 + e % kExpCols;
      bv[i] = (j < nsh && mn < nff2) ? d.ebub[(size_t)j * nff2 + mn] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      const int e = tid + 256 * i;
      Bs[e / kExpCols][e % kExpCols] = bv[i];
    }
  }
  {
    // the thread's (up to 5) entries of the row tile, the loop slices of each
    // loaded 4 at a time and added in slice order
    constexpr int kPer = (kExpRows * kExpK + 255) / 256;
    const double* src[kPer];
    bool ok[kPer], neg[kPer];
    double v[kPer];
#pragma unroll
    for (int s5 = 0; s5 < kPer; ++s5) {
      const int e = tid + 256 * s5, rr = e / nsh, j = e % nsh, row = r0 + rr;
      ok[s5] = e < kExpRows * nsh && row < 2 * nrow;
      neg[s5] = false;
      src[s5] = fin;
      v[s5] = 0.0;
      if (ok[s5]) {
        const int ch = row / nrow, q = reps ? d.irr[row % nrow] : row % nrow;
        const int32_t pk = d.symmap[(size_t)q * nsh + j];
        const int slot = pk & 0xffff, oo = ch * nsh + ((pk >> 16) & 0x7f);
        neg[s5] = (pk >> 24) & 1;
        src[s5] = fin ? fin + (size_t)slot * nout + oo : b.ghat + d.ws_gh + (size_t)slot * nout + oo;
      }
    }
    const int nsl = fin ? 1 : d.nsplit;
    const size_t sstride = (size_t)d.nirr * nout;
    for (int sl0 = 0; sl0 < nsl; sl0 += 4) {
      double t[kPer][4];
#pragma unroll
      for (int s5 = 0; s5 < kPer; ++s5)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          t[s5][u] = (ok[s5] && sl0 + u < nsl) ? src[s5][(size_t)(sl0 + u) * sstride] : 0.0;
#pragma unroll
      for (int s5 = 0; s5 < kPer; ++s5)
#pragma unroll
        for (int u = 0; u < 4; ++u) v[s5] += t[s5][u];
    }
#pragma unroll
    for (int s5 = 0; s5 < kPer; ++s5) {
      const int e = tid + 256 * s5;
      if (e < kExpRows * nsh) As[e / nsh][e % nsh] = neg[s5] ? -v[s5] : v[s5];
    }
  }
  __syncthreads();
  const int rr = 2 * (tid >> 4), cc = 4 * (tid & 15);
  double acc[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
  for (int j = 0; j < nsh; ++j) {
    const double a0 = As[rr][j], a1 = As[rr + 1][j];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double bv = Bs[j][cc + c];
      acc[0][c] = fma(a0, bv, acc[0][c]);
      acc[1][c] = fma(a1, bv, acc[1][c]);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int row = r0 + rr + i;
    if (row >= 2 * nrow) continue;
    const int ch = row / nrow, q = reps ? d.irr[row % nrow] : row % nrow;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int mn = c0 + cc + c;
      if (mn < nff2) dchi[(size_t)ch * b.S + d.off + (size_t)q * nff2 + mn] = acc[i][c];
    }
  }
}

__global__ void __launch_bounds__(256)
k_chi_expand(Batch b, const int4* __restrict__ items, const double* __restrict__ fin,
             double* __restrict__ dchi) {
  __shared__ ExpandShared sh;
  expand_body<false>(b, items[blockIdx.x], fin, dchi, sh);
}

// ------------------------------------------------------- projections
// Forward transform (bodies and layout in transforms.h): FP64 on the matrix
// cores, with the LDS staging in dynamic shared memory.
template <int KT>
__global__ void __launch_bounds__(kLoopThreadsMax)
k_dft_fwd_part(Batch b, const int4* __restrict__ items, const double* __restrict__ X) {
  extern __shared__ double smem_fwd[];
  const int4 item = items[blockIdx.x];
  if (skip_point(b, item.x)) return;
  fwd_part_body<KT>(b, b.pts[item.x], item, X, smem_fwd);
}

__global__ void __launch_bounds__(256)
k_bond_basis(Batch b, const int4* __restrict__ items) {
  __shared__ BasisShared sh;
  basis_body<false, false>(b, items[blockIdx.x], sh);
}

// The loop expansion and the bond basis in one launch (they are independent:
// the expansion reads the loop kernel's harmonics, the basis the forward
// transform's partial sums): blocks below nexp expand, the others transform.
template <bool ONE>
__global__ void __launch_bounds__(256)
k_expand_basis(Batch b, const int4* __restrict__ exp_items, int nexp, const int4* __restrict__ basis_items,
               double* __restrict__ dchi) {
  __shared__ union {
    ExpandShared e;
    BasisShared s;
  } sh;
  if ((int)blockIdx.x < nexp) expand_body<ONE>(b, exp_items[blockIdx.x], nullptr, dchi, sh.e);
  else basis_body<ONE, true>(b, basis_items[blockIdx.x - nexp], sh.s);
}

__global__ void __launch_bounds__(64)
k_gather_g2(Batch b, const int4* __restrict__ items, const int2* __restrict__ gent, int cap) {
  __shared__ GatherShared sh;
  const int4 item = items[blockIdx.x];
  if (skip_point(b, item.x)) return;
  gather_load(b, item, gent, cap, threadIdx.x, sh);
  __syncthreads();
  gather_store(b, item, threadIdx.x, sh);
}

// Inverse transform K[ch][l][mn] = sum_k E[l][k] g2[ch][k][mn] in FP64 on the
// matrix cores: item (p, tile of 16 LT momenta l, tile of 64 columns (ch, mn));
// harmonics k in chunks of 16 through LDS; wave w owns 16 columns and LT
// accumulator tiles of v_mfma_f64_16x16x4f64 (16 momenta each; lane layout
// as in the forward transform).  LT is the largest of 4, 2, 1 that still gives
// the launch enough items.  With symmetric states (b.wedge) the rows are the
// orbit representatives irr[r] only.  NC: chunks of 16 harmonics staged
// together (3 for the one-tile form of small points, whose few harmonics
// then pass through LDS in one stage).
template <int LT, bool ONE, int NC = 1>
__global__ void __launch_bounds__(256) k_dft_inv(Batch b, const int4* __restrict__ items) {
  constexpr int TL = 16 * LT, KC = 16 * NC;
  __shared__ double Es[KC][TL + 2];   // [k][l]
  __shared__ double Gs[KC][64 + 2];   // [k][col]
  const int4 item = items[blockIdx.x];
  const int p = ONE ? 0 : item.x;   // ONE: a single-point launch
  if (skip_point(b, p)) return;
  const DevTables& d = point_tables<ONE>(b, p);
  const int nq = d.nq, ncol = d.ncol, nff2 = d.nff * d.nff, N = 3 * nff2;
  const int l0 = item.y * TL, c0 = item.z * 64, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, r16 = lane & 15, k4 = lane >> 4;
  // staging: each chunk's loads are issued together into registers before
  // they go to LDS; a thread stages LT entries of E (16 consecutive harmonics
  // of one momentum per 16 threads) and one column of g2 (rows gk + 4 i)
  const int gc = tid & 63, gk = tid >> 6, gcol = c0 + gc;
  const bool gok = gcol < N;
  const double* gsrc = b.g2 + d.ws_g2 + (gok ? (size_t)(gcol / nff2) * ncol * nff2 + gcol % nff2 : 0);
  f64x4 acc[LT];
#pragma unroll
  for (int t = 0; t < LT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int nrow = b.wedge ? d.nirr : nq;
  int lrow[LT];   // momentum of each staged row (-1 beyond the rows)
#pragma unroll
  for (int i = 0; i < LT; ++i) {
    const int r = l0 + ((tid + 256 * i) >> 4);
    lrow[i] = r < nrow ? (b.wedge ? d.irr[r] : r) : -1;
  }
  // software pipeline: stage c + 1's loads are in flight during stage c's MFMAs
  double ev[NC][LT], gv[NC][4];
  auto load = [&](int k0) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
      for (int i = 0; i < LT; ++i) {
        const int k = k0 + 16 * c + ((tid + 256 * i) & 15);
        ev[c][i] = (lrow[i] >= 0 && k < ncol) ? d.eph[(size_t)lrow[i] * ncol + k] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = k0 + 16 * c + gk + 4 * i;
        gv[c][i] = (gok && k < ncol) ? gsrc[(size_t)k * nff2] : 0.0;
      }
    }
  };
  load(0);
  for (int k0 = 0; k0 < ncol; k0 += KC) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
      for (int i = 0; i < LT; ++i) {
        const int e = tid + 256 * i;
        Es[16 * c + (e & 15)][e >> 4] = ev[c][i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) Gs[16 * c + gk + 4 * i][gc] = gv[c][i];
    }
    __syncthreads();
    if (k0 + KC < ncol) load(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const double bv = Gs[kk + k4][16 * w + r16];
#pragma unroll
      for (int t = 0; t < LT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(Es[kk + k4][16 * t + r16], bv, acc[t], 0, 0, 0);
    }
    __syncthreads();
  }
  double* K = b.kinv64 + d.ws_k;
  const int col = c0 + 16 * w + r16;
  if (col >= N) return;
  const int ch = col / nff2, mn = col % nff2;
#pragma unroll
  for (int t = 0; t < LT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = l0 + 16 * t + 4 * j + k4;
      if (r < nrow) K[((size_t)ch * nq + (b.wedge ? d.irr[r] : r)) * nff2 + mn] = acc[t][j];
    }
}

// ======================================================= mixed precision
// (BF16 hi/lo split helpers and the split-precision forward body in
// transforms.h.)
template <int KT>
__global__ void __launch_bounds__(kLoopThreadsMax)
k_dft_fwd_mix(Batch b, const int4* __restrict__ items, const double* __restrict__ X) {
  extern __shared__ double smem_fwd[];
  const int4 item = items[blockIdx.x];
  if (skip_point(b, item.x)) return;
  fwd_mix_body<KT>(b, b.pts[item.x], item, X, smem_fwd);
}

// Inverse transform in split precision: K[ch][l][mn] = sum_k E[l][k] g2[ch][k][mn]
// with FP32 accumulation of the three BF16 split products, stored in FP32.
// Item (p, tile of 16 LT momenta l, tile of 64 columns); wave w owns 16
// columns and LT accumulator tiles of 16 momenta.  The whole harmonic range
// (at most 20 quads of 4) is staged in LDS at once, with all loads in flight
// together: the block's rows of the pre-split phase table (laid out [l][kEpad],
// zero beyond Nq, rows padded to a multiple of 64) as hi and lo quads, and its
// columns of g2, split to hi and lo quads as they are staged.
template <int LT, bool ONE>
__global__ void __launch_bounds__(256)
k_dft_inv_mix(Batch b, const int4* __restrict__ items) {
  constexpr int TL = 16 * LT, QR = kEpad / 4;
  __shared__ bf16x4 Eh[TL][QR + 1], El[TL][QR + 1];
  __shared__ bf16x4 Gh[QR][64 + 1], Gl[QR][64 + 1];
  const int4 item = items[blockIdx.x];
  const int p = ONE ? 0 : item.x;   // ONE: a single-point launch
  if (skip_point(b, p)) return;
  const DevTables& d = point_tables<ONE>(b, p);
  const int nq = d.nq, ncol = d.ncol, nff2 = d.nff * d.nff, N = 3 * nff2;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, k4 = lane >> 4;
  const int l0 = item.y * TL, c0 = item.z * 64;
  const int nk = (ncol + 15) / 16 * 4;   // quads in use
  // staging: E entries tid + 256 i of [TL][QR]; g2 column gc, quads gq + 4 i
  constexpr int EPT = (TL * QR + 255) / 256;
  const bf16x4* ehq = reinterpret_cast<const bf16x4*>(d.ephr_hi);
  const bf16x4* elq = reinterpret_cast<const bf16x4*>(d.ephr_lo);
  bf16x4 eh[EPT], el[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + 256 * i, r = e / QR, q = e % QR, rr = l0 + r;
    // with symmetric states (b.wedge) the rows are the orbit representatives
    const int lsrc = b.wedge ? (rr < d.nirr && e < TL * QR ? d.irr[rr] : -1) : rr;
    const bool ok = e < TL * QR && q < nk && lsrc >= 0;
    const size_t src = (size_t)(ok ? lsrc : 0) * QR + q;
    eh[i] = ok ? ehq[src] : bf16x4{0, 0, 0, 0};
    el[i] = ok ? elq[src] : bf16x4{0, 0, 0, 0};
  }
  const int gc = tid & 63, gq = tid >> 6, gcol = c0 + gc;
  const bool gok = gcol < N;
  const double* gsrc = b.g2 + d.ws_g2 + (gok ? (size_t)(gcol / nff2) * ncol * nff2 + gcol % nff2 : 0);
  double gv[QR / 4][4];
#pragma unroll
  for (int i = 0; i < QR / 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = 4 * (gq + 4 * i) + j;
      gv[i][j] = (gok && k < ncol) ? gsrc[(size_t)k * nff2] : 0.0;
    }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + 256 * i;
    if (e < TL * QR) {
      Eh[e / QR][e % QR] = eh[i];
      El[e / QR][e % QR] = el[i];
    }
  }
#pragma unroll
  for (int i = 0; i < QR / 4; ++i) {
    bf16x4 qh, ql;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      unsigned short hi, lo;
      split_bf16(gv[i][j], hi, lo);
      qh[j] = (short)hi;
      ql[j] = (short)lo;
    }
    Gh[gq + 4 * i][gc] = qh;
    Gl[gq + 4 * i][gc] = ql;
  }
  __syncthreads();
  f32x4 acc[LT];
#pragma unroll
  for (int t = 0; t < LT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  // steps of 32 harmonics on v_mfma_f32_16x16x32_bf16 (lane (r16, k4):
  // quads q0 + 2 k4, q0 + 2 k4 + 1), a last step of 16 on the 16x16x16 form
  int q0 = 0;
  for (; q0 + 8 <= nk; q0 += 8) {
    const int q = q0 + 2 * k4;
    const bf16x8 bh = quad_pair(Gh[q][16 * w + r16], Gh[q + 1][16 * w + r16]);
    const bf16x8 bl = quad_pair(Gl[q][16 * w + r16], Gl[q + 1][16 * w + r16]);
#pragma unroll
    for (int t = 0; t < LT; ++t) {
      const bf16x8 ah = quad_pair(Eh[16 * t + r16][q], Eh[16 * t + r16][q + 1]);
      const bf16x8 al = quad_pair(El[16 * t + r16][q], El[16 * t + r16][q + 1]);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[t], 0, 0, 0);
    }
  }
  if (q0 < nk) {
    const int q = q0 + k4;
    const bf16x4 bh = Gh[q][16 * w + r16], bl = Gl[q][16 * w + r16];
#pragma unroll
    for (int t = 0; t < LT; ++t) {
      const bf16x4 ah = Eh[16 * t + r16][q], al = El[16 * t + r16][q];
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[t], 0, 0, 0);
    }
  }
  const int col = c0 + 16 * w + r16;
  if (col >= N) return;
  const int ch = col / nff2, mn = col % nff2;
  float* K = b.kinv + d.ws_k;
#pragma unroll
  for (int t = 0; t < LT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = l0 + 16 * t + 4 * k4 + j;
      if (r < (b.wedge ? d.nirr : nq)) K[((size_t)ch * nq + (b.wedge ? d.irr[r] : r)) * nff2 + mn] = acc[t][j];
    }
}

// Assembly of eqns. proj_VP/VC/VD and the products of eqns. matmul-P/C/D in
// precision R (double, or float for the mixed form); item (p, l):
//   V^P = U e0e0 - P + K^P,  V^C = U e0e0 + C + K^C,  V^D = U e0e0 + D + K^D
//   dP = V^P chi'pp V^P, dC = -V^C chi'ph V^C,
//   dD = (W chi'ph W - V^C chi'ph V^C)/2 with W = 2 V^D - V^C (the SU(2) form
//   of eqn. matmul-D: 2 dD - dC = W chi'ph W).
// K is the inverse transform (unused without cross terms); X and the loops
// are FP64; the output is scale * dX/dT (mode 1; scale = T, i.e. dX/ds with
// s = ln T, if scale_T, else 1) or V (mode 0), in FP64.  With symmetric
// states (b.wedge) the item is (p, representative l, its slot) and the result
// goes to every member q of the orbit as Y(q)_mn = s_m s_n Y(l)_{pi(m) pi(n)}
// (the point-group law of the form factors; exact sign copies).  STAGE
// (mode 1, sn.nk > 0): every element of dX also forms its element of the next
// Runge-Kutta stage as it is written (a form of its own, so that plain
// right-hand sides keep the smaller register footprint).
template <typename R, bool ONE, bool STAGE>
__global__ void __launch_bounds__(256)
k_products(Batch b, const int4* __restrict__ items, const double* __restrict__ X, const R* __restrict__ Kall,
           double* __restrict__ out, int mode, int cross, int scale_T, StageNext sn) {
  const int4 item = items[blockIdx.x];
  const int p = ONE ? 0 : item.x;   // ONE: a single-point launch
  if (skip_point(b, p)) return;
  const DevTables& d = point_tables<ONE>(b, p);
  const int nff = d.nff, nff2 = nff * nff, nq = d.nq;
  const int l = item.y;
  const double scale = scale_T ? b.Tp[p] : 1.0;
  const size_t S = (size_t)b.S;
  const R* K = Kall + d.ws_k;
  // element e of [3][S] gets the slope value v and, with a next stage,
  // sn.out[e] = X[e] + h (sum_{j < nk-1} coef_j k_j[e] + coef_{nk-1} v):
  // stage_part(e, x0, a) reads X[e] and forms the partial sum a over the
  // slopes already known, stage_put completes it with v
  const bool stage = STAGE && mode == 1 && sn.nk > 0;
  const double hstep = stage ? (sn.hp != nullptr ? sn.hp[p] : sn.h) : 0.0;
  auto stage_part = [&](size_t e, double& x0, double& a) {
    double kv[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) kv[j] = j + 1 < sn.nk ? sn.k[j][e] : 0.0;
    x0 = sn.X[e];
    a = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (j + 1 < sn.nk) a = fma(sn.coef[j], kv[j], a);
  };
  auto stage_put = [&](size_t e, double v, double x0, double a) {
    sn.out[e] = fma(hstep, fma(sn.coef[sn.nk - 1], v, a), x0);
  };
  // shared memory [10][nff2]: the second products T2 take the loops' rows
  // (read only by the first products) and one row more, after a barrier;
  // on the FP64 matrix-core path the first products stay in registers and
  // T2 takes their rows (no barrier between the two products)
  extern __shared__ double smem_prod[];
  R* Vs = reinterpret_cast<R*>(smem_prod);   // [3][nff2]
  R* Wm = Vs + 3 * nff2;                    // [nff2]
  R* T1 = Wm + nff2;                        // [3][nff2]
  R* Ch = T1 + 3 * nff2;                    // [2][nff2]
  R* T2 = (sizeof(R) == 8 && nff <= 16) ? T1 : Ch;   // [3][nff2]
  // symmetric states: the representative's orbit (at most 8 members), each
  // member's q and form-factor permutation, staged with the block's loads
  __shared__ int orb_q_s[8];
  __shared__ int32_t orb_p_s[8][32];
  int orb_n = 0;
  if (b.wedge) {
    const int e0 = d.orb_start[item.z];
    orb_n = d.orb_start[item.z + 1] - e0;
    for (int i = threadIdx.x; i < orb_n * nff; i += blockDim.x) {
      const int e = i / nff, m = i % nff;
      orb_p_s[e][m] = d.tperm[(size_t)d.orb_tr[e0 + e] * nff + m];
    }
    if ((int)threadIdx.x < orb_n) orb_q_s[threadIdx.x] = d.orb_q[e0 + threadIdx.x];
  }
  // the thread's entries mn = tid + 256 h (h < 2; 256 threads, nff^2 <= 441):
  // all of their loads in flight together, then V (and W, the loops) to LDS
  double xv[2][3], kv[2][3], cv[2][2];
  double sx[2][3], sa[2][3];   // the next stage's X and partial sums (own elements)
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int mn = threadIdx.x + 256 * h;
    const bool ok = mn < nff2;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      xv[h][ch] = ok ? X[ch * S + d.off + (size_t)l * nff2 + mn] : 0.0;
      kv[h][ch] = (ok && cross) ? (double)K[((size_t)ch * nq + l) * nff2 + mn] : 0.0;
    }
#pragma unroll
    for (int ch = 0; ch < 2; ++ch)
      cv[h][ch] = (ok && mode != 0) ? b.dchi[(size_t)ch * S + d.off + (size_t)l * nff2 + mn] : 0.0;
  }
  // the next stage's operands after the products' own (they are needed last)
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int mn = threadIdx.x + 256 * h;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      sx[h][ch] = sa[h][ch] = 0.0;
      if (mn < nff2 && stage && !b.wedge) stage_part(ch * S + d.off + (size_t)l * nff2 + mn, sx[h][ch], sa[h][ch]);
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int mn = threadIdx.x + 256 * h;
    if (mn >= nff2) continue;
    const R bare = (mn == 0) ? (R)d.U : (R)0;
    R v[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const R own = (R)xv[h][ch];
      v[ch] = bare + (ch == 0 ? -own : own) + (R)kv[h][ch];
    }
    if (mode == 0 && !b.wedge) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) out[(size_t)ch * S + d.off + (size_t)l * nff2 + mn] = (double)v[ch];
      continue;
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) Vs[ch * nff2 + mn] = v[ch];
    Wm[mn] = (R)2 * v[2] - v[1];
    Ch[mn] = (R)cv[h][0];
    Ch[nff2 + mn] = (R)cv[h][1];
  }
  if (mode == 0 && !b.wedge) return;
  __syncthreads();
  // the orbit of the representative (staged above; the barrier above or in
  // the products has made it visible)
  auto orbit = [&](auto&& value) {
    for (int w = threadIdx.x; w < orb_n * nff2; w += blockDim.x) {
      const int e = w / nff2, mn = w % nff2;
      const int a = orb_p_s[e][mn / nff], c = orb_p_s[e][mn % nff];
      const double sg = ((a ^ c) >> 8) & 1 ? -1.0 : 1.0;
      value(d.off + (size_t)orb_q_s[e] * nff2 + mn, (a & 0xff) * nff + (c & 0xff), sg);
    }
  };
  if (mode == 0) {
    orbit([&](size_t o, int src, double sg) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) out[(size_t)ch * S + o] = sg * (double)Vs[ch * nff2 + src];
    });
    return;
  }
  const R* VP = Vs;
  const R* VC = Vs + nff2;
  // N_ff <= 16: the six products on the matrix cores, one 16 x 16 tile of
  // the zero-padded matrices per wave (v_mfma_f64_16x16x4f64, or
  // v_mfma_f32_16x16x4f32 for the FP32 form; lane l holds A[l%16][k0 + l/16]
  // and B[k0 + l/16][l%16]).  Beyond, padding to 32 would triple the work
  // (the FP64 matrix and vector peaks are equal), so register tiles.
  if (nff <= 16) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    const int r16 = lane & 15, k4 = lane >> 4;
    auto mm_tile = [&](const R* A, const R* B, R* C) {
      if constexpr (sizeof(R) == 8) {
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < 16; k0 += 4) {
          const int k = k0 + k4;
          const double av = (r16 < nff && k < nff) ? (double)A[r16 * nff + k] : 0.0;
          const double bv = (k < nff && r16 < nff) ? (double)B[k * nff + r16] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = 4 * j + k4;   // f64 result layout: D[4j + l/16][l%16]
          if (r < nff && r16 < nff) C[r * nff + r16] = (R)acc[j];
        }
      } else {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < 16; k0 += 4) {
          const int k = k0 + k4;
          const float av = (r16 < nff && k < nff) ? (float)A[r16 * nff + k] : 0.f;
          const float bv = (k < nff && r16 < nff) ? (float)B[k * nff + r16] : 0.f;
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = 4 * k4 + j;   // f32 result layout: D[4(l/16) + j][l%16]
          if (r < nff && r16 < nff) C[r * nff + r16] = (R)acc[j];
        }
      }
    };
    // first products T1 = (chi'pp VP, chi'ph VC, chi'ph W); second T2 = (VP T1_0, VC T1_1, W T1_2)
    if constexpr (sizeof(R) == 8) {
      // FP64: a wave's first product stays in its registers, since the f64
      // result layout (row 4j + l/16 of column l%16 in element j) is the
      // layout of the second product's B operand for the k rows 4j .. 4j + 3
      for (int which = wv; which < 3; which += nwv) {
        const R* V1 = which == 0 ? VP : (which == 1 ? VC : Wm);
        const R* A1 = Ch + (which == 0 ? 0 : nff2);
        f64x4 t1 = {0.0, 0.0, 0.0, 0.0}, t2 = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < 16; k0 += 4) {
          const int k = k0 + k4;
          const double av = (r16 < nff && k < nff) ? (double)A1[r16 * nff + k] : 0.0;
          const double bv = (k < nff && r16 < nff) ? (double)V1[k * nff + r16] : 0.0;
          t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, t1, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = 4 * j + k4;
          const double av = (r16 < nff && k < nff) ? (double)V1[r16 * nff + k] : 0.0;
          t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, t1[j], t2, 0, 0, 0);
        }
        R* C = T2 + which * nff2;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = 4 * j + k4;
          if (r < nff && r16 < nff) C[r * nff + r16] = (R)t2[j];
        }
      }
    } else {
      for (int which = wv; which < 3; which += nwv)
        mm_tile(Ch + (which == 0 ? 0 : nff2), which == 0 ? VP : (which == 1 ? VC : Wm), T1 + which * nff2);
      __syncthreads();
      for (int which = wv; which < 3; which += nwv)
        mm_tile(which == 0 ? VP : (which == 1 ? VC : Wm), T1 + which * nff2, T2 + which * nff2);
    }
  } else {
    // 3 x 2 register tiles, k unrolled by 7: at N_ff = 21 the three products
    // of a round are 231 tiles, one per thread of the block (measured at
    // 48x48 against 3 x 3 tiles: FP64 32.6 -> 28.4 us, FP32 27.0 -> 25.3 us;
    // 7 x 3 tiles, fewer LDS reads per FMA on a single wave, ran slower);
    // every output sums k in order, so the bits do not depend on the tiling
    constexpr int TM = 3, TN = 2;
    const int ntm = (nff + TM - 1) / TM, ntn = (nff + TN - 1) / TN;
    auto product = [&](const R* A, const R* B, R* C, int ti, int tj) {
      const int m0 = TM * ti, n0 = TN * tj;
      R c[TM][TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) c[i][j] = 0;
#pragma unroll 7
      for (int k = 0; k < nff; ++k) {
        R a[TM], bb[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = m0 + i < nff ? A[(m0 + i) * nff + k] : (R)0;
#pragma unroll
        for (int j = 0; j < TN; ++j) bb[j] = n0 + j < nff ? B[k * nff + n0 + j] : (R)0;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) c[i][j] = fma(a[i], bb[j], c[i][j]);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          if (m0 + i < nff && n0 + j < nff) C[(m0 + i) * nff + n0 + j] = c[i][j];
    };
    const int nw = 3 * ntm * ntn;
    for (int w = threadIdx.x; w < nw; w += blockDim.x) {
      const int which = w / (ntm * ntn), ti = w / ntn % ntm, tj = w % ntn;
      product(Ch + (which == 0 ? 0 : nff2), which == 0 ? VP : (which == 1 ? VC : Wm), T1 + which * nff2, ti, tj);
    }
    __syncthreads();
    for (int w = threadIdx.x; w < nw; w += blockDim.x) {
      const int which = w / (ntm * ntn), ti = w / ntn % ntm, tj = w % ntn;
      product(which == 0 ? VP : (which == 1 ? VC : Wm), T1 + which * nff2, T2 + which * nff2, ti, tj);
    }
  }
  __syncthreads();
  if (b.wedge) {
    orbit([&](size_t o, int w, double sg) {
      const double v[3] = {sg * (scale * (double)T2[w]), sg * (-scale * (double)T2[nff2 + w]),
                           sg * (0.5 * scale * ((double)T2[2 * nff2 + w] - (double)T2[nff2 + w]))};
      double x0[3], a[3];
      if (stage) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) stage_part(ch * S + o, x0[ch], a[ch]);
      }
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        out[ch * S + o] = v[ch];
        if (stage) stage_put(ch * S + o, v[ch], x0[ch], a[ch]);
      }
    });
    return;
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int w = threadIdx.x + 256 * h;   // the elements whose operands were loaded first
    if (w >= nff2) continue;
    const size_t o = d.off + (size_t)l * nff2 + w;
    const double v[3] = {scale * (double)T2[w], -scale * (double)T2[nff2 + w],
                         0.5 * scale * ((double)T2[2 * nff2 + w] - (double)T2[nff2 + w])};
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      out[ch * S + o] = v[ch];
      if (stage) stage_put(ch * S + o, v[ch], sx[h][ch], sa[h][ch]);
    }
  }
}

// ----------------------------------------------------------- ODE helpers
// Segment items (p, channel, chunk): kSeg consecutive elements of one point's
// channel block in a [3][S] array.
struct SlopeSet {
  const double* k[7];
  double coef[7];
};

__device__ __forceinline__ bool seg_range(const Batch& b, const int4& it, size_t& base, int& n) {
  const DevTables& d = b.pts[it.x];
  const int64_t len = (int64_t)d.nq * d.nff * d.nff;
  const int64_t s0 = (int64_t)it.z * kSeg;
  if (s0 >= len) return false;
  n = (int)min((int64_t)kSeg, len - s0);
  base = (size_t)it.y * b.S + d.off + s0;
  return true;
}

// out = X + h sum_j coef_j k_j; frozen points untouched when skip_frozen.
// Every thread holds kSeg / 256 elements of the segment and issues all their
// loads (X and the NK slopes) before the arithmetic.  out may be X (the RK4
// update writes in place: each element is read and written by one thread), so
// neither carries __restrict__.
constexpr int kSegPer = kSeg / 256;
template <int NK>
__global__ void __launch_bounds__(256)
k_axpy(Batch b, const int4* __restrict__ items, const double* X, SlopeSet ks, double h,
       double* out, int skip_frozen, const double* __restrict__ hp) {
  const int4 it = items[blockIdx.x];
  if (skip_frozen && skip_point(b, it.x)) return;
  if (hp != nullptr) h = hp[it.x];
  size_t base;
  int n;
  if (!seg_range(b, it, base, n)) return;
  double xv[kSegPer], kv[kSegPer][NK];
#pragma unroll
  for (int u = 0; u < kSegPer; ++u) {
    const int i = threadIdx.x + 256 * u;
    const size_t e = base + (i < n ? i : 0);
    xv[u] = X[e];
#pragma unroll
    for (int j = 0; j < NK; ++j) kv[u][j] = ks.k[j][e];
  }
#pragma unroll
  for (int u = 0; u < kSegPer; ++u) {
    const int i = threadIdx.x + 256 * u;
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < NK; ++j) acc = fma(ks.coef[j], kv[u][j], acc);
    if (i < n) out[base + i] = fma(h, acc, xv[u]);
  }
}

// per-point max |x| as the ordered bit pattern of a non-negative double (NaN
// sorts above +inf, so a non-finite state is seen)
__global__ void __launch_bounds__(256)
k_maxabs(Batch b, const int4* __restrict__ items, const double* __restrict__ X,
         unsigned long long* __restrict__ words) {
  __shared__ unsigned long long red[256];
  const int4 it = items[blockIdx.x];
  unsigned long long m = 0ull;
  size_t base;
  int n;
  if (!skip_point(b, it.x) && seg_range(b, it, base, n)) {
    double xv[kSegPer];
#pragma unroll
    for (int u = 0; u < kSegPer; ++u) {
      const int i = threadIdx.x + 256 * u;
      xv[u] = X[base + (i < n ? i : 0)];
    }
#pragma unroll
    for (int u = 0; u < kSegPer; ++u) {
      unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(xv[u]));
      if (xv[u] != xv[u]) bits = 0x7ff8000000000000ull;
      if ((int)threadIdx.x + 256 * u < n) m = bits > m ? bits : m;
    }
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && red[threadIdx.x + s] > red[threadIdx.x])
      red[threadIdx.x] = red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != 0ull) atomicMax(words + it.x, red[0]);
}

// The first local flat index (channel, q, m, n) of point p whose |x| has the
// bit pattern words[p] (its max|x| from k_maxabs, NaN ordered as there):
// atomic minimum into first[p]; segment items as k_maxabs.
__global__ void __launch_bounds__(256)
k_first_max(Batch b, const int4* __restrict__ items, const double* __restrict__ X,
            const unsigned long long* __restrict__ words, int* __restrict__ first) {
  const int4 it = items[blockIdx.x];
  size_t base;
  int n;
  if (skip_point(b, it.x) || !seg_range(b, it, base, n)) return;
  const DevTables& d = b.pts[it.x];
  const int len = d.nq * d.nff * d.nff;
  const unsigned long long target = words[it.x];
  int best = INT_MAX;
#pragma unroll
  for (int u = 0; u < kSegPer; ++u) {
    const int i = threadIdx.x + 256 * u;
    if (i < n) {
      const double v = X[base + i];
      unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(v));
      if (v != v) bits = 0x7ff8000000000000ull;
      if (bits == target) best = min(best, it.y * len + it.z * kSeg + i);
    }
  }
  if (best != INT_MAX) atomicMin(first + it.x, best);
}

// The last stage of a Dormand-Prince step in one pass: y5 = y0 + h sum_j b5_j k_j
// (as k_axpy<7>); per segment the partial sum of ((h sum_j e_j k_j) / (atol +
// rtol max(|y0|,|y5|)))^2 in a fixed order (each thread's elements in turn,
// then a tree: deterministic); and the point's max |y5| (as k_maxabs, into
// word p of max_out).
struct Coef7 {
  double c[7];
};
__global__ void __launch_bounds__(256)
k_dp_final(Batch b, const int4* __restrict__ items, const double* __restrict__ y0, SlopeSet ks, Coef7 e,
           double h, double rtol, double atol, double* __restrict__ y5, double* __restrict__ red_out,
           unsigned long long* __restrict__ max_out, const double* __restrict__ hp) {
  __shared__ double red[256];
  __shared__ unsigned long long mred[256];
  const int4 it = items[blockIdx.x];
  if (skip_point(b, it.x)) {
    if (threadIdx.x == 0) red_out[blockIdx.x] = 0.0;
    return;
  }
  if (hp != nullptr) h = hp[it.x];
  double acc = 0.0;
  unsigned long long m = 0ull;
  size_t base;
  int n;
  if (seg_range(b, it, base, n)) {
    double av[kSegPer], kv[kSegPer][7];
#pragma unroll
    for (int u = 0; u < kSegPer; ++u) {
      const int i = threadIdx.x + 256 * u;
      const size_t idx = base + (i < n ? i : 0);
      av[u] = y0[idx];
#pragma unroll
      for (int j = 0; j < 7; ++j) kv[u][j] = ks.k[j][idx];
    }
#pragma unroll
    for (int u = 0; u < kSegPer; ++u) {
      const int i = threadIdx.x + 256 * u;
      double a5 = 0.0, er = 0.0;
#pragma unroll
      for (int j = 0; j < 7; ++j) a5 = fma(ks.coef[j], kv[u][j], a5);
#pragma unroll
      for (int j = 0; j < 7; ++j) er = fma(e.c[j], kv[u][j], er);
      const double x5 = fma(h, a5, av[u]);
      er *= h;
      const double sc = atol + rtol * fmax(fabs(av[u]), fabs(x5));
      const double r = er / sc;
      unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(x5));
      if (x5 != x5) bits = 0x7ff8000000000000ull;
      if (i < n) {
        y5[base + i] = x5;
        acc = fma(r, r, acc);
        m = bits > m ? bits : m;
      }
    }
  }
  red[threadIdx.x] = acc;
  mred[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[threadIdx.x] += red[threadIdx.x + s];
      if (mred[threadIdx.x + s] > mred[threadIdx.x]) mred[threadIdx.x] = mred[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    red_out[blockIdx.x] = red[0];
    if (mred[0] != 0ull) atomicMax(max_out + it.x, mred[0]);
  }
}

// Step control of the adaptive flow, one block per point (the Dormand-Prince
// 5(4) rules of the flow options: RMS error norm of the attempt, accepted
// when <= 1; step factor 0.9 err^(-1/5) in [0.2, 5]; stop after an accepted
// step with max|X| > xmax, at s_end, on a non-finite error, or when
// max_steps attempts are used up).  The error partial sums of the point's
// segments are added in a fixed order: thread i sums partials i, i + 256, ...
// in turn, then a fixed tree over the threads.  The next attempt's step is
// clipped so that it does not pass s_end.
__global__ void __launch_bounds__(256) k_dp_control(DpControl c) {
  __shared__ double red[256];
  const int p = blockIdx.x;
  const int status = c.st[p].status;
  if (status != 0) {
    if (threadIdx.x == 0) {
      c.max_words[p] = 0ull;
      c.st[p].accept = 0;   // the stopping step's state was taken by the last acceptance
    }
    return;
  }
  const int2 sg = c.seg[p];
  double acc = 0.0;
  for (int i = threadIdx.x; i < sg.y; i += 256) acc += c.red[sg.x + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  DpState st = c.st[p];
  const unsigned long long mw = c.max_words[p];
  c.max_words[p] = 0ull;
  const double err = sqrt(red[0] / c.n_el[p]);
  st.err = err;
  st.accept = 0;
  ++st.n_att;
  if (!isfinite(err)) {
    st.status = TUFRG_FLOW_NONFINITE;
    st.s0 = st.s;
    st.m0 = st.m1;
    st.s1 = st.s + st.h;
    st.m1 = __longlong_as_double(0x7ff8000000000000ll);
  } else {
    if (err <= 1.0) {
      st.accept = 1;
      ++st.n_acc;
      st.s0 = st.s1;
      st.m0 = st.m1;
      st.s = st.s + st.h;
      st.s1 = st.s;
      st.m1 = __longlong_as_double((long long)mw);
      if (st.m1 > c.xmax) st.status = TUFRG_FLOW_DIVERGED;
      else if (st.s <= c.s_end + 1e-15) st.status = TUFRG_FLOW_REACHED_TMIN;
    }
    const double fac = err == 0.0 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(err, -0.2)));
    st.h *= fac;
    if (st.status == 0 && st.n_att >= c.max_steps) st.status = TUFRG_FLOW_MAX_STEPS;
    if (st.s + st.h < c.s_end) st.h = c.s_end - st.s;
  }
  if (st.status != 0) c.frozen[p] = 1;
  c.s_arr[p] = st.s;
  c.h_arr[p] = st.h;
  c.st[p] = st;
  if (c.status_out != nullptr) c.status_out[p] = st.status;
}

// y = y5 and k0 = k6 (first same as last) for the points whose attempt was
// accepted; then, for every point still flowing (accepted or not), the first
// stage of its next attempt, stage1 = y + h (a10 k0) with the step the
// control has just set (the operations of k_axpy<1>); segment items as k_axpy
__global__ void __launch_bounds__(256)
k_dp_accept(Batch b, const int4* __restrict__ items, const DpState* __restrict__ st, const double* __restrict__ y5,
            const double* __restrict__ k6, double* __restrict__ y, double* __restrict__ k0, double a10,
            const double* __restrict__ h_arr, double* __restrict__ stage1) {
  const int4 it = items[blockIdx.x];
  const bool acc = st[it.x].accept != 0;
  const bool flowing = !skip_point(b, it.x);
  if (!acc && !flowing) return;
  size_t base;
  int n;
  if (!seg_range(b, it, base, n)) return;
  const double h = flowing ? h_arr[it.x] : 0.0;
  double yv[kSegPer], kv[kSegPer];
#pragma unroll
  for (int u = 0; u < kSegPer; ++u) {
    const int i = threadIdx.x + 256 * u;
    const size_t e = base + (i < n ? i : 0);
    yv[u] = acc ? y5[e] : y[e];
    kv[u] = acc ? k6[e] : k0[e];
  }
#pragma unroll
  for (int u = 0; u < kSegPer; ++u) {
    const int i = threadIdx.x + 256 * u;
    if (i < n) {
      if (acc) {
        y[base + i] = yv[u];
        k0[base + i] = kv[u];
      }
      if (flowing) stage1[base + i] = fma(h, a10 * kv[u], yv[u]);
    }
  }
}

// Tp[p] = exp(s[p] + c h[p]) (stage temperatures of the adaptive flow)
__global__ void k_set_T_sh(double* Tp, int npts, const double* __restrict__ s_arr, const double* __restrict__ h_arr,
                           double c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < npts) Tp[i] = exp(fma(c, h_arr[i], s_arr[i]));
}

// Dense projection operator (TUFRG_DENSE_PROJECTION, small contexts): the
// cross terms K of the projections as one matrix A of the point's state,
// K_i = sum_j A_ij X_j over the point's local index i = ch Nq Nff^2 + q Nff^2 +
// mn (the layout of K), A stored column-major (column j = K of the unit state
// e_j).  Item (p, tile of 256 rows, split of kDenseCols columns): the partial
// sum over the split's columns, each thread one row (column loads coalesced
// across the block, the split's X values staged in LDS).
constexpr int kDenseCols = 64;
__global__ void __launch_bounds__(256)
k_dense_part(Batch b, const int4* __restrict__ items, const double* __restrict__ X) {
  __shared__ double xs[kDenseCols];
  const int4 it = items[blockIdx.x];
  if (skip_point(b, it.x)) return;
  const DevTables& d = b.pts[it.x];
  const int64_t nqn = (int64_t)d.nq * d.nff * d.nff, N = 3 * nqn;
  const int64_t j0 = (int64_t)it.z * kDenseCols;
  const int nj = (int)min((int64_t)kDenseCols, N - j0);
  if ((int)threadIdx.x < nj) {
    const int64_t j = j0 + threadIdx.x;
    xs[threadIdx.x] = X[(j / nqn) * b.S + d.off + j % nqn];
  }
  __syncthreads();
  const int64_t i = (int64_t)it.y * 256 + threadIdx.x;
  if (i >= N) return;
  const double* a = d.dense_A + j0 * N + i;
  double acc = 0.0;
  int j = 0;
  for (; j + 4 <= nj; j += 4) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = a[(int64_t)(j + u) * N];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = fma(v[u], xs[j + u], acc);
  }
  for (; j < nj; ++j) acc = fma(a[(int64_t)j * N], xs[j], acc);
  double* part = b.dense_ws + d.ws_dp;
  part[(int64_t)it.z * N + i] = acc;
}

// K_i = the splits' partial sums added in split order; item (p, tile of 256 rows)
__global__ void __launch_bounds__(256)
k_dense_sum(Batch b, const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  if (skip_point(b, it.x)) return;
  const DevTables& d = b.pts[it.x];
  const int64_t N = 3 * (int64_t)d.nq * d.nff * d.nff;
  const int64_t i = (int64_t)it.y * 256 + threadIdx.x;
  if (i >= N) return;
  const double* part = b.dense_ws + d.ws_dp + i;
  double acc = 0.0;
  int s = 0;
  for (; s + 4 <= d.dense_splits; s += 4) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = part[(int64_t)(s + u) * N];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += v[u];
  }
  for (; s < d.dense_splits; ++s) acc += part[(int64_t)s * N];
  b.kinv64[d.ws_k + i] = acc;
}

// X[prev] = 0, X[cur] = 1 (the unit states that probe the dense operator)
__global__ void k_set_unit(double* X, int64_t prev, int64_t cur) {
  if (threadIdx.x == 0) {
    if (prev >= 0) X[prev] = 0.0;
    if (cur >= 0) X[cur] = 1.0;
  }
}

// Largest deviation of a state from the C4v covariance law, per point:
// max over channels, orbit members q of representative r and (m, n) of
// |X(q)_mn - s_m s_n X(r)_{pi(m) pi(n)}| as an ordered bit pattern (NaN sorts
// above +inf), into words[p].  Item (p, representative slot).
__global__ void __launch_bounds__(256)
k_sym_defect(Batch b, const int2* __restrict__ items, const double* __restrict__ X,
             unsigned long long* __restrict__ words) {
  __shared__ unsigned long long red[256];
  const int2 it = items[blockIdx.x];
  const DevTables& d = b.pts[it.x];
  const int nff = d.nff, nff2 = nff * nff, slot = it.y, r = d.irr[slot];
  const int e0 = d.orb_start[slot], ne = d.orb_start[slot + 1] - e0;
  const size_t S = (size_t)b.S;
  unsigned long long m = 0ull;
  for (int w = threadIdx.x; w < 3 * ne * nff2; w += blockDim.x) {
    const int ch = w / (ne * nff2), rem = w % (ne * nff2), e = rem / nff2, mn = rem % nff2;
    const int q = d.orb_q[e0 + e], tr = d.orb_tr[e0 + e];
    const int pa = d.tperm[(size_t)tr * nff + mn / nff], pc = d.tperm[(size_t)tr * nff + mn % nff];
    const double sg = ((pa ^ pc) >> 8) & 1 ? -1.0 : 1.0;
    const double* Xc = X + ch * S + d.off;
    const double v = Xc[(size_t)q * nff2 + mn] - sg * Xc[(size_t)r * nff2 + (pa & 0xff) * nff + (pc & 0xff)];
    unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(v));
    if (v != v) bits = 0x7ff8000000000000ull;
    m = bits > m ? bits : m;
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && red[threadIdx.x + s] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != 0ull) atomicMax(words + it.x, red[0]);
}

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_i32(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Tp[p] = Ttab[4 * step + stage] for every point (the RK4 stage temperature)
__global__ void k_set_T(double* Tp, int npts, const double* __restrict__ Ttab,
                        const int* __restrict__ step, int stage) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < npts) Tp[i] = Ttab[4 * step[0] + stage];
}

// Tp[i] = T[i] for a host array passed by value (up to 64 points per launch)
struct TValues {
  double v[64];
};
__global__ void k_set_Tv(double* Tp, int n, TValues tv) {
  const int i = threadIdx.x;
  if (i < n) Tp[i] = tv.v[i];
}

// End of an RK4 step: record max|X| per point, stop points whose state passed
// Xmax or became non-finite (frozen = step index of the stop), clear the max
// words and advance the step counter; status_out (mapped host memory, may be
// null) receives every point's frozen word.
__global__ void k_step_end(unsigned long long* words, int npts, int* frozen, double* hist,
                           int* step, int nsteps, double xmax, int* status_out) {
  const int i = threadIdx.x;
  const int s = step[0];
  for (int p = i; p < npts; p += blockDim.x) {
    const double m = __longlong_as_double((long long)words[p]);
    int f = frozen[p];
    if (!f) {
      hist[(size_t)(s + 1) * npts + p] = m;
      if (!(m <= xmax)) {
        f = s + 1;
        frozen[p] = f;
      }
    }
    if (status_out != nullptr) status_out[p] = f;
    words[p] = 0ull;
  }
  __syncthreads();
  if (i == 0 && s < nsteps) step[0] = s + 1;
}

}  // namespace

// ============================================================== launchers
void launch_chi_expand(const Launch& L, const ItemRange& r, const double* fin, double* dchi,
                       hipStream_t s) {
  if (r.n <= 0) return;
  hipLaunchKernelGGL(k_chi_expand, dim3(r.n), dim3(256), 0, s, L.b, L.exp_items + r.begin, fin, dchi);
}

void launch_fwd(const Launch& L, const Ranges& r, const double* X, bool mixed, hipStream_t s) {
  if (r.fwd.n <= 0) return;
  const int cols = 16 * ((int)L.front_threads / 64);
  auto launch = [&](const ItemRange& ir, int kt, size_t sm) {
    if (ir.n <= 0) return;
    const int4* it = L.fwd_items + ir.begin;
    const dim3 g(ir.n), blk(L.front_threads);
    if (mixed) {
      switch (kt) {
        case 1: hipLaunchKernelGGL(k_dft_fwd_mix<1>, g, blk, sm, s, L.b, it, X); break;
        case 2: hipLaunchKernelGGL(k_dft_fwd_mix<2>, g, blk, sm, s, L.b, it, X); break;
        case 3: hipLaunchKernelGGL(k_dft_fwd_mix<3>, g, blk, sm, s, L.b, it, X); break;
        default: hipLaunchKernelGGL(k_dft_fwd_mix<5>, g, blk, sm, s, L.b, it, X); break;
      }
    } else {
      switch (kt) {
        case 1: hipLaunchKernelGGL(k_dft_fwd_part<1>, g, blk, sm, s, L.b, it, X); break;
        case 2: hipLaunchKernelGGL(k_dft_fwd_part<2>, g, blk, sm, s, L.b, it, X); break;
        case 3: hipLaunchKernelGGL(k_dft_fwd_part<3>, g, blk, sm, s, L.b, it, X); break;
        default: hipLaunchKernelGGL(k_dft_fwd_part<5>, g, blk, sm, s, L.b, it, X); break;
      }
    }
  };
  if (r.nfwd_cls == 0) {
    launch(r.fwd, L.fwd_kt, L.fwd_smem);
    return;
  }
  // one launch per harmonic tile count, each with the LDS of its own tiles:
  // FP64 chunks of 32 momenta [32][16 KT + 2] + [32][cols + 2]; split precision
  // hi and lo quads [8][16 KT] + [8][cols]
  for (int c = 0; c < r.nfwd_cls; ++c) {
    const int kt = r.fwd_cls_kt[c];
    const size_t sm = mixed ? (size_t)16 * 8 * (16 * kt + cols)
                            : sizeof(double) * 32 * ((size_t)(16 * kt + 2) + (size_t)(cols + 2));
    launch(r.fwd_cls[c], kt, sm);
  }
}

void launch_gather(const Launch& L, const Ranges& r, hipStream_t s) {
  if (r.gather.n > 0)
    hipLaunchKernelGGL(k_gather_g2, dim3(r.gather.n), dim3(64), 0, s, L.b, L.gather_items + r.gather.begin,
                       L.gather_ent, L.gather_cap);
}

void launch_gather_inv(const Launch& L, const Ranges& r, bool mixed, hipStream_t s) {
  launch_gather(L, r, s);
  launch_inv(L, r, mixed, s);
}

void launch_inv(const Launch& L, const Ranges& r, bool mixed, hipStream_t s) {
  if (r.inv.n > 0) {
    const int4* it = L.inv_items + r.inv.begin;
    const dim3 g(r.inv.n), blk(256);
    const bool one = L.one_point;
    if (mixed) {
      switch (L.inv_lt) {
        case 1: if (one) hipLaunchKernelGGL((k_dft_inv_mix<1, true>), g, blk, 0, s, L.b, it);
          else hipLaunchKernelGGL((k_dft_inv_mix<1, false>), g, blk, 0, s, L.b, it);
          break;
        case 2: if (one) hipLaunchKernelGGL((k_dft_inv_mix<2, true>), g, blk, 0, s, L.b, it);
          else hipLaunchKernelGGL((k_dft_inv_mix<2, false>), g, blk, 0, s, L.b, it);
          break;
        default: if (one) hipLaunchKernelGGL((k_dft_inv_mix<4, true>), g, blk, 0, s, L.b, it);
          else hipLaunchKernelGGL((k_dft_inv_mix<4, false>), g, blk, 0, s, L.b, it);
          break;
      }
    } else {
      switch (L.inv_lt) {
        case 1: if (one) hipLaunchKernelGGL((k_dft_inv<1, true, 3>), g, blk, 0, s, L.b, it);
          else hipLaunchKernelGGL((k_dft_inv<1, false, 3>), g, blk, 0, s, L.b, it);
          break;
        case 2: if (one) hipLaunchKernelGGL((k_dft_inv<2, true>), g, blk, 0, s, L.b, it);
          else hipLaunchKernelGGL((k_dft_inv<2, false>), g, blk, 0, s, L.b, it);
          break;
        default: if (one) hipLaunchKernelGGL((k_dft_inv<4, true>), g, blk, 0, s, L.b, it);
          else hipLaunchKernelGGL((k_dft_inv<4, false>), g, blk, 0, s, L.b, it);
          break;
      }
    }
  }
}

void launch_basis(const Launch& L, const Ranges& r, hipStream_t s) {
  if (r.basis.n > 0)
    hipLaunchKernelGGL(k_bond_basis, dim3(r.basis.n), dim3(256), 0, s, L.b, L.basis_items + r.basis.begin);
}

void launch_front(const Launch& L, const Ranges& r, const double* X, bool mixed, hipStream_t s) {
  launch_fwd(L, r, X, mixed, s);
  launch_basis(L, r, s);
  launch_gather_inv(L, r, mixed, s);
}

void launch_dense(const Launch& L, const Ranges& r, const double* X, hipStream_t s) {
  if (r.dpart.n > 0)
    hipLaunchKernelGGL(k_dense_part, dim3(r.dpart.n), dim3(256), 0, s, L.b, L.dpart_items + r.dpart.begin, X);
  if (r.dsum.n > 0)
    hipLaunchKernelGGL(k_dense_sum, dim3(r.dsum.n), dim3(256), 0, s, L.b, L.dsum_items + r.dsum.begin);
}

void launch_set_unit(double* X, int64_t prev, int64_t cur, hipStream_t s) {
  hipLaunchKernelGGL(k_set_unit, dim3(1), dim3(64), 0, s, X, prev, cur);
}

void launch_expand_basis(const Launch& L, const Ranges& r, double* dchi, bool cross, hipStream_t s) {
  const int nb = cross ? r.basis.n : 0;
  if (r.exp.n + nb <= 0) return;
  if (L.one_point)
    hipLaunchKernelGGL(k_expand_basis<true>, dim3(r.exp.n + nb), dim3(256), 0, s, L.b, L.exp_items + r.exp.begin,
                       r.exp.n, L.basis_items + r.basis.begin, dchi);
  else
    hipLaunchKernelGGL(k_expand_basis<false>, dim3(r.exp.n + nb), dim3(256), 0, s, L.b, L.exp_items + r.exp.begin,
                       r.exp.n, L.basis_items + r.basis.begin, dchi);
}

void launch_back(const Launch& L, const Ranges& r, const double* X, double* out, int mode,
                 bool cross, bool scale_T, bool mixed, hipStream_t s, const StageNext* sn) {
  if (r.prod.n <= 0) return;
  StageNext sv{};
  if (sn != nullptr && mode == 1) sv = *sn;
  auto launch = [&](const ItemRange& ir, size_t smem64) {
    if (ir.n <= 0) return;
    const int4* it = L.prod_items + ir.begin;
    const int c = cross ? 1 : 0, st = scale_T ? 1 : 0;
    const float* k32 = (const float*)L.b.kinv;
    const double* k64 = (const double*)L.b.kinv64;
    auto go = [&](auto stage_form) {
      constexpr bool SF = decltype(stage_form)::value;
      if (mixed && L.one_point)
        hipLaunchKernelGGL((k_products<float, true, SF>), dim3(ir.n), dim3(256), smem64 / 2, s, L.b, it, X, k32,
                           out, mode, c, st, sv);
      else if (mixed)
        hipLaunchKernelGGL((k_products<float, false, SF>), dim3(ir.n), dim3(256), smem64 / 2, s, L.b, it, X, k32,
                           out, mode, c, st, sv);
      else if (L.one_point)
        hipLaunchKernelGGL((k_products<double, true, SF>), dim3(ir.n), dim3(256), smem64, s, L.b, it, X, k64,
                           out, mode, c, st, sv);
      else
        hipLaunchKernelGGL((k_products<double, false, SF>), dim3(ir.n), dim3(256), smem64, s, L.b, it, X, k64,
                           out, mode, c, st, sv);
    };
    if (sv.nk > 0) go(std::true_type{});
    else go(std::false_type{});
  };
  if (r.nprod_cls == 0) {
    launch(r.prod, L.prod_smem);
    return;
  }
  // one launch per N_ff, each with the [10][N_ff^2] shared memory of its own matrices
  for (int c = 0; c < r.nprod_cls; ++c)
    launch(r.prod_cls[c], sizeof(double) * 10 * (size_t)r.prod_cls_nff[c] * r.prod_cls_nff[c]);
}

void launch_axpy(const Launch& L, const ItemRange& r, const double* X, const double* const* k,
                 const double* coef, int nk, double h, double* out, bool skip_frozen, hipStream_t s,
                 const double* hp) {
  if (r.n <= 0) return;
  SlopeSet ks{};
  for (int j = 0; j < nk; ++j) {
    ks.k[j] = k[j];
    ks.coef[j] = coef[j];
  }
  const dim3 g(r.n), blk(256);
  const int4* it = L.seg_items + r.begin;
  const int sf = skip_frozen ? 1 : 0;
  switch (nk) {
    case 1: hipLaunchKernelGGL(k_axpy<1>, g, blk, 0, s, L.b, it, X, ks, h, out, sf, hp); break;
    case 2: hipLaunchKernelGGL(k_axpy<2>, g, blk, 0, s, L.b, it, X, ks, h, out, sf, hp); break;
    case 3: hipLaunchKernelGGL(k_axpy<3>, g, blk, 0, s, L.b, it, X, ks, h, out, sf, hp); break;
    case 4: hipLaunchKernelGGL(k_axpy<4>, g, blk, 0, s, L.b, it, X, ks, h, out, sf, hp); break;
    case 5: hipLaunchKernelGGL(k_axpy<5>, g, blk, 0, s, L.b, it, X, ks, h, out, sf, hp); break;
    case 6: hipLaunchKernelGGL(k_axpy<6>, g, blk, 0, s, L.b, it, X, ks, h, out, sf, hp); break;
    default: hipLaunchKernelGGL(k_axpy<7>, g, blk, 0, s, L.b, it, X, ks, h, out, sf, hp); break;
  }
}

void launch_maxabs(const Launch& L, const ItemRange& r, const double* X, unsigned long long* words,
                   hipStream_t s) {
  if (r.n <= 0) return;
  hipLaunchKernelGGL(k_maxabs, dim3(r.n), dim3(256), 0, s, L.b, L.seg_items + r.begin, X, words);
}

void launch_dp_final(const Launch& L, const ItemRange& r, const double* y0, const double* const* k,
                     const double* b5, const double* e, double h, double rtol, double atol, double* y5,
                     double* red, unsigned long long* max_words, hipStream_t s, const double* hp) {
  if (r.n <= 0) return;
  SlopeSet ks{};
  Coef7 ec{};
  for (int j = 0; j < 7; ++j) {
    ks.k[j] = k[j];
    ks.coef[j] = b5[j];
    ec.c[j] = e[j];
  }
  hipLaunchKernelGGL(k_dp_final, dim3(r.n), dim3(256), 0, s, L.b, L.seg_items + r.begin, y0, ks, ec, h,
                     rtol, atol, y5, red, max_words, hp);
}

void launch_first_max(const Launch& L, const ItemRange& r, const double* X, const unsigned long long* words,
                      int* first, hipStream_t s) {
  if (r.n <= 0) return;
  hipLaunchKernelGGL(k_first_max, dim3(r.n), dim3(256), 0, s, L.b, L.seg_items + r.begin, X, words, first);
}

void launch_dp_control(const DpControl& c, hipStream_t s) {
  hipLaunchKernelGGL(k_dp_control, dim3(c.npts), dim3(256), 0, s, c);
}

void launch_dp_accept(const Launch& L, const ItemRange& r, const DpState* st, const double* y5, const double* k6,
                      double* y, double* k0, double a10, const double* h_arr, double* stage1, hipStream_t s) {
  if (r.n <= 0) return;
  hipLaunchKernelGGL(k_dp_accept, dim3(r.n), dim3(256), 0, s, L.b, L.seg_items + r.begin, st, y5, k6, y, k0, a10,
                     h_arr, stage1);
}

void launch_set_T_sh(double* Tp, int npts, const double* s_arr, const double* h_arr, double c, hipStream_t s) {
  hipLaunchKernelGGL(k_set_T_sh, dim3((npts + 255) / 256), dim3(256), 0, s, Tp, npts, s_arr, h_arr, c);
}

void launch_sym_defect(const Launch& L, const int2* items, int n, const double* X, unsigned long long* words,
                       hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_sym_defect, dim3(n), dim3(256), 0, s, L.b, items, X, words);
}

void launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
}

void launch_fill_i32(int* p, int n, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
}

void launch_set_T(double* Tp, int npts, const double* Ttab, const int* step, int stage,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_set_T, dim3((npts + 255) / 256), dim3(256), 0, s, Tp, npts, Ttab, step, stage);
}

void launch_set_T_values(double* Tp, const double* T_host, int n, hipStream_t s) {
  for (int p0 = 0; p0 < n; p0 += 64) {
    TValues tv{};
    const int m = std::min(64, n - p0);
    for (int i = 0; i < m; ++i) tv.v[i] = T_host[p0 + i];
    hipLaunchKernelGGL(k_set_Tv, dim3(1), dim3(64), 0, s, Tp + p0, m, tv);
  }
}

void launch_step_end(unsigned long long* words, int npts, int* frozen, double* hist, int* step,
                     int nsteps, double xmax, hipStream_t s, int* status_out) {
  hipLaunchKernelGGL(k_step_end, dim3(1), dim3(256), 0, s, words, npts, frozen, hist, step, nsteps,
                     xmax, status_out);
}

}  // namespace tufrg
