// Device bodies of the forward transform of the projections (Sec. 2.4,
// eqns. proj_VP/VC/VD: the Fourier sums of the channel couplings over the
// transfer grid), shared by the stand-alone forward-transform kernels and by
// the combined loop + forward-transform launch of the right-hand side.
//
// The transforms are the partial sums over one split of the transfer grid at
// the half-integer frequencies S/2,
//   xp[s][k][ch mn] = sum_{u in split s} E[u][k] X[ch][u][mn],
//   E = (cos(u.S'/2) | sin(u.S'/2)),
// with the splits added in order (and divided by Nq) by the bond-basis
// kernel.  A block of nw = blockDim.x / 64 waves owns 16 nw consecutive
// columns (ch, mn); wave w owns 16 of them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "tufrg_internal.h"

namespace tufrg {
namespace {

__device__ __forceinline__ bool skip_point(const Batch& b, int p) {
  return b.frozen != nullptr && b.frozen[p] != 0;
}

// The tables of point p; ONE (a single-point launch, p = 0): the copy in the
// launch's arguments, which needs no load of the device array first
template <bool ONE>
__device__ __forceinline__ const DevTables& point_tables(const Batch& b, int p) {
  if constexpr (ONE) return b.pt0;
  else return b.pts[p];
}

typedef double f64x4 __attribute__((ext_vector_type(4)));
// BF16 hi/lo split with round to nearest even: x ~ hi + lo (about 16 mantissa
// bits); products hi*hi + hi*lo + lo*hi accumulate in FP32 on the matrix cores.
// v_mfma_f32_16x16x16bf16_1k operand layout: lane l holds A[l%16][4(l/16)+j],
// B[4(l/16)+j][l%16] (j = 0..3) and D[4(l/16)+j][l%16].
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// v_mfma_f32_16x16x32_bf16 (CDNA4: twice the K of the _1k form per
// instruction, at the same issue cost): lane l holds A[l%16][8(l/16)+j],
// B[8(l/16)+j][l%16] (j = 0..7), D as above; an operand is two quads of
// consecutive k, kept together in LDS.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short short8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ bf16x8 quad_pair(bf16x4 a, bf16x4 b) {
  const short8 s = __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_bit_cast(bf16x8, s);
}

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}
__device__ __forceinline__ void split_bf16(double x, unsigned short& hi, unsigned short& lo) {
  const float f = (float)x;
  hi = bf16_rne(f);
  lo = bf16_rne(f - bf16_to_f32(hi));
}

// FP64 on the matrix cores.  Item (p, column tile c, transfer split s): the
// block's columns against KT tiles of 16 harmonic rows k (E from its copy
// padded with zero columns to kEpad).  Chunks of 32 momenta u pass through
// LDS (32 (16 KT + 2) + 32 (16 nw + 2) doubles); wave w accumulates KT tiles of
// v_mfma_f64_16x16x4f64 (lane l holds A[l%16][l/16], B[l/16][l%16] and, in
// register j, D[4j+l/16][l%16]).
template <int KT>
__device__ __forceinline__ void fwd_part_body(const Batch& b, const DevTables& d, const int4 item,
                                              const double* __restrict__ X, double* smem) {
  constexpr int TK = 16 * KT, ES = TK + 2;
  const int nw = (int)blockDim.x >> 6, CW = 16 * nw, XS = CW + 2;
  double* Es = smem;             // [32][ES]
  double* Xs = smem + 32 * ES;   // [32][XS]
  const int nq = d.nq, ncol = d.ncol, nff2 = d.nff * d.nff, N = 3 * nff2;
  const int c0 = item.y * CW, split = item.z;
  const int u0 = (int)((int64_t)nq * split / d.nsu), u1 = (int)((int64_t)nq * (split + 1) / d.nsu);
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, k4 = lane >> 4;
  // staging: each chunk's loads are issued together into registers before
  // they go to LDS.  A thread stages one column of X (the block has 4 CW
  // threads: rows tid / CW + 4 i, i < 8) and up to EPT entries of E.
  constexpr int EPT = (32 * TK + 255) / 256;
  const int xc = tid % CW, xr = tid / CW, xcol = c0 + xc;
  const bool xok = xcol < N;
  const double* xsrc = X + d.off + (xok ? (size_t)(xcol / nff2) * b.S + xcol % nff2 : 0);
  f64x4 acc[KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  // software pipeline: chunk c + 1's loads are in flight during chunk c's MFMAs
  double ev[EPT], xv[8];
  auto load = [&](int ub) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nt, uu = e / TK, k = e % TK, u = ub + uu;
      ev[i] = (e < 32 * TK && u < u1) ? d.ephp[(size_t)u * kEpad + k] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int u = ub + xr + 4 * i;
      xv[i] = (xok && u < u1) ? xsrc[(size_t)u * nff2] : 0.0;
    }
  };
  if (u0 < u1) load(u0);
  for (int ub = u0; ub < u1; ub += 32) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nt;
      if (e < 32 * TK) Es[(e / TK) * ES + e % TK] = ev[i];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) Xs[(xr + 4 * i) * XS + xc] = xv[i];
    __syncthreads();
    if (ub + 32 < u1) load(ub + 32);
#pragma unroll
    for (int uk = 0; uk < 32; uk += 4) {
      const double bv = Xs[(uk + k4) * XS + 16 * w + r16];
#pragma unroll
      for (int t = 0; t < KT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(Es[(uk + k4) * ES + 16 * t + r16], bv, acc[t], 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = b.xp + d.ws_xp + (size_t)split * ncol * N;
  const int col = c0 + 16 * w + r16;
  if (col >= N) return;
#pragma unroll
  for (int t = 0; t < KT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = 16 * t + 4 * j + k4;
      if (k < ncol) out[(size_t)k * N + col] = acc[t][j];
    }
}

// Split precision: the same contraction and output, with products
// hi*hi + hi*lo + lo*hi of the BF16 splits accumulated in FP32 over one
// split; splits start on multiples of 16 momenta.  Chunks of 32 momenta (8
// quads of 4) pass through LDS: the pre-split phase table (laid out
// [u/4][kEpad][4], zero beyond Nq) as hi and lo quads for the KT harmonic
// tiles, and the block's columns of X, split to hi and lo quads as they are
// staged (each thread stages two (quad, column) pairs: 8 loads in flight).
// Each wave then takes the chunk in one v_mfma_f32_16x16x32_bf16 step per
// product and tile; the next chunk's loads are in flight meanwhile.  LDS
// holds the quads in pairs of consecutive quads (one 16-byte operand read).
template <int KT>
__device__ __forceinline__ void fwd_mix_body(const Batch& b, const DevTables& d, const int4 item,
                                             const double* __restrict__ X, double* smem) {
  constexpr int TK = 16 * KT;
  const int nw = (int)blockDim.x >> 6, CW = 16 * nw, nt = blockDim.x;
  bf16x8* Eh = reinterpret_cast<bf16x8*>(smem);   // [4][TK] quad pairs
  bf16x8* El = Eh + 4 * TK;
  bf16x8* Xh = El + 4 * TK;                        // [4][CW]
  bf16x8* Xl = Xh + 4 * CW;
  // quad q of column (or harmonic) c in a [4][C] pair array
  auto quad = [](bf16x8* a, int C, int q, int c) -> bf16x4& {
    return reinterpret_cast<bf16x4*>(a)[((q >> 1) * C + c) * 2 + (q & 1)];
  };
  const int nq = d.nq, ncol = d.ncol, nff2 = d.nff * d.nff, N = 3 * nff2;
  const int split = item.z, nq16 = (nq + 15) >> 4;
  const int u0 = 16 * (int)((int64_t)nq16 * split / d.nsu);
  const int u1 = 16 * (int)((int64_t)nq16 * (split + 1) / d.nsu);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, k4 = lane >> 4;
  const int c0 = item.y * CW;
  // staging roles: X column xc (constant), quads xq and xq + 4; E entries
  // tid + i nt of the [8][TK] quad tile (hi and lo)
  constexpr int EPT = (8 * TK + 255) / 256;
  const int xc = tid % CW, xq = tid / CW, xcol = c0 + xc;
  const bool xok = xcol < N;
  const double* xsrc = X + d.off + (xok ? (size_t)(xcol / nff2) * b.S + xcol % nff2 : 0);
  const bf16x4* ehq = reinterpret_cast<const bf16x4*>(d.ephq_hi);
  const bf16x4* elq = reinterpret_cast<const bf16x4*>(d.ephq_lo);
  f32x4 acc[KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x4 eh[EPT], el[EPT];
  double xv[2][4];
  auto load = [&](int ub) {
    const int nst = min(32, u1 - ub) >> 4;   // steps of 16 in this chunk (1 or 2)
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nt, q = e / TK, k = e % TK;
      const size_t src = (size_t)((ub >> 2) + q) * kEpad + k;
      const bool ok = e < 8 * TK && q < 4 * nst;
      eh[i] = ok ? ehq[src] : bf16x4{0, 0, 0, 0};
      el[i] = ok ? elq[src] : bf16x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int u = ub + 4 * (xq + 4 * h) + j;
        xv[h][j] = (xok && u < nq && u < u1) ? xsrc[(size_t)u * nff2] : 0.0;
      }
  };
  if (u0 < u1) load(u0);
  for (int ub = u0; ub < u1; ub += 32) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nt;
      if (e < 8 * TK) {
        quad(Eh, TK, e / TK, e % TK) = eh[i];
        quad(El, TK, e / TK, e % TK) = el[i];
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      bf16x4 qh, ql;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        unsigned short hi, lo;
        split_bf16(xv[h][j], hi, lo);
        qh[j] = (short)hi;
        ql[j] = (short)lo;
      }
      quad(Xh, CW, xq + 4 * h, xc) = qh;
      quad(Xl, CW, xq + 4 * h, xc) = ql;
    }
    __syncthreads();
    if (ub + 32 < u1) load(ub + 32);
    // lane (r16, k4): momenta 8 k4 .. 8 k4 + 7 of the chunk (quad pair k4)
    const bf16x8 bh = Xh[k4 * CW + 16 * w + r16], bl = Xl[k4 * CW + 16 * w + r16];
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      const bf16x8 ah = Eh[k4 * TK + 16 * t + r16], al = El[k4 * TK + 16 * t + r16];
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[t], 0, 0, 0);
    }
    __syncthreads();
  }
  const int col = c0 + 16 * w + r16;
  if (col >= N) return;
  double* out = b.xp + d.ws_xp + (size_t)split * ncol * N;
#pragma unroll
  for (int t = 0; t < KT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = 16 * t + 4 * k4 + j;
      if (k < ncol) out[(size_t)k * N + col] = (double)acc[t][j];
    }
}

}  // namespace
}  // namespace tufrg
