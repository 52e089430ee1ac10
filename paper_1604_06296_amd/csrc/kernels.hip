// HIP kernels for gfx950 (CDNA4): loops, projections, products and ODE helpers
// of the TUfRG flow right-hand side.
//
// Every kernel is driven by a table of work items (point, a, b, c): one launch
// covers any set of points with uneven grids and truncations, a single point
// being a batch of one.  The point's tables are read from a device array of
// DevTables; temperatures are read from a per-point device array (so that a
// captured HIP graph can be replayed with new temperatures), and points whose
// flow has stopped are skipped through a per-point device flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "loop_math.h"
#include "tufrg_internal.h"

namespace tufrg {
namespace {

__device__ __forceinline__ bool skip_point(const Batch& b, int p) {
  return b.frozen != nullptr && b.frozen[p] != 0;
}

struct DevRcp {
  __device__ double operator()(double x) const {
    double r = __builtin_amdgcn_rcp(x);       // hardware estimate, refined by Newton steps
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
  }
};
struct Exp2F { __device__ float operator()(float x) const { return __builtin_amdgcn_exp2f(x); } };
struct RcpF { __device__ float operator()(float x) const { return __builtin_amdgcn_rcpf(x); } };

__device__ __forceinline__ void neumaier_add(float& s, float& c, float v) {
  const float t = s + v;
  const bool sbig = fabsf(s) >= fabsf(v);
  const float big = sbig ? s : v, small = sbig ? v : s;
  c += (big - t) + small;
  s = t;
}

// ------------------------------------------------------------------ loops
// Step ii.) of Sec. 2.4, eqn. chis, at the point's temperature.  Work item
// (p, slot * nsplit + split): one representative transfer momentum q =
// irr[slot] (point-group orbits; every other momentum follows by symmetry in
// the expansion kernel) and one slice of the rows
// py in [0, Lk/2] of the fine grid (the loop weight is even in p: the
// self-paired rows py = 0 and Lk/2 carry weight 1, the others weight 2).
// Threads own one column px and a chunk of the slice's rows; they accumulate
// row sums of the loop derivative against cos(n py) and sin(n py), n <= smax.
// The block contracts the rows against cos(px Sx), sin(px Sx) into
// ghat(q, S) = (1/Nk) sum_p L'(p) cos(p.S) for the half set of harmonics S in
// bonds + bonds.
// In the persistent form queue[0] is the next item and queue[1] counts
// finished blocks; both are zero at entry, and the last block to finish sets
// them back to zero for the next launch (device-scope atomics, valid across
// XCDs).  MIXED selects the FP32 pair math with blocked Neumaier-compensated
// FP32 row sums; otherwise everything is FP64.
//
// One loop work item with the point's exact harmonic count NH = 2 smax + 1
// (compile-time, so the per-row harmonic loops carry no guards).
template <int SMAX, bool MIXED>
__device__ __forceinline__ void loop_item(const Batch& b, const DevTables& d, int p, int item_b,
                                          double* smem) {
  constexpr int NH = 2 * SMAX + 1;
  const int t = threadIdx.x;
  const int nsplit = d.nsplit, nchunk = d.nchunk;
  const int slot = item_b / nsplit, split = item_b % nsplit;
  const int q = d.irr[slot];
  const int lk = d.lk;
  const int rows = lk / 2 + 1;
  const int R0 = (int)((int64_t)rows * split / nsplit);
  const int R1 = (int)((int64_t)rows * (split + 1) / nsplit);
  const int nr = R1 - R0;
  const int lq = d.lq;
  const int ix = q / lq, iy = q % lq;
  const double T = b.Tp[p];
  const double inv2T = 0.5 / T;

  double* y1 = smem;                        // cos(py + qy/2)        [nr]
  double* y2 = y1 + nr;                     // cos(py - qy/2)        [nr]
  double* pyt = y2 + nr;                    // weighted py harmonics [nr][NH]
  double* rs = pyt + nr * NH;               // row sums              [lk][2][NH]
  double* gh = rs + lk * 2 * NH;            // harmonic partials     [nseg][2 nsh]
  for (int j = t; j < nr; j += blockDim.x) {
    const double* c = d.cshift + ((size_t)iy * lk + (R0 + j)) * 2;
    y1[j] = c[0];
    y2[j] = c[1];
  }
  for (int j = t; j < nr * NH; j += blockDim.x) pyt[j] = d.pytab[R0 * NH + j];
  for (int j = t; j < lk * 2 * NH; j += blockDim.x) rs[j] = 0.0;
  __syncthreads();

  const bool active = t < lk * nchunk;
  const int px = t % lk, c = t / lk;
  double acc[2][NH];
#pragma unroll
  for (int n = 0; n < NH; ++n) acc[0][n] = acc[1][n] = 0.0;
  if (active) {
    const double cx1 = d.cshift[((size_t)ix * lk + px) * 2];       // cos(px + qx/2)
    const double cx2 = d.cshift[((size_t)ix * lk + px) * 2 + 1];   // cos(px - qx/2)
    // alpha = eps(p + q/2)/(2T) = A1 + B1 cos(py + qy/2); beta likewise
    const double A1 = (-2.0 * d.t * cx1 - d.mu) * inv2T;
    const double B1 = (-2.0 * d.t - 4.0 * d.tp * cx1) * inv2T;
    const double A2 = (-2.0 * d.t * cx2 - d.mu) * inv2T;
    const double B2 = (-2.0 * d.t - 4.0 * d.tp * cx2) * inv2T;
    const int r0 = (int)((int64_t)nr * c / nchunk);
    const int r1 = (int)((int64_t)nr * (c + 1) / nchunk);
    if constexpr (!MIXED) {
#pragma unroll 2
      for (int r = r0; r < r1; ++r) {
        const double al = fma(B1, y1[r], A1);
        const double be = fma(B2, y2[r], A2);
        double dph, dpp;
        loop_dot_pair_t(al, be, dph, dpp, DevRcp());
        const double* w = pyt + r * NH;
#pragma unroll
        for (int n = 0; n < NH; ++n) {
          acc[0][n] = fma(dpp, w[n], acc[0][n]);
          acc[1][n] = fma(dph, w[n], acc[1][n]);
        }
      }
    } else {
      // FP32 pair math from FP64 energies; rows blocked by 8 in FP32 and
      // added into Neumaier-compensated FP32 running sums
      constexpr int RB = 8;
      float sum[2][NH], cmp[2][NH];
#pragma unroll
      for (int n = 0; n < NH; ++n) sum[0][n] = sum[1][n] = cmp[0][n] = cmp[1][n] = 0.0f;
      for (int rb = r0; rb < r1; rb += RB) {
        float blk[2][NH];
#pragma unroll
        for (int n = 0; n < NH; ++n) blk[0][n] = blk[1][n] = 0.0f;
        const int re = min(rb + RB, r1);
        for (int r = rb; r < re; ++r) {
          const double al = fma(B1, y1[r], A1);
          const double be = fma(B2, y2[r], A2);
          float dph, dpp;
          loop_dot_pair_f32((float)al, (float)be, (float)(al - be), (float)(al + be), dph, dpp,
                            Exp2F(), RcpF());
          const double* w = pyt + r * NH;
#pragma unroll
          for (int n = 0; n < NH; ++n) {
            const float wf = (float)w[n];
            blk[0][n] = fmaf(dpp, wf, blk[0][n]);
            blk[1][n] = fmaf(dph, wf, blk[1][n]);
          }
        }
#pragma unroll
        for (int n = 0; n < NH; ++n) {
          neumaier_add(sum[0][n], cmp[0][n], blk[0][n]);
          neumaier_add(sum[1][n], cmp[1][n], blk[1][n]);
        }
      }
#pragma unroll
      for (int n = 0; n < NH; ++n) {
        acc[0][n] = (double)sum[0][n] + (double)cmp[0][n];
        acc[1][n] = (double)sum[1][n] + (double)cmp[1][n];
      }
    }
  }
  // add the chunks into the row sums one after another (fixed order)
  for (int cc = 0; cc < nchunk; ++cc) {
    if (active && c == cc) {
      double* dst = rs + px * 2 * NH;
#pragma unroll
      for (int n = 0; n < NH; ++n) {
        dst[n] += acc[0][n];
        dst[NH + n] += acc[1][n];
      }
    }
    __syncthreads();
  }
  // contraction over px into the half-set harmonics, split into segments
  const int nout = 2 * d.nsh;
  int nseg = (int)blockDim.x / nout;
  if (nseg < 1) nseg = 1;
  for (int w = t; w < nout * nseg; w += blockDim.x) {
    const int o = w % nout, seg = w / nout;
    const int ch = o / d.nsh, j = o % d.nsh;
    const int sx = d.hx[j], sy = d.hy[j];          // sx >= 0
    const int ay = sy < 0 ? -sy : sy;
    const double sg = sy < 0 ? -1.0 : 1.0;
    double g = 0.0;
    for (int x = seg; x < lk; x += nseg) {
      const double* r = rs + x * 2 * NH + ch * NH;
      // cos(px sx + py sy) = cos(px sx) cos(py |sy|) - sin(px sx) sgn(sy) sin(py |sy|)
      double v = d.pxtab[x * NH + sx] * r[ay];
      if (sx > 0 && ay > 0) v = fma(-sg * d.pxtab[x * NH + SMAX + sx], r[SMAX + ay], v);
      g += v;
    }
    gh[seg * nout + o] = g;
  }
  __syncthreads();
  for (int o = t; o < nout; o += blockDim.x) {
    double g = 0.0;
    for (int s = 0; s < nseg; ++s) g += gh[s * nout + o];
    gh[o] = g;
  }
  __syncthreads();
  // ghat_X(q, S_j) = sgn_X gh_j / (4 T^2 Nk) (pp carries the minus sign of
  // dL^pp/dT = -Dh/(4T^2)), written to slice `split` of the representative's
  // harmonics; chi'_mn = sum_j Ebub_{mn,j} ghat(q, S_j) follows in the
  // expansion kernel.
  const double base = 1.0 / (4.0 * T * T * (double)lk * (double)lk);
  for (int o = t; o < nout; o += blockDim.x)
    b.ghat[d.ws_gh + ((size_t)split * d.nirr + slot) * nout + o] = gh[o] * (o < d.nsh ? -base : base);
  __syncthreads();
}

template <int SMAX, bool MIXED>
__device__ __forceinline__ void loop_dispatch(const Batch& b, const int4 item, double* smem) {
  const int p = item.x;
  if (skip_point(b, p)) return;
  const DevTables& d = b.pts[p];
  if constexpr (SMAX >= 4) {
    if (d.smax == 4) {
      loop_item<4, MIXED>(b, d, p, item.y, smem);
      return;
    }
  }
  if constexpr (SMAX >= 2) {
    if (d.smax == 2) {
      loop_item<2, MIXED>(b, d, p, item.y, smem);
      return;
    }
  }
  loop_item<0, MIXED>(b, d, p, item.y, smem);
}

// Loop kernel over work items (p, q * nsplit + split); SMAX is the largest
// smax of the batch, and each item runs the body compiled for its own smax.
// Without a queue every block runs item blockIdx.x (the hardware dispatcher
// balances the load, items being ordered costliest first); with a queue the
// kernel is persistent and blocks take items until the queue is empty.
template <int SMAX, bool MIXED>
__global__ void __launch_bounds__(kLoopThreadsMax)
k_loops(Batch b, const int4* __restrict__ items, int nitems, int* __restrict__ queue) {
  extern __shared__ double smem[];
  __shared__ int cur;
  if (b.item_count != nullptr) nitems = min(nitems, *b.item_count);
  if (queue == nullptr) {
    if ((int)blockIdx.x < nitems) loop_dispatch<SMAX, MIXED>(b, items[blockIdx.x], smem);
    return;
  }
  const int t = threadIdx.x;
  for (;;) {
    if (t == 0) cur = atomicAdd(queue, 1);
    __syncthreads();
    const int it = cur;
    __syncthreads();
    if (it >= nitems) break;
    loop_dispatch<SMAX, MIXED>(b, items[it], smem);
  }
  if (t == 0 && atomicAdd(queue + 1, 1) == (int)gridDim.x - 1) {
    atomicExch(queue, 0);
    atomicExch(queue + 1, 0);
  }
}

// chi'_mn(q) = sum_j Ebub_{mn,j} ghat(q, S_j) for every momentum, with
// ghat(q, S_j) = sign ghat(r, S_j') of its representative (pack_sym entry of
// the symmetry map), as one contraction over j: rows (channel, q), columns
// mn.  Item (p, row tile of 32, column tile of 64); the representatives'
// harmonics are the sums of their loop slices, or come from fin
// [nirr][2][nsh] (single point).  Each thread owns 2 rows x 4 columns.
constexpr int kExpRows = 32, kExpCols = 64, kExpK = 36;
__global__ void __launch_bounds__(256)
k_chi_expand(Batch b, const int4* __restrict__ items, const double* __restrict__ fin,
             double* __restrict__ dchi) {
  __shared__ double As[kExpRows][kExpK];
  __shared__ double Bs[kExpK][kExpCols];
  const int4 item = items[blockIdx.x];
  const int p = item.x;
  if (skip_point(b, p)) return;
  const DevTables& d = b.pts[p];
  const int nq = d.nq, nsh = d.nsh, nout = 2 * nsh, nff2 = d.nff * d.nff;
  const int r0 = item.y * kExpRows, c0 = item.z * kExpCols;
  const int tid = threadIdx.x;
  for (int e = tid; e < kExpRows * nsh; e += 256) {
    const int rr = e / nsh, j = e % nsh, row = r0 + rr;
    double v = 0.0;
    if (row < 2 * nq) {
      const int ch = row / nq, q = row % nq;
      const int32_t pk = d.symmap[(size_t)q * nsh + j];
      const int slot = pk & 0xffff, oo = ch * nsh + ((pk >> 16) & 0x7f);
      if (fin) {
        v = fin[(size_t)slot * nout + oo];
      } else {
        for (int sl = 0; sl < d.nsplit; ++sl) v += b.ghat[d.ws_gh + ((size_t)sl * d.nirr + slot) * nout + oo];
      }
      if ((pk >> 24) & 1) v = -v;
    }
    As[rr][j] = v;
  }
  for (int e = tid; e < nsh * kExpCols; e += 256) {
    const int j = e / kExpCols, c = e % kExpCols, mn = c0 + c;
    Bs[j][c] = mn < nff2 ? d.ebub[(size_t)mn * nsh + j] : 0.0;
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
    if (row >= 2 * nq) continue;
    const int ch = row / nq, q = row % nq;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int mn = c0 + cc + c;
      if (mn < nff2) dchi[(size_t)ch * b.S + d.off + (size_t)q * nff2 + mn] = acc[i][c];
    }
  }
}

// ------------------------------------------------------- projections
// Forward transform: the partial Fourier sums over the transfer grid at the
// half-integer frequencies S/2,
//   xt[ch][k][mn] = (1/Nq) sum_u E[u][k] X[ch][u][mn],  E = (cos(u.S'/2) | sin(u.S'/2)),
// as a contraction on the FP64 matrix cores, split over the transfer grid.
// Item (p, column tile c, transfer split s): 64 consecutive columns (ch, mn)
// against KT tiles of 16 harmonic rows k (E from its copy padded with zero
// columns to kEpad).  Chunks of 32 momenta u pass through LDS; wave w owns
// 16 columns and KT accumulator tiles of v_mfma_f64_16x16x4f64 (lane l holds
// A[l%16][l/16], B[l/16][l%16] and, in register j, D[4j+l/16][l%16]).  Partial sums go to
// xp[s][k][col]; the bond-basis kernel adds the splits in order.
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <int KT>
__global__ void __launch_bounds__(256)
k_dft_fwd_part(Batch b, const int4* __restrict__ items, const double* __restrict__ X) {
  constexpr int TK = 16 * KT;
  __shared__ double Es[32][TK + 2];
  __shared__ double Xs[32][64 + 2];
  const int4 item = items[blockIdx.x];
  const int p = item.x;
  if (skip_point(b, p)) return;
  const DevTables& d = b.pts[p];
  const int nq = d.nq, ncol = d.ncol, nff2 = d.nff * d.nff, N = 3 * nff2;
  const int c0 = item.y * 64, split = item.z;
  const int u0 = (int)((int64_t)nq * split / d.nsu), u1 = (int)((int64_t)nq * (split + 1) / d.nsu);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, k4 = lane >> 4;
  const double* Xp = X + d.off;
  f64x4 acc[KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int ub = u0; ub < u1; ub += 32) {
    for (int e = tid; e < 32 * TK; e += 256) {
      const int uu = e / TK, k = e % TK, u = ub + uu;
      Es[uu][k] = u < u1 ? d.ephp[(size_t)u * kEpad + k] : 0.0;
    }
    for (int e = tid; e < 32 * 64; e += 256) {
      const int uu = e >> 6, c = e & 63, u = ub + uu, col = c0 + c;
      double v = 0.0;
      if (u < u1 && col < N) {
        const int ch = col / nff2, mn = col % nff2;
        v = Xp[(size_t)ch * b.S + (size_t)u * nff2 + mn];
      }
      Xs[uu][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int uk = 0; uk < 32; uk += 4) {
      const double bv = Xs[uk + k4][16 * w + r16];
#pragma unroll
      for (int t = 0; t < KT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(Es[uk + k4][16 * t + r16], bv, acc[t], 0, 0, 0);
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

// Bond basis of the transformed propagators, for every harmonic of the full
// list v (+S'_j for v < nsh, -S'_{v-nsh+1} otherwise):
//   yb[in][v][b1 b2] = sum_{m' in shell(b1), n' in shell(b2)} c_{m'b1} c_{n'b2} xt^{in}_{m'n'}(v)
// with xt(-S') = conj(xt(S')).  These are the bond-space Fourier coefficients
// Yhat_{R1R2}(W) of the propagators at frequency 2W - R1 - R2 = v.
// Item (p, in * nv + v): the harmonic's transform and the coefficients are
// staged in LDS; threads own bond pairs (b1, b2).  The transform is the
// in-order FP64 sum of the forward-transform splits (xp), taken here.
__global__ void __launch_bounds__(256)
k_bond_basis(Batch b, const int4* __restrict__ items) {
  const int4 item = items[blockIdx.x];
  const int p = item.x;
  if (skip_point(b, p)) return;
  const DevTables& d = b.pts[p];
  const int nff = d.nff, nff2 = nff * nff, nsh = d.nsh, ncol = d.ncol, nv = 2 * nsh - 1;
  const int total = 3 * nv * nff2;
  const int in = item.y / nv, v = item.y % nv;
  const int j = v < nsh ? v : v - nsh + 1;
  const double sim = v < nsh ? 1.0 : -1.0;
  __shared__ double cs[2 * 441];
  __shared__ double xs[2 * 441];
  {
    const int N = 3 * nff2;
    const size_t sstride = (size_t)ncol * N;
    const double* pr = b.xp + d.ws_xp + (size_t)j * N + (size_t)in * nff2;
    const double* pi = b.xp + d.ws_xp + (size_t)(nsh - 1 + j) * N + (size_t)in * nff2;
    const double inv = 1.0 / (double)d.nq;
    for (int i = threadIdx.x; i < nff2; i += blockDim.x) {
      double vr = 0.0, vi = 0.0;
#pragma unroll 4
      for (int sp = 0; sp < d.nsu; ++sp) {
        vr += pr[sp * sstride + i];
        if (j > 0) vi += pi[sp * sstride + i];
      }
      xs[i] = vr * inv;
      xs[nff2 + i] = sim * vi * inv;
    }
  }
  for (int i = threadIdx.x; i < nff2; i += blockDim.x) {
    cs[i] = d.cre[i];
    cs[nff2 + i] = d.cim[i];
  }
  __syncthreads();
  double* yb = b.yb + d.ws_yb;
  for (int bb = threadIdx.x; bb < nff2; bb += blockDim.x) {
    const int b1 = bb / nff, b2 = bb % nff;
    const int s1 = d.shell_of[b1], s2 = d.shell_of[b2];
    const int m0 = d.shell_start[s1], m1 = d.shell_start[s1 + 1];
    const int n0 = d.shell_start[s2], n1 = d.shell_start[s2 + 1];
    double yr = 0.0, yi = 0.0;
    for (int mp = m0; mp < m1; ++mp) {
      const double c1r = cs[mp * nff + b1], c1i = cs[nff2 + mp * nff + b1];
#pragma unroll 4
      for (int np = n0; np < n1; ++np) {
        const double c2r = cs[np * nff + b2], c2i = cs[nff2 + np * nff + b2];
        const double wr = c1r * c2r - c1i * c2i, wi = c1r * c2i + c1i * c2r;
        const double ar = xs[mp * nff + np], ai = xs[nff2 + mp * nff + np];
        yr = fma(wr, ar, fma(-wi, ai, yr));
        yi = fma(wr, ai, fma(wi, ar, yi));
      }
    }
    const size_t idx = ((size_t)in * nv + v) * nff2 + bb;
    yb[idx] = yr;
    yb[(size_t)total + idx] = yi;
  }
}

// Gather and basis change, independent of the transfer momentum.  Item
// (p, half-set harmonic j, output channel X).  For V = +S'_j and V = -S'_j:
//   M^X_AB(V) = sum_entries (+-) yb^{in}_{b1 b2}(v)          (eqn. proj_pos in bonds)
//   N^X(V) = C M^X(V) C^T                                  (back to form factors)
// and the real coefficients of cos(l.V/2), sin(l.V/2) for the inverse transform:
//   Re[e^{-il.V/2} N(V) + e^{+il.V/2} N(-V)] = cos (ReN+ + ReN-) + sin (ImN+ - ImN-).
__global__ void __launch_bounds__(256)
k_gather_g2(Batch b, const int4* __restrict__ items) {
  const int4 item = items[blockIdx.x];
  const int p = item.x;
  if (skip_point(b, p)) return;
  const DevTables& d = b.pts[p];
  const int j = item.y, X = item.z;
  const int nff = d.nff, nff2 = nff * nff, nsh = d.nsh, ncol = d.ncol;
  const int nv = 2 * nsh - 1;
  const int nvl = (j == 0) ? 1 : 2;
  const size_t ybim = (size_t)3 * nv * nff2;
  const double* yb = b.yb + d.ws_yb;
  double* g2 = b.g2 + d.ws_g2;
  extern __shared__ double sm[];
  double* Mre = sm;                  // [2][nff2]
  double* Mim = Mre + 2 * nff2;
  double* cr = Mim + 2 * nff2;       // coefficients c_{m,b} [nff2]
  double* ci = cr + nff2;
  for (int i = threadIdx.x; i < nff2; i += blockDim.x) {
    cr[i] = d.cre[i];
    ci[i] = d.cim[i];
  }
  for (int w = threadIdx.x; w < nvl * nff2; w += blockDim.x) {
    const int vi = w / nff2, ab = w % nff2;
    const int vf = (vi == 0) ? j : (nsh - 1 + j);
    const size_t row = ((size_t)X * nv + vf) * nff2 + ab;
    double re = 0.0, im = 0.0;
    const int e0 = d.mrow[row], e1 = d.mrow[row + 1];
    for (int e = e0; e < e1; e += 4) {
      // entries four at a time: independent loads, then the sums in order
      int32_t pk[4];
      double yr[4], yi[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) pk[u] = e + u < e1 ? d.ment[e + u] : -1;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        yr[u] = yi[u] = 0.0;
        if (pk[u] >= 0) {
          const int in = pk[u] & 3, b1 = (pk[u] >> 2) & 31, b2 = (pk[u] >> 7) & 31, v = (pk[u] >> 12) & 127;
          const size_t o = ((size_t)in * nv + v) * nff2 + b1 * nff + b2;
          yr[u] = yb[o];
          yi[u] = yb[ybim + o];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (pk[u] < 0) continue;
        if ((pk[u] >> 19) & 1) { re -= yr[u]; im -= yi[u]; } else { re += yr[u]; im += yi[u]; }
      }
    }
    Mre[vi * nff2 + ab] = re;
    Mim[vi * nff2 + ab] = im;
  }
  __syncthreads();
  for (int mn = threadIdx.x; mn < nff2; mn += blockDim.x) {
    const int m = mn / nff, n = mn % nff;
    const int sm_ = d.shell_of[m], sn = d.shell_of[n];
    double nr[2] = {0.0, 0.0}, ni[2] = {0.0, 0.0};
    for (int a = d.shell_start[sm_]; a < d.shell_start[sm_ + 1]; ++a) {
      const double c1r = cr[m * nff + a], c1i = ci[m * nff + a];
      for (int bb = d.shell_start[sn]; bb < d.shell_start[sn + 1]; ++bb) {
        const double c2r = cr[n * nff + bb], c2i = ci[n * nff + bb];
        const double wr = c1r * c2r - c1i * c2i, wi = c1r * c2i + c1i * c2r;
        for (int vi = 0; vi < nvl; ++vi) {
          const double mr = Mre[vi * nff2 + a * nff + bb], mi = Mim[vi * nff2 + a * nff + bb];
          nr[vi] += wr * mr - wi * mi;
          ni[vi] += wr * mi + wi * mr;
        }
      }
    }
    if (j == 0) {
      g2[((size_t)X * ncol + 0) * nff2 + mn] = nr[0];
    } else {
      g2[((size_t)X * ncol + j) * nff2 + mn] = nr[0] + nr[1];
      g2[((size_t)X * ncol + nsh - 1 + j) * nff2 + mn] = ni[0] - ni[1];
    }
  }
}

// Inverse transform K[ch][l][mn] = sum_k E[l][k] g2[ch][k][mn] in FP64 on the
// matrix cores: item (p, tile of 64 momenta l, tile of 64 columns (ch, mn));
// harmonics k in chunks of 16 through LDS; wave w owns 16 columns and 4
// accumulator tiles of v_mfma_f64_16x16x4f64 (16 momenta each; lane layout
// as in the forward transform).
__global__ void __launch_bounds__(256) k_dft_inv(Batch b, const int4* __restrict__ items) {
  __shared__ double Es[16][64 + 2];   // [k][l]
  __shared__ double Gs[16][64 + 2];   // [k][col]
  const int4 item = items[blockIdx.x];
  const int p = item.x;
  if (skip_point(b, p)) return;
  const DevTables& d = b.pts[p];
  const int nq = d.nq, ncol = d.ncol, nff2 = d.nff * d.nff, N = 3 * nff2;
  const int l0 = item.y * 64, c0 = item.z * 64, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, r16 = lane & 15, k4 = lane >> 4;
  const double* g2 = b.g2 + d.ws_g2;
  f64x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < ncol; k0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int r = e & 63, kk = e >> 6, l = l0 + r, k = k0 + kk;
      Es[kk][r] = (l < nq && k < ncol) ? d.eph[(size_t)l * ncol + k] : 0.0;
    }
    for (int e = tid; e < 16 * 64; e += 256) {
      const int kk = e >> 6, c = e & 63, col = c0 + c, k = k0 + kk;
      double v = 0.0;
      if (col < N && k < ncol) {
        const int ch = col / nff2, mn = col % nff2;
        v = g2[((size_t)ch * ncol + k) * nff2 + mn];
      }
      Gs[kk][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const double bv = Gs[kk + k4][16 * w + r16];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(Es[kk + k4][16 * t + r16], bv, acc[t], 0, 0, 0);
    }
    __syncthreads();
  }
  double* K = b.kinv64 + d.ws_k;
  const int col = c0 + 16 * w + r16;
  if (col >= N) return;
  const int ch = col / nff2, mn = col % nff2;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int l = l0 + 16 * t + 4 * j + k4;
      if (l < nq) K[((size_t)ch * nq + l) * nff2 + mn] = acc[t][j];
    }
}

// ======================================================= mixed precision
// BF16 hi/lo split with round to nearest even: x ~ hi + lo (about 16 mantissa
// bits); products hi*hi + hi*lo + lo*hi accumulate in FP32 on the matrix cores.
// v_mfma_f32_16x16x16bf16_1k operand layout: lane l holds A[l%16][4(l/16)+j],
// B[4(l/16)+j][l%16] (j = 0..3) and D[4(l/16)+j][l%16].
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

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

// Forward transform in split precision: the same contraction and output as
// the FP64 form (partial sums over transfer splits in xp, added in order by
// the bond-basis kernel), with products hi*hi + hi*lo + lo*hi of the BF16
// splits accumulated in FP32 over one split.  Item (p, column tile c, split
// s); splits start on multiples of 16 momenta.  Wave w owns 16 columns; per
// step of 16 momenta each lane loads its 4 values of X (split on the fly) and,
// for each of the KT harmonic tiles, one quad of the pre-split phase table
// laid out [u/4][kEpad][4] (zero beyond Nq), straight from the cache: there
// is no reuse across waves worth an LDS pass.
template <int KT>
__global__ void __launch_bounds__(256)
k_dft_fwd_mix(Batch b, const int4* __restrict__ items, const double* __restrict__ X) {
  const int4 item = items[blockIdx.x];
  const int p = item.x;
  if (skip_point(b, p)) return;
  const DevTables& d = b.pts[p];
  const int nq = d.nq, ncol = d.ncol, nff2 = d.nff * d.nff, N = 3 * nff2;
  const int split = item.z, nq16 = (nq + 15) >> 4;
  const int u0 = 16 * (int)((int64_t)nq16 * split / d.nsu);
  const int u1 = 16 * (int)((int64_t)nq16 * (split + 1) / d.nsu);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r16 = lane & 15, k4 = lane >> 4;
  const int col = item.y * 64 + 16 * w + r16;
  const bool cok = col < N;
  const int ch = cok ? col / nff2 : 0, mn = cok ? col % nff2 : 0;
  const double* xc = X + d.off + (size_t)ch * b.S + mn;
  const bf16x4* eh = reinterpret_cast<const bf16x4*>(d.ephq_hi);
  const bf16x4* el = reinterpret_cast<const bf16x4*>(d.ephq_lo);
  f32x4 acc[KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int ub = u0; ub < u1; ub += 16) {
    bf16x4 bh, bl;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int u = ub + 4 * k4 + j;
      unsigned short h = 0, l = 0;
      if (cok && u < nq) split_bf16(xc[(size_t)u * nff2], h, l);
      bh[j] = (short)h;
      bl[j] = (short)l;
    }
    const size_t qrow = (size_t)((ub >> 2) + k4) * kEpad;
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      const bf16x4 ah = eh[qrow + 16 * t + r16], al = el[qrow + 16 * t + r16];
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[t], 0, 0, 0);
    }
  }
  if (!cok) return;
  double* out = b.xp + d.ws_xp + (size_t)split * ncol * N;
#pragma unroll
  for (int t = 0; t < KT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = 16 * t + 4 * k4 + j;
      if (k < ncol) out[(size_t)k * N + col] = (double)acc[t][j];
    }
}

// Inverse transform in split precision: K[ch][l][mn] = sum_k E[l][k] g2[ch][k][mn]
// with FP32 accumulation of the three BF16 split products, stored in FP32.
// Item (p, tile of 64 momenta l, tile of 64 columns); wave w owns 16 columns
// and 4 accumulator tiles of 16 momenta.  The pre-split phase table is laid
// out [l][kEpad] (zero beyond Nq, rows padded to a multiple of 64), so a
// lane's 4 consecutive harmonics are one 8-byte load; g2 is split on the fly.
__global__ void __launch_bounds__(256)
k_dft_inv_mix(Batch b, const int4* __restrict__ items) {
  const int4 item = items[blockIdx.x];
  const int p = item.x;
  if (skip_point(b, p)) return;
  const DevTables& d = b.pts[p];
  const int nq = d.nq, ncol = d.ncol, nff2 = d.nff * d.nff, N = 3 * nff2;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r16 = lane & 15, k4 = lane >> 4;
  const int l0 = item.y * 64, col = item.z * 64 + 16 * w + r16;
  const bool cok = col < N;
  const int ch = cok ? col / nff2 : 0, mn = cok ? col % nff2 : 0;
  const double* gc = b.g2 + d.ws_g2 + (size_t)ch * ncol * nff2 + mn;
  const bf16x4* eh = reinterpret_cast<const bf16x4*>(d.ephr_hi);
  const bf16x4* el = reinterpret_cast<const bf16x4*>(d.ephr_lo);
  constexpr int QR = kEpad / 4;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < ncol; k0 += 16) {
    bf16x4 bh, bl;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + 4 * k4 + j;
      unsigned short h = 0, l = 0;
      if (cok && k < ncol) split_bf16(gc[(size_t)k * nff2], h, l);
      bh[j] = (short)h;
      bl[j] = (short)l;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const size_t a = (size_t)(l0 + 16 * t + r16) * QR + (k0 >> 2) + k4;
      const bf16x4 ah = eh[a], al = el[a];
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[t], 0, 0, 0);
    }
  }
  if (!cok) return;
  float* K = b.kinv + d.ws_k;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int l = l0 + 16 * t + 4 * k4 + j;
      if (l < nq) K[((size_t)ch * nq + l) * nff2 + mn] = acc[t][j];
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
// s = ln T, if scale_T, else 1) or V (mode 0), in FP64.
template <typename R>
__global__ void __launch_bounds__(256)
k_products(Batch b, const int4* __restrict__ items, const double* __restrict__ X, const R* __restrict__ Kall,
           double* __restrict__ out, int mode, int cross, int scale_T) {
  const int4 item = items[blockIdx.x];
  const int p = item.x;
  if (skip_point(b, p)) return;
  const DevTables& d = b.pts[p];
  const int nff = d.nff, nff2 = nff * nff, nq = d.nq;
  const int l = item.y;
  const double scale = scale_T ? b.Tp[p] : 1.0;
  const size_t S = (size_t)b.S;
  const R* K = Kall + d.ws_k;
  extern __shared__ double smem_prod[];
  R* Vs = reinterpret_cast<R*>(smem_prod);   // [3][nff2]
  R* Ch = Vs + 3 * nff2;                    // [2][nff2]
  R* Wm = Ch + 2 * nff2;                    // [nff2]
  R* T1 = Wm + nff2;                        // [3][nff2]
  R* T2 = T1 + 3 * nff2;                    // [3][nff2]
  for (int w = threadIdx.x; w < 3 * nff2; w += blockDim.x) {
    const int ch = w / nff2, mn = w % nff2;
    const R bare = (mn == 0) ? (R)d.U : (R)0;
    const R own = (R)X[ch * S + d.off + (size_t)l * nff2 + mn];
    const R kk = cross ? K[((size_t)ch * nq + l) * nff2 + mn] : (R)0;
    Vs[w] = bare + (ch == 0 ? -own : own) + kk;
  }
  if (mode == 0) {
    __syncthreads();
    for (int w = threadIdx.x; w < 3 * nff2; w += blockDim.x)
      out[(size_t)(w / nff2) * S + d.off + (size_t)l * nff2 + w % nff2] = (double)Vs[w];
    return;
  }
  for (int w = threadIdx.x; w < 2 * nff2; w += blockDim.x) {
    const int ch = w / nff2, mn = w % nff2;
    Ch[w] = (R)b.dchi[(size_t)ch * S + d.off + (size_t)l * nff2 + mn];
  }
  __syncthreads();
  const R* VP = Vs;
  const R* VC = Vs + nff2;
  const R* VD = Vs + 2 * nff2;
  for (int w = threadIdx.x; w < nff2; w += blockDim.x) Wm[w] = (R)2 * VD[w] - VC[w];
  __syncthreads();
  for (int w = threadIdx.x; w < 3 * nff2; w += blockDim.x) {
    const int which = w / nff2, m = (w % nff2) / nff, n = w % nff;
    const R* A = Ch + (which == 0 ? 0 : nff2) + m * nff;
    const R* B = which == 0 ? VP : (which == 1 ? VC : Wm);
    R v = 0;
    for (int k = 0; k < nff; ++k) v = fma(A[k], B[k * nff + n], v);
    T1[w] = v;
  }
  __syncthreads();
  for (int w = threadIdx.x; w < 3 * nff2; w += blockDim.x) {
    const int which = w / nff2, m = (w % nff2) / nff, n = w % nff;
    const R* A = (which == 0 ? VP : (which == 1 ? VC : Wm)) + m * nff;
    const R* B = T1 + which * nff2;
    R v = 0;
    for (int k = 0; k < nff; ++k) v = fma(A[k], B[k * nff + n], v);
    T2[w] = v;
  }
  __syncthreads();
  for (int w = threadIdx.x; w < nff2; w += blockDim.x) {
    const size_t o = d.off + (size_t)l * nff2 + w;
    out[o] = scale * (double)T2[w];
    out[S + o] = -scale * (double)T2[nff2 + w];
    out[2 * S + o] = 0.5 * scale * ((double)T2[2 * nff2 + w] - (double)T2[nff2 + w]);
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

// out = X + h sum_j coef_j k_j; frozen points untouched when skip_frozen
__global__ void __launch_bounds__(256)
k_axpy(Batch b, const int4* __restrict__ items, const double* __restrict__ X, SlopeSet ks, int nk,
       double h, double* __restrict__ out, int skip_frozen) {
  const int4 it = items[blockIdx.x];
  if (skip_frozen && skip_point(b, it.x)) return;
  size_t base;
  int n;
  if (!seg_range(b, it, base, n)) return;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const size_t e = base + i;
    double acc = 0.0;
    for (int j = 0; j < nk; ++j) acc = fma(ks.coef[j], ks.k[j][e], acc);
    out[e] = fma(h, acc, X[e]);
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
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double x = X[base + i];
      unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(x));
      if (x != x) bits = 0x7ff8000000000000ull;
      m = bits > m ? bits : m;
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

// Partial sums of ((h sum_j e_j k_j) / (atol + rtol max(|y0|,|y5|)))^2 per
// segment, in a fixed tree order (deterministic).
__global__ void __launch_bounds__(256)
k_errnorm(Batch b, const int4* __restrict__ items, const double* __restrict__ y0,
          const double* __restrict__ y5, SlopeSet ks, int nk, double h, double rtol, double atol,
          double* __restrict__ red_out) {
  __shared__ double red[256];
  const int4 it = items[blockIdx.x];
  double acc = 0.0;
  size_t base;
  int n;
  if (seg_range(b, it, base, n)) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const size_t e = base + i;
      double er = 0.0;
      for (int j = 0; j < nk; ++j) er = fma(ks.coef[j], ks.k[j][e], er);
      er *= h;
      const double sc = atol + rtol * fmax(fabs(y0[e]), fabs(y5[e]));
      const double r = er / sc;
      acc = fma(r, r, acc);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) red_out[blockIdx.x] = red[0];
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
// words and advance the step counter.
__global__ void k_step_end(unsigned long long* words, int npts, int* frozen, double* hist,
                           int* step, int nsteps, double xmax) {
  const int i = threadIdx.x;
  const int s = step[0];
  for (int p = i; p < npts; p += blockDim.x) {
    const double m = __longlong_as_double((long long)words[p]);
    if (!frozen[p]) {
      hist[(size_t)(s + 1) * npts + p] = m;
      if (!(m <= xmax)) frozen[p] = s + 1;
    }
    words[p] = 0ull;
  }
  __syncthreads();
  if (i == 0 && s < nsteps) step[0] = s + 1;
}

}  // namespace

// ============================================================== launchers
void launch_loops(const Launch& L, const ItemRange& r, int* queue, bool mixed, hipStream_t s) {
  if (r.n <= 0) return;
  if (!L.loop_persistent) queue = nullptr;
  const int grid = L.loop_persistent ? std::min(r.n, L.loop_blocks) : r.n;
  const dim3 blk(L.loop_threads);
  const size_t sm = L.loop_smem;
  const int4* it = L.loop_items + r.begin;
  switch (L.smax_max) {
    case 0:
      if (mixed) hipLaunchKernelGGL((k_loops<0, true>), dim3(grid), blk, sm, s, L.b, it, r.n, queue);
      else hipLaunchKernelGGL((k_loops<0, false>), dim3(grid), blk, sm, s, L.b, it, r.n, queue);
      break;
    case 2:
      if (mixed) hipLaunchKernelGGL((k_loops<2, true>), dim3(grid), blk, sm, s, L.b, it, r.n, queue);
      else hipLaunchKernelGGL((k_loops<2, false>), dim3(grid), blk, sm, s, L.b, it, r.n, queue);
      break;
    default:
      if (mixed) hipLaunchKernelGGL((k_loops<4, true>), dim3(grid), blk, sm, s, L.b, it, r.n, queue);
      else hipLaunchKernelGGL((k_loops<4, false>), dim3(grid), blk, sm, s, L.b, it, r.n, queue);
      break;
  }
}

void launch_chi_expand(const Launch& L, const ItemRange& r, const double* fin, double* dchi,
                       hipStream_t s) {
  if (r.n <= 0) return;
  hipLaunchKernelGGL(k_chi_expand, dim3(r.n), dim3(256), 0, s, L.b, L.exp_items + r.begin, fin, dchi);
}

void launch_front(const Launch& L, const Ranges& r, const double* X, bool mixed, hipStream_t s) {
  if (r.fwd.n > 0) {
    const int4* it = L.fwd_items + r.fwd.begin;
    const dim3 g(r.fwd.n), blk(256);
    if (mixed) {
      switch (L.fwd_kt) {
        case 1: hipLaunchKernelGGL(k_dft_fwd_mix<1>, g, blk, 0, s, L.b, it, X); break;
        case 2: hipLaunchKernelGGL(k_dft_fwd_mix<2>, g, blk, 0, s, L.b, it, X); break;
        case 3: hipLaunchKernelGGL(k_dft_fwd_mix<3>, g, blk, 0, s, L.b, it, X); break;
        default: hipLaunchKernelGGL(k_dft_fwd_mix<5>, g, blk, 0, s, L.b, it, X); break;
      }
    } else {
      switch (L.fwd_kt) {
        case 1: hipLaunchKernelGGL(k_dft_fwd_part<1>, g, blk, 0, s, L.b, it, X); break;
        case 2: hipLaunchKernelGGL(k_dft_fwd_part<2>, g, blk, 0, s, L.b, it, X); break;
        case 3: hipLaunchKernelGGL(k_dft_fwd_part<3>, g, blk, 0, s, L.b, it, X); break;
        default: hipLaunchKernelGGL(k_dft_fwd_part<5>, g, blk, 0, s, L.b, it, X); break;
      }
    }
  }
  if (r.basis.n > 0)
    hipLaunchKernelGGL(k_bond_basis, dim3(r.basis.n), dim3(256), 0, s, L.b,
                       L.basis_items + r.basis.begin);
  if (r.gather.n > 0)
    hipLaunchKernelGGL(k_gather_g2, dim3(r.gather.n), dim3(256), L.gather_smem, s, L.b,
                       L.gather_items + r.gather.begin);
  if (r.inv.n > 0) {
    if (mixed)
      hipLaunchKernelGGL(k_dft_inv_mix, dim3(r.inv.n), dim3(256), 0, s, L.b, L.inv_items + r.inv.begin);
    else
      hipLaunchKernelGGL(k_dft_inv, dim3(r.inv.n), dim3(256), 0, s, L.b, L.inv_items + r.inv.begin);
  }
}

void launch_back(const Launch& L, const Ranges& r, const double* X, double* out, int mode,
                 bool cross, bool scale_T, bool mixed, hipStream_t s) {
  if (r.prod.n <= 0) return;
  const int4* it = L.prod_items + r.prod.begin;
  if (mixed)
    hipLaunchKernelGGL(k_products<float>, dim3(r.prod.n), dim3(256), L.prod_smem / 2, s, L.b, it, X,
                       (const float*)L.b.kinv, out, mode, cross ? 1 : 0, scale_T ? 1 : 0);
  else
    hipLaunchKernelGGL(k_products<double>, dim3(r.prod.n), dim3(256), L.prod_smem, s, L.b, it, X,
                       (const double*)L.b.kinv64, out, mode, cross ? 1 : 0, scale_T ? 1 : 0);
}

void launch_axpy(const Launch& L, const ItemRange& r, const double* X, const double* const* k,
                 const double* coef, int nk, double h, double* out, bool skip_frozen, hipStream_t s) {
  if (r.n <= 0) return;
  SlopeSet ks{};
  for (int j = 0; j < nk; ++j) {
    ks.k[j] = k[j];
    ks.coef[j] = coef[j];
  }
  hipLaunchKernelGGL(k_axpy, dim3(r.n), dim3(256), 0, s, L.b, L.seg_items + r.begin, X, ks, nk, h,
                     out, skip_frozen ? 1 : 0);
}

void launch_maxabs(const Launch& L, const ItemRange& r, const double* X, unsigned long long* words,
                   hipStream_t s) {
  if (r.n <= 0) return;
  hipLaunchKernelGGL(k_maxabs, dim3(r.n), dim3(256), 0, s, L.b, L.seg_items + r.begin, X, words);
}

void launch_errnorm(const Launch& L, const ItemRange& r, const double* y0, const double* y5,
                    const double* const* k, const double* e, int nk, double h, double rtol,
                    double atol, double* red, hipStream_t s) {
  if (r.n <= 0) return;
  SlopeSet ks{};
  for (int j = 0; j < nk; ++j) {
    ks.k[j] = k[j];
    ks.coef[j] = e[j];
  }
  hipLaunchKernelGGL(k_errnorm, dim3(r.n), dim3(256), 0, s, L.b, L.seg_items + r.begin, y0, y5, ks,
                     nk, h, rtol, atol, red);
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
                     int nsteps, double xmax, hipStream_t s) {
  hipLaunchKernelGGL(k_step_end, dim3(1), dim3(256), 0, s, words, npts, frozen, hist, step, nsteps,
                     xmax);
}

const void* loop_kernel_symbol(int smax_max, bool mixed) {
  switch (smax_max) {
    case 0: return mixed ? (const void*)k_loops<0, true> : (const void*)k_loops<0, false>;
    case 2: return mixed ? (const void*)k_loops<2, true> : (const void*)k_loops<2, false>;
    default: return mixed ? (const void*)k_loops<4, true> : (const void*)k_loops<4, false>;
  }
}

}  // namespace tufrg
