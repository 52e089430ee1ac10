// Device bodies of the loop kernel (step ii. of Sec. 2.4, eqn. chis), shared
// by the stand-alone loop kernels, the combined loop + forward-transform
// launch and the single-launch right-hand side.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "loop_math.h"
#include "transforms.h"
#include "tufrg_internal.h"

namespace tufrg {
namespace {

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
// (p, slot * nsplit + split, q, ix << 16 | iy): one representative transfer
// momentum q = irr[slot] (point-group orbits; every other momentum follows by
// symmetry in the expansion kernel; on a non-uniform mesh every momentum is
// its own representative) with the indices of its x and y components in the
// shifted-cosine tables (in the item, which saves the kernel a dependent
// load), and one slice of the rows
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
template <int SMAX, bool MIXED, bool OMEGA, bool UNROLL>
__device__ __forceinline__ void loop_item(const Batch& b, const DevTables& d, int p, int item_b, int qa,
                                          double T, double* smem) {
  constexpr int NH = 2 * SMAX + 1;
  const int t = threadIdx.x;
  const int nsplit = d.nsplit, nchunk = d.nchunk;
  const int slot = item_b / nsplit, split = item_b % nsplit;
  const int lk = d.lk;
  const int rows = lk / 2 + 1;
  const int R0 = (int)((int64_t)rows * split / nsplit);
  const int R1 = (int)((int64_t)rows * (split + 1) / nsplit);
  const int nr = R1 - R0;
  const int ix = qa >> 16, iy = qa & 0xffff;   // axis indices of the momentum (from the item)
  // loop arguments: eps/(2T) for the temperature flow, eps/Om for the Omega cutoff
  const double inv_s = OMEGA ? 1.0 / T : 0.5 / T;

  double* y1 = smem;                        // cos(py + qy/2)        [nr]
  double* y2 = y1 + nr;                     // cos(py - qy/2)        [nr]
  double* pyt = y2 + nr;                    // weighted py harmonics [nr][NH]
  double* rs = pyt + nr * NH;               // row sums              [lk][2][NH]
  double* pxs = rs + lk * 2 * NH;           // px harmonics          [lk][NH]
  double* gh = pxs + lk * NH;               // harmonic partials     [nseg][2 nsh]
  for (int j = t; j < nr; j += blockDim.x) {
    const double* c = d.cshift_y + ((size_t)iy * lk + (R0 + j)) * 2;
    y1[j] = c[0];
    y2[j] = c[1];
  }
  for (int j = t; j < nr * NH; j += blockDim.x) pyt[j] = d.pytab[R0 * NH + j];
  for (int j = t; j < lk * 2 * NH; j += blockDim.x) rs[j] = 0.0;
  for (int j = t; j < lk * NH; j += blockDim.x) pxs[j] = d.pxtab[j];
  __syncthreads();

  const bool active = t < lk * nchunk;
  const int px = t % lk, c = t / lk;
  double acc[2][NH];
#pragma unroll
  for (int n = 0; n < NH; ++n) acc[0][n] = acc[1][n] = 0.0;
  if (active) {
    const double cx1 = d.cshift[((size_t)ix * lk + px) * 2];       // cos(px + qx/2)
    const double cx2 = d.cshift[((size_t)ix * lk + px) * 2 + 1];   // cos(px - qx/2)
    // alpha = eps(p + q/2) inv_s = A1 + B1 cos(py + qy/2); beta likewise
    const double A1 = (-2.0 * d.t * cx1 - d.mu) * inv_s;
    const double B1 = (-2.0 * d.t - 4.0 * d.tp * cx1) * inv_s;
    const double A2 = (-2.0 * d.t * cx2 - d.mu) * inv_s;
    const double B2 = (-2.0 * d.t - 4.0 * d.tp * cx2) * inv_s;
    const int r0 = (int)((int64_t)nr * c / nchunk);
    const int r1 = (int)((int64_t)nr * (c + 1) / nchunk);
    if constexpr (!MIXED) {
      auto row = [&](int r) {
        const double al = fma(B1, y1[r], A1);
        const double be = fma(B2, y2[r], A2);
        double dph, dpp;
        if constexpr (OMEGA) omega_dot_pair_t(al, be, dph, dpp, DevRcp());
        else loop_dot_pair_t(al, be, dph, dpp, DevRcp());
        const double* w = pyt + r * NH;
#pragma unroll
        for (int n = 0; n < NH; ++n) {
          acc[0][n] = fma(dpp, w[n], acc[0][n]);
          acc[1][n] = fma(dph, w[n], acc[1][n]);
        }
      };
      // two rows in flight where the launch can afford the registers
      if constexpr (UNROLL) {
#pragma unroll 2
        for (int r = r0; r < r1; ++r) row(r);
      } else {
        for (int r = r0; r < r1; ++r) row(r);
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
          if constexpr (OMEGA) omega_dot_pair_f32((float)al, (float)be, dph, dpp, RcpF());
          else loop_dot_pair_f32((float)al, (float)be, (float)(al - be), (float)(al + be), dph, dpp,
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
  // (the segment count follows the launch's loop geometry, not the block
  // size, so that every launch form sums in the same order)
  const int nout = 2 * d.nsh;
  int nseg = b.loop_threads / nout;
  if (nseg < 1) nseg = 1;
  for (int w = t; w < nout * nseg; w += blockDim.x) {
    const int o = w % nout, seg = w / nout;
    const int ch = o / d.nsh, j = o % d.nsh;
    const int sx = d.hx[j], sy = d.hy[j];          // sx >= 0
    const int ay = sy < 0 ? -sy : sy;
    const double sg = sy < 0 ? -1.0 : 1.0;
    // cos(px sx + py sy) = cos(px sx) cos(py |sy|) - sin(px sx) sgn(sy) sin(py |sy|);
    // four columns' operands are loaded before their terms are added in order
    const bool two = sx > 0 && ay > 0;
    double g = 0.0;
    int x = seg;
    for (; x + 3 * nseg < lk; x += 4 * nseg) {
      double c[4], rc[4], sn[4], rsn[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int xx = x + u * nseg;
        const double* r = rs + xx * 2 * NH + ch * NH;
        c[u] = pxs[xx * NH + sx];
        rc[u] = r[ay];
        sn[u] = two ? pxs[xx * NH + SMAX + sx] : 0.0;
        rsn[u] = two ? r[SMAX + ay] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        double v = c[u] * rc[u];
        if (two) v = fma(-sg * sn[u], rsn[u], v);
        g += v;
      }
    }
    for (; x < lk; x += nseg) {
      const double* r = rs + x * 2 * NH + ch * NH;
      double v = pxs[x * NH + sx] * r[ay];
      if (two) v = fma(-sg * pxs[x * NH + SMAX + sx], r[SMAX + ay], v);
      g += v;
    }
    gh[seg * nout + o] = g;
  }
  __syncthreads();
  for (int o = t; o < nout; o += blockDim.x) {
    double g = 0.0;
    int s = 0;
    for (; s + 3 < nseg; s += 4) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = gh[(s + u) * nout + o];
#pragma unroll
      for (int u = 0; u < 4; ++u) g += v[u];
    }
    for (; s < nseg; ++s) g += gh[s * nout + o];
    gh[o] = g;
  }
  __syncthreads();
  // ghat_X(q, S_j) = sgn_X gh_j / (4 T^2 Nk) (pp carries the minus sign of
  // dL^pp/dT = -Dh/(4T^2); with the Omega cutoff T is Om and h is f), written
  // to slice `split` of the representative's
  // harmonics; chi'_mn = sum_j Ebub_{mn,j} ghat(q, S_j) follows in the
  // expansion kernel.
  const double base = 1.0 / (4.0 * T * T * (double)lk * (double)lk);
  for (int o = t; o < nout; o += blockDim.x)
    b.ghat[d.ws_gh + ((size_t)split * d.nirr + slot) * nout + o] = gh[o] * (o < d.nsh ? -base : base);
  __syncthreads();
}

// The point's temperature: from the launch's TArg when there is one (fused
// launches), else from the per-point array.
__device__ __forceinline__ double point_T(const Batch& b, const TArg* ta, int p) {
  if (ta != nullptr) {
    if (ta->mode == 1 && p >= ta->p0 && p < ta->p0 + ta->n) return ta->v[p - ta->p0];
    if (ta->mode == 2) return ta->Ttab[4 * ta->step[0] + ta->stage];
    if (ta->mode == 3) return exp(fma(ta->c, ta->h[p], ta->s[p]));
  }
  return b.Tp[p];
}

// Runs the body compiled for the item's own smax.
template <int SMAX, bool MIXED, bool OMEGA, bool UNROLL>
__device__ __forceinline__ void loop_smax(const Batch& b, const DevTables& d, int p, int item_b, int qa,
                                          double T, double* smem) {
  if constexpr (SMAX >= 4) {
    if (d.smax == 4) {
      loop_item<4, MIXED, OMEGA, UNROLL>(b, d, p, item_b, qa, T, smem);
      return;
    }
  }
  if constexpr (SMAX >= 2) {
    if (d.smax == 2) {
      loop_item<2, MIXED, OMEGA, UNROLL>(b, d, p, item_b, qa, T, smem);
      return;
    }
  }
  loop_item<0, MIXED, OMEGA, UNROLL>(b, d, p, item_b, qa, T, smem);
}

// ONE (a single-point launch, compiled for the point's own smax): point 0,
// its tables from the launch's arguments
template <int SMAX, bool MIXED, bool OMEGA, bool UNROLL, bool ONE = false>
__device__ __forceinline__ void loop_dispatch(const Batch& b, const int4 item, double* smem,
                                              const TArg* ta = nullptr) {
  const int p = ONE ? 0 : item.x;
  if (skip_point(b, p)) return;
  const DevTables& d = point_tables<ONE>(b, p);
  if constexpr (ONE) loop_item<SMAX, MIXED, OMEGA, UNROLL>(b, d, p, item.y, item.w, point_T(b, ta, p), smem);
  else loop_smax<SMAX, MIXED, OMEGA, UNROLL>(b, d, p, item.y, item.w, point_T(b, ta, p), smem);
}

}  // namespace
}  // namespace tufrg
