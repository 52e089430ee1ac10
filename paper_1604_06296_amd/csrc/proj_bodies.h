// Device bodies of the projections' middle step shared by the per-stage
// kernels and the single-launch right-hand side.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "transforms.h"
#include "tufrg_internal.h"

namespace tufrg {
namespace {

// Bond basis of the transformed propagators, for every harmonic of the full
// list v (+S'_j for v < nsh, -S'_{v-nsh+1} otherwise):
//   yb[in][v][b1 b2] = sum_{m' in shell(b1), n' in shell(b2)} c_{m'b1} c_{n'b2} xt^{in}_{m'n'}(v)
// with xt(-S') = conj(xt(S')).  These are the bond-space Fourier coefficients
// Yhat_{R1R2}(W) of the propagators at frequency 2W - R1 - R2 = v.
// Item (p, in * nv + v, r0, r1): the rows m' in [r0, r1) (whole shells) of the
// harmonic's transform and the coefficients are staged in LDS; threads own
// bond pairs (b1, b2) with b1 in [r0, r1), which need only those rows since
// c is block diagonal over shells.  The transform is the in-order FP64 sum
// of the forward-transform splits (xp), taken here.
struct alignas(16) BasisShared {
  double cs[2 * 441];
  double xs[2 * 441];
  double ts[2 * 441];
};
// WIDE: all splits of a sum in one round of loads where the splits are few
// (the launches of small contexts); otherwise 8 splits of 4 sums per round
// (fewer registers for the many blocks of large contexts).
template <bool ONE, bool WIDE, int NT = 256>
__device__ __forceinline__ void basis_body(const Batch& b, const int4 item, BasisShared& sh) {
  const int p = ONE ? 0 : item.x;
  if (skip_point(b, p)) return;
  const DevTables& d = point_tables<ONE>(b, p);
  const int nff = d.nff, nff2 = nff * nff, nsh = d.nsh, ncol = d.ncol, nv = 2 * nsh - 1;
  const int total = 3 * nv * nff2;
  const int in = item.y / nv, v = item.y % nv;
  const int r0 = item.z, r1 = item.w;   // rows m' (and b1) of the item
  const int j = v < nsh ? v : v - nsh + 1;
  const double sim = v < nsh ? 1.0 : -1.0;
  double* cs = sh.cs;
  double* xs = sh.xs;
  {
    // 2 (r1 - r0) nff sums of nsu terms (real and imaginary parts of the
    // item's rows); each of the NT threads keeps up to kSums sums and kSplits
    // splits of each in flight, then adds them in split order
    constexpr int kSums = WIDE ? 2 : 4, kSplits = WIDE ? 16 : 8;
    const int N = 3 * nff2, nrow = (r1 - r0) * nff, nel = 2 * nrow, e_lo = r0 * nff;
    const size_t sstride = (size_t)ncol * N;
    const double* base = b.xp + d.ws_xp + (size_t)in * nff2;
    const double inv = 1.0 / (double)d.nq;
    for (int e0 = threadIdx.x; e0 < nel; e0 += kSums * NT) {
      const double* src[kSums];
      bool ok[kSums];
      double acc[kSums];
      int dst[kSums];   // element of xs: [re | im][m' n']
#pragma unroll
      for (int s4 = 0; s4 < kSums; ++s4) {
        const int e = e0 + NT * s4;
        const bool im = e >= nrow;
        const int g = e_lo + (im ? e - nrow : e);
        ok[s4] = e < nel && (!im || j > 0);
        src[s4] = base + (size_t)(im ? nsh - 1 + j : j) * N + g;
        dst[s4] = e < nel ? (im ? nff2 + g : g) : -1;
        acc[s4] = 0.0;
      }
      for (int sp0 = 0; sp0 < d.nsu; sp0 += kSplits) {
        double v[kSums][kSplits];
#pragma unroll
        for (int s4 = 0; s4 < kSums; ++s4)
#pragma unroll
          for (int u = 0; u < kSplits; ++u)
            v[s4][u] = (ok[s4] && sp0 + u < d.nsu) ? src[s4][(size_t)(sp0 + u) * sstride] : 0.0;
#pragma unroll
        for (int s4 = 0; s4 < kSums; ++s4)
#pragma unroll
          for (int u = 0; u < kSplits; ++u) acc[s4] += v[s4][u];
      }
#pragma unroll
      for (int s4 = 0; s4 < kSums; ++s4)
        if (dst[s4] >= 0) xs[dst[s4]] = (dst[s4] < nff2 ? 1.0 : sim) * acc[s4] * inv;
    }
  }
  for (int i = threadIdx.x; i < nff2; i += blockDim.x) {
    cs[i] = d.cre[i];
    cs[nff2 + i] = d.cim[i];
  }
  __syncthreads();
  // the change of basis as two products through shared memory:
  // ts[m'][b2] = sum_{n' in shell(b2)} c_{n'b2} xt_{m'n'}, then
  // yb[b1 b2] = sum_{m' in shell(b1)} c_{m'b1} ts[m'][b2]
  double* ts = sh.ts;
  for (int i = r0 * nff + threadIdx.x; i < r1 * nff; i += blockDim.x) {
    const int mp = i / nff, b2 = i % nff;
    const int s2 = d.shell_of[b2];
    const int n0 = d.shell_start[s2], n1 = d.shell_start[s2 + 1];
    double tr = 0.0, ti = 0.0;
    for (int np = n0; np < n1; ++np) {
      const double c2r = cs[np * nff + b2], c2i = cs[nff2 + np * nff + b2];
      const double ar = xs[mp * nff + np], ai = xs[nff2 + mp * nff + np];
      tr = fma(c2r, ar, fma(-c2i, ai, tr));
      ti = fma(c2r, ai, fma(c2i, ar, ti));
    }
    ts[i] = tr;
    ts[nff2 + i] = ti;
  }
  __syncthreads();
  double* yb = b.yb + d.ws_yb;
  for (int bb = r0 * nff + threadIdx.x; bb < r1 * nff; bb += blockDim.x) {
    const int b1 = bb / nff, b2 = bb % nff;
    const int s1 = d.shell_of[b1];
    const int m0 = d.shell_start[s1], m1 = d.shell_start[s1 + 1];
    double yr = 0.0, yi = 0.0;
    for (int mp = m0; mp < m1; ++mp) {
      const double c1r = cs[mp * nff + b1], c1i = cs[nff2 + mp * nff + b1];
      const double tr = ts[mp * nff + b2], ti = ts[nff2 + mp * nff + b2];
      yr = fma(c1r, tr, fma(-c1i, ti, yr));
      yi = fma(c1r, ti, fma(c1i, tr, yi));
    }
    const size_t idx = ((size_t)in * nv + v) * nff2 + bb;
    yb[idx] = yr;
    yb[(size_t)total + idx] = yi;
  }
}

// Gather and basis change, independent of the transfer momentum.  For
// V = +S'_j and V = -S'_j:
//   M^X_AB(V) = sum_entries (+-) yb^{in}_{b1 b2}(v)          (eqn. proj_pos in bonds)
//   N^X(V) = C M^X(V) C^T                                  (back to form factors)
// and the real coefficients of cos(l.V/2), sin(l.V/2) for the inverse transform:
//   Re[e^{-il.V/2} N(V) + e^{+il.V/2} N(-V)] = cos (ReN+ + ReN-) + sin (ImN+ - ImN-).
// C is block diagonal over shells, so the item is (p, half-set harmonic j,
// (X, shell of m, shell of n)): one wave gathers the shell block of M (at
// most kShellMax^2 bond pairs per harmonic) into LDS and transforms it.  The
// item packs j, X and both shells' start and size (y) and the index of its
// rows' entries (w: cap per row, absolute yb offsets of the real and
// imaginary parts, a negative imaginary offset for a negated entry, a
// negative real offset for padding), so that the yb loads wait for two loads
// only; the entries of a row are added in the order of the entry lists.
// The wave's work is two phases with a barrier of the caller's block between
// them (a block of one wave, or of several waves running one item each, all
// of which call both phases); the second phase has a block barrier of its own.
struct GatherShared {
  double Mre[2][kShellMax * kShellMax];
  double Mim[2][kShellMax * kShellMax];
  double C1[2][kShellMax * kShellMax];   // c_{m a}, m and a in shell sm (re, im)
  double C2[2][kShellMax * kShellMax];   // c_{n b}, n and b in shell sn
  double Tre[2][kShellMax * kShellMax];  // M C^T of the shell block, [a][n]
  double Tim[2][kShellMax * kShellMax];
};

// phase 1 (lane of the wave): the rows' entries and their yb values, and the
// shells' coefficients, into LDS
__device__ __forceinline__ void gather_load(const Batch& b, const int4 item, const int2* __restrict__ gent,
                                            int cap, int lane, GatherShared& sh) {
  const int p = item.x;
  const int j = item.y & 0xff, na = (item.y >> 10) & 15, nb = (item.y >> 14) & 15;
  const int a0 = (item.y >> 18) & 31, b0 = (item.y >> 23) & 31;
  const int nab = na * nb, nvl = j == 0 ? 1 : 2;
  // the rows' entries and their yb values first: they depend on the item only
  for (int w = lane; w < nvl * nab; w += 64) {
    const int2* en = gent + item.w + (size_t)w * cap;
    double re = 0.0, im = 0.0;
    for (int e = 0; e < cap; e += 4) {
      int2 pk[4];
      double yr[4], yi[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) pk[u] = e + u < cap ? en[e + u] : make_int2(-1, 0);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        yr[u] = yi[u] = 0.0;
        if (pk[u].x >= 0) {
          yr[u] = b.yb[pk[u].x];
          yi[u] = b.yb[pk[u].y >= 0 ? pk[u].y : -pk[u].y - 1];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (pk[u].x < 0) continue;
        if (pk[u].y < 0) { re -= yr[u]; im -= yi[u]; } else { re += yr[u]; im += yi[u]; }
      }
    }
    sh.Mre[w / nab][w % nab] = re;
    sh.Mim[w / nab][w % nab] = im;
  }
  const DevTables& d = b.pts[p];
  const int nff = d.nff;
  if (lane < na * na) {
    const int i = lane, c = (a0 + i / na) * nff + a0 + i % na;
    sh.C1[0][i] = d.cre[c];
    sh.C1[1][i] = d.cim[c];
  }
  if (lane < nb * nb) {
    const int i = lane, c = (b0 + i / nb) * nff + b0 + i % nb;
    sh.C2[0][i] = d.cre[c];
    sh.C2[1][i] = d.cim[c];
  }
}

// phase 2 (after the barrier): N = C M C^T of the shell block as two
// products, T = M C^T (each entry a sum over b in bond order) and then
// N = C T (a sum over a), with a barrier of the caller's block between them,
// and its inverse-transform coefficients into g2
__device__ __forceinline__ void gather_store(const Batch& b, const int4 item, int lane, GatherShared& sh) {
  const int p = item.x;
  const int j = item.y & 0xff, X = (item.y >> 8) & 3, na = (item.y >> 10) & 15, nb = (item.y >> 14) & 15;
  const int a0 = (item.y >> 18) & 31, b0 = (item.y >> 23) & 31;
  const int nab = na * nb, nvl = j == 0 ? 1 : 2;
  for (int w = lane; w < nvl * nab; w += 64) {
    const int vi = w / nab, a = w % nab / nb, n = w % nb;   // T[vi][a][n]
    double tr = 0.0, ti = 0.0;
    for (int bb = 0; bb < nb; ++bb) {
      const double c2r = sh.C2[0][n * nb + bb], c2i = sh.C2[1][n * nb + bb];
      const double mr = sh.Mre[vi][a * nb + bb], mi = sh.Mim[vi][a * nb + bb];
      tr += c2r * mr - c2i * mi;
      ti += c2r * mi + c2i * mr;
    }
    sh.Tre[vi][a * nb + n] = tr;
    sh.Tim[vi][a * nb + n] = ti;
  }
  __syncthreads();
  const DevTables& d = b.pts[p];
  const int nff = d.nff, nff2 = nff * nff, nsh = d.nsh, ncol = d.ncol;
  double* g2 = b.g2 + d.ws_g2;
  for (int w = lane; w < nab; w += 64) {
    const int m = a0 + w / nb, n = b0 + w % nb, mn = m * nff + n;
    double nr[2] = {0.0, 0.0}, ni[2] = {0.0, 0.0};
    for (int a = 0; a < na; ++a) {
      const double c1r = sh.C1[0][(m - a0) * na + a], c1i = sh.C1[1][(m - a0) * na + a];
      for (int vi = 0; vi < nvl; ++vi) {
        const double tr = sh.Tre[vi][a * nb + n - b0], ti = sh.Tim[vi][a * nb + n - b0];
        nr[vi] += c1r * tr - c1i * ti;
        ni[vi] += c1r * ti + c1i * tr;
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

}  // namespace
}  // namespace tufrg
