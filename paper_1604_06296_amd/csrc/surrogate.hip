// Loop surrogate: features and targets of the loop harmonics, training-set
// sampling, and the inference pipeline with its exact fallback.
//
// A query is one (q, S_j) of a point at its temperature; the loop harmonic
// ghat_X(q, S_j) (X = pp, ph) determines the projected loops through
// chi'_mn(q) = sum_j Ebub_{mn,j} ghat(q, S_j).  Features (9):
//   (qx/pi, qy/pi, log10 T, mu/t, t'/t, R_a/2, R_b/2)
// with (R_a, R_b) the canonical bond pair of S_j; targets (4):
//   (T (1 + 4T) ghat_pp, (1 + 4T^2) ghat_ph, 0, 0).
// Inference runs on the representatives of the transfer momenta (point-group
// orbits; the expansion kernel serves the rest).  One or two networks predict
// every query; a representative takes the exact loop kernel when two networks
// disagree by more than tol relative to its largest predicted harmonic, when
// it is in this call's check set (slot = phase mod stride, rotating per
// call), or when its fallback flag is set.  Checked representatives compare
// prediction and exact harmonics; a failure (relative residual above tol)
// flags it and the representatives of its 8 grid neighbours, and a later
// passing check clears the flag.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "tufrg_internal.h"

namespace tufrg {
namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

__device__ __forceinline__ void target_scales(double T, double& spp, double& sph) {
  spp = T * (1.0 + 4.0 * T);
  sph = 1.0 + 4.0 * T * T;
}

__device__ __forceinline__ void write_features(const DevTables& d, double T, int q, int j, float* x) {
  const int ix = q / d.lq, iy = q % d.lq;
  x[0] = (float)(2.0 * (double)(ix - d.lq / 2) / (double)d.lq);
  x[1] = (float)(2.0 * (double)(iy - d.lq / 2) / (double)d.lq);
  x[2] = (float)log10(T);
  x[3] = (float)(d.mu / d.t);
  x[4] = (float)(d.tp / d.t);
  const int32_t* pr = d.pairs + 4 * j;
  x[5] = 0.5f * (float)pr[0];
  x[6] = 0.5f * (float)pr[1];
  x[7] = 0.5f * (float)pr[2];
  x[8] = 0.5f * (float)pr[3];
}

// harmonic o = ch * nsh + j of representative `slot`: the sum of its loop slices
__device__ __forceinline__ double slot_harmonic(const Batch& b, const DevTables& d, int slot, int o) {
  const int nout = 2 * d.nsh;
  double v = 0.0;
  for (int s = 0; s < d.nsplit; ++s) v += b.ghat[d.ws_gh + ((size_t)s * d.nirr + slot) * nout + o];
  return v;
}

// exact harmonic o = ch * nsh + j of any momentum q, through the symmetry map
__device__ __forceinline__ double exact_harmonic(const Batch& b, const DevTables& d, int q, int o) {
  const int nsh = d.nsh, ch = o / nsh, j = o % nsh;
  const int32_t pk = d.symmap[(size_t)q * nsh + j];
  const double v = slot_harmonic(b, d, pk & 0xffff, ch * nsh + ((pk >> 16) & 0x7f));
  return ((pk >> 24) & 1) ? -v : v;
}

// summed harmonics of point p: out[gh_off + q * 2 nsh + o]
__global__ void k_ghat_sum(Batch b, int p, double* __restrict__ out) {
  const DevTables& d = b.pts[p];
  const int nout = 2 * d.nsh;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)d.nq * nout) return;
  out[d.gh_off + i] = exact_harmonic(b, d, (int)(i / nout), (int)(i % nout));
}

// n training samples (p, q, j) drawn uniformly with a counter-based hash
__global__ void k_sur_dataset(Batch b, int npts, int64_t n, uint64_t seed, float* __restrict__ x,
                              float* __restrict__ y, int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t h1 = mix64(seed ^ mix64((uint64_t)i));
  const uint64_t h2 = mix64(h1), h3 = mix64(h2);
  const int p = (int)(h1 % (uint64_t)npts);
  const DevTables& d = b.pts[p];
  const int q = (int)(h2 % (uint64_t)d.nq);
  const int j = (int)(h3 % (uint64_t)d.nsh);
  const double T = b.Tp[p];
  write_features(d, T, q, j, x + 9 * i);
  double spp, sph;
  target_scales(T, spp, sph);
  y[4 * i + 0] = (float)(spp * exact_harmonic(b, d, q, j));
  y[4 * i + 1] = (float)(sph * exact_harmonic(b, d, q, d.nsh + j));
  y[4 * i + 2] = 0.0f;
  y[4 * i + 3] = 0.0f;
  if (idx) {
    idx[3 * i + 0] = p;
    idx[3 * i + 1] = q;
    idx[3 * i + 2] = j;
  }
}

// features of every query (representative slot, j) of point p
__global__ void k_sur_features(Batch b, int p, float* __restrict__ x) {
  const DevTables& d = b.pts[p];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)d.nirr * d.nsh) return;
  write_features(d, b.Tp[p], d.irr[i / d.nsh], (int)(i % d.nsh), x + 9 * i);
}

__device__ __forceinline__ double block_max64(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 32; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// one block of 64 threads per representative slot q: ensemble mean as the
// predicted harmonics, disagreement test, and the momenta that take the
// exact kernel
__global__ void __launch_bounds__(64)
k_sur_pred(Batch b, int p, const float* __restrict__ ya, const float* __restrict__ yb, SurState st) {
  __shared__ double red[64];
  const DevTables& d = b.pts[p];
  const int q = blockIdx.x, nsh = d.nsh, nout = 2 * nsh;
  double spp, sph;
  target_scales(b.Tp[p], spp, sph);
  double dmax = 0.0, vmax = 0.0;
  for (int o = threadIdx.x; o < nout; o += 64) {
    const int j = o % nsh, c = o / nsh;
    const size_t i = ((size_t)q * nsh + j) * 4 + c;
    const double inv = c == 0 ? 1.0 / spp : 1.0 / sph;
    const double a = (double)ya[i] * inv, bb = (double)yb[i] * inv;
    const double m = 0.5 * (a + bb);
    st.pred[(size_t)q * nout + o] = m;
    dmax = fmax(dmax, fabs(a - bb));
    vmax = fmax(vmax, fabs(m));
  }
  dmax = block_max64(dmax, red);
  vmax = block_max64(vmax, red);
  if (threadIdx.x == 0) {
    const int phase = *st.phase;
    const bool disagree = !(dmax <= st.tol * vmax);
    st.need[q] = (disagree || st.state[q] != 0 || q % st.stride == phase) ? 1 : 0;
  }
}

// Loop items (p, slot * nsplit + s, flat momentum of the representative) of
// the representatives that need the exact kernel, in increasing slot (one
// block, deterministic prefix sum); count = items.  Below, q always denotes a
// representative slot.
__global__ void __launch_bounds__(1024) k_sur_compact(Batch b, int p, SurState st) {
  __shared__ int sums[1024];
  const DevTables& d = b.pts[p];
  const int nq = d.nirr, ns = d.nsplit;
  const int per = (nq + 1023) / 1024;
  const int q0 = threadIdx.x * per, q1 = min(nq, q0 + per);
  int c = 0;
  for (int q = q0; q < q1; ++q) c += st.need[q];
  sums[threadIdx.x] = c;
  __syncthreads();
  for (int s = 1; s < 1024; s <<= 1) {
    const int v = (int)threadIdx.x >= s ? sums[threadIdx.x - s] : 0;
    __syncthreads();
    sums[threadIdx.x] += v;
    __syncthreads();
  }
  int pos = sums[threadIdx.x] - c;     // exclusive prefix: first slot of this thread
  for (int q = q0; q < q1; ++q)
    if (st.need[q]) {
      for (int s = 0; s < ns; ++s) st.items[(size_t)pos * ns + s] =
            make_int4(p, q * ns + s, d.irr[q], ((d.irr[q] / d.lq) << 16) | (d.irr[q] % d.lq));
      ++pos;
    }
  if (threadIdx.x == 1023) {
    const int total = sums[1023];
    *st.count = total * ns;
    st.stats[0] += (unsigned long long)total;
    st.stats[1] += (unsigned long long)nq;
  }
}

// one block of 64 threads per q: final harmonics (exact where computed) and
// the residual check of this call's check set
__global__ void __launch_bounds__(64) k_sur_select(Batch b, int p, SurState st) {
  __shared__ double red[64];
  const DevTables& d = b.pts[p];
  const int q = blockIdx.x, nout = 2 * d.nsh;
  const bool exact = st.need[q] != 0;
  double rmax = 0.0, emax = 0.0;
  for (int o = threadIdx.x; o < nout; o += 64) {
    const size_t k = (size_t)q * nout + o;
    double v = st.pred[k];
    if (exact) {
      const double e = slot_harmonic(b, d, q, o);
      rmax = fmax(rmax, fabs(v - e));
      emax = fmax(emax, fabs(e));
      v = e;
    }
    st.fin[k] = v;
  }
  rmax = block_max64(rmax, red);
  emax = block_max64(emax, red);
  if (threadIdx.x == 0) {
    const bool checked = q % st.stride == *st.phase;
    const int f = (checked && !(rmax <= st.tol * emax)) ? 1 : 0;
    st.fail[q] = f;
    if (f) atomicAdd(&st.stats[2], 1ull);
  }
}

// fallback flags: checked representatives take their check result; a
// failure also flags the representatives of the 8 grid neighbours (periodic
// grid); then the check phase advances
__global__ void k_sur_state(Batch b, int p, SurState st) {
  const DevTables& d = b.pts[p];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= d.nirr) return;
  const int lq = d.lq, q = d.irr[r], ix = q / lq, iy = q % lq;
  const bool checked = r % st.stride == *st.phase;
  int f = checked ? st.fail[r] : st.state[r];
  for (int dx = -1; dx <= 1; ++dx)
    for (int dy = -1; dy <= 1; ++dy) {
      if (dx == 0 && dy == 0) continue;
      const int nb = ((ix + dx + lq) % lq) * lq + (iy + dy + lq) % lq;
      if (st.fail[d.symmap[(size_t)nb * d.nsh] & 0xffff]) f = 1;
    }
  st.state[r] = f;
}

__global__ void k_sur_advance(SurState st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *st.phase = (*st.phase + 1) % st.stride;
}

}  // namespace

// The launchers below that read loop harmonics require L.b.ghat (they launch
// nothing without it).
void launch_ghat_sum(const Launch& L, int p, const DevTables& d, double* out, hipStream_t s) {
  if (L.b.ghat == nullptr) return;
  const int64_t n = (int64_t)d.nq * 2 * d.nsh;
  hipLaunchKernelGGL(k_ghat_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, L.b, p, out);
}

void launch_sur_dataset(const Launch& L, int npts, int64_t n, uint64_t seed, float* x, float* y,
                        int32_t* idx, hipStream_t s) {
  if (n <= 0 || L.b.ghat == nullptr) return;
  hipLaunchKernelGGL(k_sur_dataset, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, L.b, npts, n, seed,
                     x, y, idx);
}

void launch_surrogate_front(const Launch& L, int p, const DevTables& d, float* x, hipStream_t s) {
  const int64_t n = (int64_t)d.nirr * d.nsh;
  hipLaunchKernelGGL(k_sur_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, L.b, p, x);
}

void launch_surrogate_decide(const Launch& L, int p, const DevTables& d, const float* ya, const float* yb,
                             const SurState& st, hipStream_t s) {
  hipLaunchKernelGGL(k_sur_pred, dim3(d.nirr), dim3(64), 0, s, L.b, p, ya, yb, st);
  hipLaunchKernelGGL(k_sur_compact, dim3(1), dim3(1024), 0, s, L.b, p, st);
}

void launch_surrogate_finish(const Launch& L, int p, const DevTables& d, const SurState& st, hipStream_t s) {
  if (L.b.ghat == nullptr) return;
  hipLaunchKernelGGL(k_sur_select, dim3(d.nirr), dim3(64), 0, s, L.b, p, st);
  hipLaunchKernelGGL(k_sur_state, dim3((d.nirr + 255) / 256), dim3(256), 0, s, L.b, p, st);
  hipLaunchKernelGGL(k_sur_advance, dim3(1), dim3(64), 0, s, st);
}

}  // namespace tufrg
