// HIP kernels for gfx950 (CDNA4): loops, projections, products and ODE helpers
// of the TUfRG flow right-hand side.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "loop_math.h"
#include "tufrg_internal.h"

namespace tufrg {
namespace {

constexpr int kBubThreads = 512;   // upper bound of the loop kernel's block size

// ------------------------------------------------------------------ loops
// Step ii.) of Sec. 2.4, eqn. chis, at one temperature.  One block per
// transfer momentum q.  Threads own one px column of the fine grid and a
// chunk of py rows (py in [0, Lk/2] only: the loop weight is even in p, the
// self-paired rows py = 0, Lk/2 carry weight 1 and the others weight 2).
// Each thread accumulates row sums of the loop derivative against cos(n py)
// and sin(n py), n <= SMAX; the block then contracts the rows against
// cos(px Sx), sin(px Sx) into ghat(q, S) = (1/Nk) sum_p L'(p) cos(p.S) for
// the half set of harmonics S in bonds + bonds, and finally
// chi'_mn(q) = sum_S Ebub_{mn,S} ghat(q, S).
struct DevRcp {
  __device__ double operator()(double x) const {
    double r = __builtin_amdgcn_rcp(x);       // hardware estimate, refined by Newton steps
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
  }
};

template <int SMAX>
__global__ void __launch_bounds__(kBubThreads)
k_loops_f64(DevTables d, double T, int nsplit, int nchunk, double* __restrict__ dchi, int64_t S,
            double* __restrict__ dpart) {
  constexpr int NH = 2 * SMAX + 1;     // row sums per channel: cos n=0..SMAX, sin n=1..SMAX
  const int q = blockIdx.x / nsplit, split = blockIdx.x % nsplit;
  const int lk = d.lk;
  const int rows = lk / 2 + 1;
  const int R0 = (int)((int64_t)rows * split / nsplit);
  const int R1 = (int)((int64_t)rows * (split + 1) / nsplit);
  const int nr = R1 - R0;
  const int lq = d.lq;
  const int ix = q / lq, iy = q % lq;
  const double inv2T = 0.5 / T;

  extern __shared__ double smem[];
  double* y1 = smem;                        // cos(py + qy/2)        [nr]
  double* y2 = y1 + nr;                     // cos(py - qy/2)        [nr]
  double* pyt = y2 + nr;                    // weighted py harmonics [nr][NH]
  double* rs = pyt + nr * NH;               // row sums              [lk][2][NH]
  double* gh = rs + lk * 2 * NH;            // harmonic partials     [nseg][2 nsh]

  // cos(py +- qy/2) for this block's rows from the init-time table [lq][lk][2]
  for (int j = threadIdx.x; j < nr; j += blockDim.x) {
    const double* c = d.cshift + ((size_t)iy * lk + (R0 + j)) * 2;
    y1[j] = c[0];
    y2[j] = c[1];
  }
  for (int j = threadIdx.x; j < nr * NH; j += blockDim.x) pyt[j] = d.pytab[R0 * NH + j];
  for (int j = threadIdx.x; j < lk * 2 * NH; j += blockDim.x) rs[j] = 0.0;
  __syncthreads();

  // thread t owns column px = t % lk and the chunk c = t / lk of this block's rows
  const int t = threadIdx.x;
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
  for (int w = threadIdx.x; w < nout * nseg; w += blockDim.x) {
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
  for (int o = threadIdx.x; o < nout; o += blockDim.x) {
    double g = 0.0;
    for (int s = 0; s < nseg; ++s) g += gh[s * nout + o];
    gh[o] = g;
  }
  __syncthreads();
  // chi'_mn = sgn / (4 T^2 Nk) sum_j Ebub_{mn,j} ghat_j (pp carries the minus
  // sign of dL^pp/dT = -Dh/(4T^2)).  With one split the block writes chi'
  // itself; otherwise its rows' share goes to slice `split` of dpart
  // [nsplit][2][Nq][nff^2] and the consumer adds the slices in split order.
  const int nff2 = d.nff * d.nff;
  const double base = 1.0 / (4.0 * T * T * (double)lk * (double)lk);
  for (int w = threadIdx.x; w < 2 * nff2; w += blockDim.x) {
    const int ch = w / nff2, mn = w % nff2;
    const double* e = d.ebub + (size_t)mn * d.nsh;
    const double* g = gh + ch * d.nsh;
    double v = 0.0;
    for (int j = 0; j < d.nsh; ++j) v = fma(e[j], g[j], v);
    v *= (ch == 0 ? -base : base);
    if (nsplit == 1)
      dchi[(size_t)ch * S + (size_t)q * nff2 + mn] = v;
    else
      dpart[(((size_t)split * 2 + ch) * d.nq + q) * nff2 + mn] = v;
  }
}

// chi' = sum over the split slices in split order (loops with nsplit > 1)
__global__ void __launch_bounds__(256)
k_chi_sum(const double* __restrict__ dpart, int nsplit, int nq, int nff2, double* __restrict__ dchi,
          int64_t S) {
  const int64_t n = (int64_t)2 * nq * nff2;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int s = 0; s < nsplit; ++s) v += dpart[(size_t)s * n + i];
    const int64_t ch = i / ((int64_t)nq * nff2), r = i % ((int64_t)nq * nff2);
    dchi[ch * S + r] = v;
  }
}

// ------------------------------------------------------- projections
// Forward transform of the projections: the partial Fourier sums over the
// transfer grid at the half-integer frequencies S/2,
//   xt[ch][k][mn] = (1/Nq) sum_u E[u][k] X[ch][u][mn],  E = (cos(u.S'/2) | sin(u.S'/2)).
// A block owns 64 consecutive columns (ch, mn) and KG harmonic columns; its NW
// waves split the transfer grid and are reduced in LDS in a fixed order.
template <int KG, int NW>
__global__ void __launch_bounds__(64 * NW)
k_dft_fwd(const double* __restrict__ eph, int nq, int ncol, const double* __restrict__ X,
          int64_t S, int nff2, double* __restrict__ xt) {
  __shared__ double red[NW][KG][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int col = blockIdx.x * 64 + lane;
  const int k0 = blockIdx.y * KG;
  const int kn = min(KG, ncol - k0);
  const bool ok = col < 3 * nff2;
  const int ch = ok ? col / nff2 : 0, mn = ok ? col % nff2 : 0;
  const double* xp = X + (size_t)ch * S + mn;
  const int u0 = (int)((int64_t)nq * w / NW), u1 = (int)((int64_t)nq * (w + 1) / NW);
  double acc[KG];
#pragma unroll
  for (int i = 0; i < KG; ++i) acc[i] = 0.0;
#pragma unroll 4
  for (int u = u0; u < u1; ++u) {
    const double x = ok ? xp[(size_t)u * nff2] : 0.0;
    const double* e = eph + (size_t)u * ncol + k0;
#pragma unroll
    for (int i = 0; i < KG; ++i)
      if (i < kn) acc[i] = fma(e[i], x, acc[i]);
  }
#pragma unroll
  for (int i = 0; i < KG; ++i) red[w][i][lane] = acc[i];
  __syncthreads();
  if (w == 0 && ok) {
    const double inv = 1.0 / (double)nq;
    for (int i = 0; i < kn; ++i) {
      double v = 0.0;
      for (int ww = 0; ww < NW; ++ww) v += red[ww][i][lane];
      xt[((size_t)ch * ncol + k0 + i) * nff2 + mn] = v * inv;
    }
  }
}

// Bond basis of the transformed propagators, for every harmonic of the full
// list v (+S'_j for v < nsh, -S'_{v-nsh+1} otherwise):
//   yb[in][v][b1 b2] = sum_{m' in shell(b1), n' in shell(b2)} c_{m'b1} c_{n'b2} xt^{in}_{m'n'}(v)
// with xt(-S') = conj(xt(S')).  These are the bond-space Fourier coefficients
// Yhat_{R1R2}(W) of the propagators at frequency 2W - R1 - R2 = v.
__global__ void __launch_bounds__(256)
k_bond_basis(DevTables d, const double* __restrict__ xt, double* __restrict__ yb) {
  const int nff = d.nff, nff2 = nff * nff, nsh = d.nsh, ncol = d.ncol, nv = 2 * nsh - 1;
  const int total = 3 * nv * nff2;
  __shared__ double cs[2 * 441];
  for (int i = threadIdx.x; i < nff2; i += blockDim.x) {
    cs[i] = d.cre[i];
    cs[nff2 + i] = d.cim[i];
  }
  __syncthreads();
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int in = idx / (nv * nff2), v = (idx / nff2) % nv, b = idx % nff2;
  const int b1 = b / nff, b2 = b % nff;
  const int j = v < nsh ? v : v - nsh + 1;
  const double sim = v < nsh ? 1.0 : -1.0;
  const double* xr = xt + ((size_t)in * ncol + j) * nff2;
  const double* xi = xt + ((size_t)in * ncol + (nsh - 1 + j)) * nff2;
  const int s1 = d.shell_of[b1], s2 = d.shell_of[b2];
  double yr = 0.0, yi = 0.0;
  const int m0 = d.shell_start[s1], m1 = d.shell_start[s1 + 1];
  const int n0 = d.shell_start[s2], n1 = d.shell_start[s2 + 1];
  for (int mp = m0; mp < m1; ++mp) {
    const double c1r = cs[mp * nff + b1], c1i = cs[nff2 + mp * nff + b1];
#pragma unroll 4
    for (int np = n0; np < n1; ++np) {
      const double c2r = cs[np * nff + b2], c2i = cs[nff2 + np * nff + b2];
      const double wr = c1r * c2r - c1i * c2i, wi = c1r * c2i + c1i * c2r;
      const double ar = xr[mp * nff + np];
      const double ai = j > 0 ? sim * xi[mp * nff + np] : 0.0;
      yr = fma(wr, ar, fma(-wi, ai, yr));
      yi = fma(wr, ai, fma(wi, ar, yi));
    }
  }
  yb[idx] = yr;
  yb[(size_t)total + idx] = yi;
}

// Gather and basis change, independent of the transfer momentum.  One block
// per (output channel X, half-set harmonic j).  For V = +S'_j and V = -S'_j:
//   M^X_AB(V) = sum_entries (+-) yb^{in}_{b1 b2}(v)          (eqn. proj_pos in bonds)
//   N^X(V) = C M^X(V) C^T                                  (back to form factors)
// and the real coefficients of cos(l.V/2), sin(l.V/2) for the inverse transform:
//   Re[e^{-il.V/2} N(V) + e^{+il.V/2} N(-V)] = cos (ReN+ + ReN-) + sin (ImN+ - ImN-).
__global__ void __launch_bounds__(256)
k_gather_g2(DevTables d, const double* __restrict__ yb, double* __restrict__ g2) {
  const int X = blockIdx.y, j = blockIdx.x;
  const int nff = d.nff, nff2 = nff * nff, nsh = d.nsh, ncol = d.ncol;
  const int nv = 2 * nsh - 1;
  const int nvl = (j == 0) ? 1 : 2;
  const size_t ybim = (size_t)3 * nv * nff2;
  extern __shared__ double sm[];
  double* Mre = sm;                  // [2][nff2]
  double* Mim = Mre + 2 * nff2;
  for (int w = threadIdx.x; w < nvl * nff2; w += blockDim.x) {
    const int vi = w / nff2, ab = w % nff2;
    const int vf = (vi == 0) ? j : (nsh - 1 + j);
    const size_t row = ((size_t)X * nv + vf) * nff2 + ab;
    double re = 0.0, im = 0.0;
    for (int e = d.mrow[row]; e < d.mrow[row + 1]; ++e) {
      const int32_t pk = d.ment[e];
      const int in = pk & 3, b1 = (pk >> 2) & 31, b2 = (pk >> 7) & 31, v = (pk >> 12) & 127;
      const int neg = (pk >> 19) & 1;
      const size_t o = ((size_t)in * nv + v) * nff2 + b1 * nff + b2;
      const double yr = yb[o], yi = yb[ybim + o];
      if (neg) { re -= yr; im -= yi; } else { re += yr; im += yi; }
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
      const double c1r = d.cre[m * nff + a], c1i = d.cim[m * nff + a];
      for (int b = d.shell_start[sn]; b < d.shell_start[sn + 1]; ++b) {
        const double c2r = d.cre[n * nff + b], c2i = d.cim[n * nff + b];
        const double wr = c1r * c2r - c1i * c2i, wi = c1r * c2i + c1i * c2r;
        for (int vi = 0; vi < nvl; ++vi) {
          const double mr = Mre[vi * nff2 + a * nff + b], mi = Mim[vi * nff2 + a * nff + b];
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

// Inverse transform fused with the assembly of eqns. proj_VP/VC/VD and, in
// mode 1, with the products of eqns. matmul-P/C/D.  One block per lt momenta l.
//   K^X_mn(l) = sum_k E[l][k] g2[X][k][mn]
//   V^P = U e0e0 - P + K^P,  V^C = U e0e0 + C + K^C,  V^D = U e0e0 + D + K^D
//   dP = V^P chi'pp V^P, dC = -V^C chi'ph V^C,
//   dD = (W chi'ph W - V^C chi'ph V^C)/2 with W = 2 V^D - V^C (the SU(2) form
//   of eqn. matmul-D: 2 dD - dC = W chi'ph W).
constexpr int kLT = 4;   // largest number of momenta per block
__global__ void __launch_bounds__(256)
k_proj_back(DevTables d, const double* __restrict__ X, int64_t S, const double* __restrict__ g2,
            const double* __restrict__ dchi, const double* __restrict__ dpart, int nsplit,
            double* __restrict__ out, int mode, int cross, double scale, int lt) {
  const int nff = d.nff, nff2 = nff * nff, ncol = d.ncol, nq = d.nq;
  const int l0 = blockIdx.x * lt;
  const int nl = min(lt, nq - l0);
  extern __shared__ double sm[];
  double* Et = sm;                         // [lt][ncol]
  double* Vs = Et + lt * ncol;             // [lt][3][nff2]
  double* T1 = Vs + lt * 3 * nff2;         // [3][nff2]
  double* T2 = T1 + 3 * nff2;              // [3][nff2]
  double* Ch = T2 + 3 * nff2;              // [2][nff2]
  double* Wm = Ch + 2 * nff2;              // [nff2]
  for (int i = threadIdx.x; i < nl * ncol; i += blockDim.x)
    Et[i] = d.eph[(size_t)(l0 + i / ncol) * ncol + i % ncol];
  __syncthreads();
  for (int w = threadIdx.x; w < 3 * nff2; w += blockDim.x) {
    const int ch = w / nff2, mn = w % nff2;
    double acc[kLT];
#pragma unroll
    for (int i = 0; i < kLT; ++i) acc[i] = 0.0;
    if (cross) {
      const double* g = g2 + (size_t)ch * ncol * nff2 + mn;
#pragma unroll 8
      for (int k = 0; k < ncol; ++k) {
        const double gv = g[(size_t)k * nff2];
#pragma unroll
        for (int i = 0; i < kLT; ++i)
          if (i < nl) acc[i] = fma(Et[i * ncol + k], gv, acc[i]);
      }
    }
    const double bare = (mn == 0) ? d.U : 0.0;
    const double sgn = (ch == 0) ? -1.0 : 1.0;
    for (int i = 0; i < nl; ++i) {
      const double own = X[(size_t)ch * S + (size_t)(l0 + i) * nff2 + mn];
      Vs[(i * 3 + ch) * nff2 + mn] = bare + sgn * own + acc[i];
    }
  }
  __syncthreads();
  if (mode == 0) {
    for (int w = threadIdx.x; w < nl * 3 * nff2; w += blockDim.x) {
      const int i = w / (3 * nff2), r = w % (3 * nff2), ch = r / nff2, mn = r % nff2;
      out[(size_t)ch * S + (size_t)(l0 + i) * nff2 + mn] = Vs[w];
    }
    return;
  }
  for (int i = 0; i < nl; ++i) {
    const int l = l0 + i;
    const double* VP = Vs + (i * 3 + 0) * nff2;
    const double* VC = Vs + (i * 3 + 1) * nff2;
    const double* VD = Vs + (i * 3 + 2) * nff2;
    for (int w = threadIdx.x; w < 2 * nff2; w += blockDim.x) {
      const int ch = w / nff2, mn = w % nff2;
      if (nsplit == 1) {
        Ch[w] = dchi[(size_t)ch * S + (size_t)l * nff2 + mn];
      } else {
        double v = 0.0;
        for (int s = 0; s < nsplit; ++s) v += dpart[(((size_t)s * 2 + ch) * nq + l) * nff2 + mn];
        Ch[w] = v;
      }
    }
    for (int w = threadIdx.x; w < nff2; w += blockDim.x) Wm[w] = 2.0 * VD[w] - VC[w];
    __syncthreads();
    // T1 = chi'pp V^P, chi'ph V^C, chi'ph W
    for (int w = threadIdx.x; w < 3 * nff2; w += blockDim.x) {
      const int which = w / nff2, m = (w % nff2) / nff, n = w % nff;
      const double* A = Ch + (which == 0 ? 0 : nff2) + m * nff;
      const double* B = which == 0 ? VP : (which == 1 ? VC : Wm);
      double v = 0.0;
      for (int k = 0; k < nff; ++k) v = fma(A[k], B[k * nff + n], v);
      T1[w] = v;
    }
    __syncthreads();
    // T2 = V^P T1p, V^C T1c, W T1w
    for (int w = threadIdx.x; w < 3 * nff2; w += blockDim.x) {
      const int which = w / nff2, m = (w % nff2) / nff, n = w % nff;
      const double* A = (which == 0 ? VP : (which == 1 ? VC : Wm)) + m * nff;
      const double* B = T1 + which * nff2;
      double v = 0.0;
      for (int k = 0; k < nff; ++k) v = fma(A[k], B[k * nff + n], v);
      T2[w] = v;
    }
    __syncthreads();
    for (int w = threadIdx.x; w < nff2; w += blockDim.x) {
      const size_t o = (size_t)l * nff2 + w;
      out[o] = scale * T2[w];
      out[(size_t)S + o] = -scale * T2[nff2 + w];
      out[2 * (size_t)S + o] = 0.5 * scale * (T2[2 * nff2 + w] - T2[nff2 + w]);
    }
    __syncthreads();
  }
}

// ======================================================= mixed precision
// Loops in FP32: energies and alpha +- beta in FP64, the pair math in FP32,
// row sums blocked over 8 rows in FP32 and added into Neumaier-compensated
// FP32 running sums; the short reductions over columns and slices in FP64.
struct Exp2F { __device__ float operator()(float x) const { return __builtin_amdgcn_exp2f(x); } };
struct RcpF { __device__ float operator()(float x) const { return __builtin_amdgcn_rcpf(x); } };

__device__ __forceinline__ void neumaier_add(float& s, float& c, float v) {
  const float t = s + v;
  const bool sbig = fabsf(s) >= fabsf(v);
  const float big = sbig ? s : v, small = sbig ? v : s;
  c += (big - t) + small;
  s = t;
}

template <int SMAX>
__global__ void __launch_bounds__(kBubThreads)
k_loops_mixed(DevTables d, double T, int nsplit, int nchunk, double* __restrict__ dchi, int64_t S,
              double* __restrict__ dpart) {
  constexpr int NH = 2 * SMAX + 1;
  constexpr int RB = 8;
  const int q = blockIdx.x / nsplit, split = blockIdx.x % nsplit;
  const int lk = d.lk;
  const int rows = lk / 2 + 1;
  const int R0 = (int)((int64_t)rows * split / nsplit);
  const int R1 = (int)((int64_t)rows * (split + 1) / nsplit);
  const int nr = R1 - R0;
  const int lq = d.lq;
  const int ix = q / lq, iy = q % lq;
  const double inv2T = 0.5 / T;

  extern __shared__ double smem[];
  double* y1 = smem;
  double* y2 = y1 + nr;
  float* pyt = reinterpret_cast<float*>(y2 + nr);      // [nr][NH] (FP32 weights)
  double* rs = reinterpret_cast<double*>(pyt + ((nr * NH + 1) & ~1));
  double* gh = rs + lk * 2 * NH;

  for (int j = threadIdx.x; j < nr; j += blockDim.x) {
    const double* c = d.cshift + ((size_t)iy * lk + (R0 + j)) * 2;
    y1[j] = c[0];
    y2[j] = c[1];
  }
  for (int j = threadIdx.x; j < nr * NH; j += blockDim.x) pyt[j] = (float)d.pytab[R0 * NH + j];
  for (int j = threadIdx.x; j < lk * 2 * NH; j += blockDim.x) rs[j] = 0.0;
  __syncthreads();

  const int t = threadIdx.x;
  const bool active = t < lk * nchunk;
  const int px = t % lk, c = t / lk;
  float sum[2][NH], cmp[2][NH];
#pragma unroll
  for (int n = 0; n < NH; ++n) sum[0][n] = sum[1][n] = cmp[0][n] = cmp[1][n] = 0.0f;
  if (active) {
    const double cx1 = d.cshift[((size_t)ix * lk + px) * 2];
    const double cx2 = d.cshift[((size_t)ix * lk + px) * 2 + 1];
    const double A1 = (-2.0 * d.t * cx1 - d.mu) * inv2T;
    const double B1 = (-2.0 * d.t - 4.0 * d.tp * cx1) * inv2T;
    const double A2 = (-2.0 * d.t * cx2 - d.mu) * inv2T;
    const double B2 = (-2.0 * d.t - 4.0 * d.tp * cx2) * inv2T;
    const int r0 = (int)((int64_t)nr * c / nchunk);
    const int r1 = (int)((int64_t)nr * (c + 1) / nchunk);
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
        const float* w = pyt + r * NH;
#pragma unroll
        for (int n = 0; n < NH; ++n) {
          blk[0][n] = fmaf(dpp, w[n], blk[0][n]);
          blk[1][n] = fmaf(dph, w[n], blk[1][n]);
        }
      }
#pragma unroll
      for (int n = 0; n < NH; ++n) {
        neumaier_add(sum[0][n], cmp[0][n], blk[0][n]);
        neumaier_add(sum[1][n], cmp[1][n], blk[1][n]);
      }
    }
  }
  for (int cc = 0; cc < nchunk; ++cc) {
    if (active && c == cc) {
      double* dst = rs + px * 2 * NH;
#pragma unroll
      for (int n = 0; n < NH; ++n) {
        dst[n] += (double)sum[0][n] + (double)cmp[0][n];
        dst[NH + n] += (double)sum[1][n] + (double)cmp[1][n];
      }
    }
    __syncthreads();
  }
  const int nout = 2 * d.nsh;
  int nseg = (int)blockDim.x / nout;
  if (nseg < 1) nseg = 1;
  for (int w = threadIdx.x; w < nout * nseg; w += blockDim.x) {
    const int o = w % nout, seg = w / nout;
    const int ch = o / d.nsh, j = o % d.nsh;
    const int sx = d.hx[j], sy = d.hy[j];
    const int ay = sy < 0 ? -sy : sy;
    const double sg = sy < 0 ? -1.0 : 1.0;
    double g = 0.0;
    for (int x = seg; x < lk; x += nseg) {
      const double* r = rs + x * 2 * NH + ch * NH;
      double v = d.pxtab[x * NH + sx] * r[ay];
      if (sx > 0 && ay > 0) v = fma(-sg * d.pxtab[x * NH + SMAX + sx], r[SMAX + ay], v);
      g += v;
    }
    gh[seg * nout + o] = g;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < nout; o += blockDim.x) {
    double g = 0.0;
    for (int s2 = 0; s2 < nseg; ++s2) g += gh[s2 * nout + o];
    gh[o] = g;
  }
  __syncthreads();
  const int nff2 = d.nff * d.nff;
  const double base = 1.0 / (4.0 * T * T * (double)lk * (double)lk);
  for (int w = threadIdx.x; w < 2 * nff2; w += blockDim.x) {
    const int ch = w / nff2, mn = w % nff2;
    const double* e = d.ebub + (size_t)mn * d.nsh;
    const double* g = gh + ch * d.nsh;
    double v = 0.0;
    for (int j = 0; j < d.nsh; ++j) v = fma(e[j], g[j], v);
    v *= (ch == 0 ? -base : base);
    if (nsplit == 1)
      dchi[(size_t)ch * S + (size_t)q * nff2 + mn] = v;
    else
      dpart[(((size_t)split * 2 + ch) * d.nq + q) * nff2 + mn] = v;
  }
}

// BF16 hi/lo split with round to nearest even: x ~ hi + lo (about 16 mantissa
// bits); products hi*hi + hi*lo + lo*hi accumulate in FP32 on the matrix cores.
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

// Forward transform on the matrix cores:
//   xt[ch][k][mn] = (1/Nq) sum_u E[u][k] X[ch][u][mn]
// as C[M=ncol][N=3 nff^2] = A^T B with A = E (pre-split, [Nq][ncol]) and
// B = X (split on the fly).  One 16x16 output tile per block; its 4 waves
// split the transfer grid and are added in LDS in a fixed order.
// v_mfma_f32_16x16x16bf16_1k operand layout: lane l holds A[l%16][4(l/16)+j],
// B[4(l/16)+j][l%16] (j = 0..3) and D[4(l/16)+j][l%16].
__global__ void __launch_bounds__(256)
k_dft_fwd_mfma(const unsigned short* __restrict__ eh, const unsigned short* __restrict__ el,
               int nq, int ncol, const double* __restrict__ X, int64_t S, int nff2,
               double* __restrict__ xt) {
  __shared__ float red[4][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.x * 16, n0 = blockIdx.y * 16;
  const int ml = m0 + (lane & 15), nl = n0 + (lane & 15), kq = 4 * (lane >> 4);
  const bool mok = ml < ncol, nok = nl < 3 * nff2;
  const int ch = nok ? nl / nff2 : 0, mn = nok ? nl % nff2 : 0;
  const double* xp = X + (size_t)ch * S + mn;
  const int nsteps = (nq + 15) / 16;
  const int s0 = nsteps * w / 4, s1 = nsteps * (w + 1) / 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int st = s0; st < s1; ++st) {
    bf16x4 ah, al, bh, bl;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int u = st * 16 + kq + j;
      const bool ok = u < nq;
      ah[j] = (short)((ok && mok) ? eh[(size_t)u * ncol + ml] : 0);
      al[j] = (short)((ok && mok) ? el[(size_t)u * ncol + ml] : 0);
      unsigned short h = 0, l = 0;
      if (ok && nok) split_bf16(xp[(size_t)u * nff2], h, l);
      bh[j] = (short)h;
      bl[j] = (short)l;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) red[w][lane * 4 + j] = acc[j];
  __syncthreads();
  if (w == 0) {
    const double inv = 1.0 / (double)nq;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double v = ((double)red[0][lane * 4 + j] + (double)red[1][lane * 4 + j]) +
                       ((double)red[2][lane * 4 + j] + (double)red[3][lane * 4 + j]);
      const int m = m0 + kq + j, n = n0 + (lane & 15);
      if (m < ncol && n < 3 * nff2) {
        const int c2 = n / nff2, mn2 = n % nff2;
        xt[((size_t)c2 * ncol + m) * nff2 + mn2] = v * inv;
      }
    }
  }
}

// Inverse transform on the matrix cores:
//   K[ch][l][mn] = sum_k E[l][k] g2[ch][k][mn]
// as C[M=Nq][N=3 nff^2] = A B with A = E (pre-split, [Nq][ncol]) and B = g2
// (split on the fly).  Each wave owns one 16x16 output tile.
__global__ void __launch_bounds__(256)
k_dft_inv_mfma(const unsigned short* __restrict__ eh, const unsigned short* __restrict__ el,
               int nq, int ncol, const double* __restrict__ g2, int nff2, float* __restrict__ K) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.x * 16, n0 = (blockIdx.y * 4 + w) * 16;
  const int ml = m0 + (lane & 15), nl = n0 + (lane & 15), kq = 4 * (lane >> 4);
  const bool mok = ml < nq, nok = nl < 3 * nff2;
  const int ch = nok ? nl / nff2 : 0, mn = nok ? nl % nff2 : 0;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < ncol; k0 += 16) {
    bf16x4 ah, al, bh, bl;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + kq + j;
      const bool ok = k < ncol;
      ah[j] = (short)((ok && mok) ? eh[(size_t)ml * ncol + k] : 0);
      al[j] = (short)((ok && mok) ? el[(size_t)ml * ncol + k] : 0);
      unsigned short h = 0, l = 0;
      if (ok && nok) split_bf16(g2[((size_t)ch * ncol + k) * nff2 + mn], h, l);
      bh[j] = (short)h;
      bl[j] = (short)l;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int m = m0 + kq + j, n = n0 + (lane & 15);
    if (m < nq && n < 3 * nff2) {
      const int c2 = n / nff2, mn2 = n % nff2;
      K[((size_t)c2 * nq + m) * nff2 + mn2] = acc[j];
    }
  }
}

// Assembly of V and the products in FP32; one block per momentum.  Inputs:
// K (inverse transform, FP32, may be null without cross terms), X and the
// loops (FP64); output scale * dX/dT in FP64.
__global__ void __launch_bounds__(256)
k_products_f32(DevTables d, const double* __restrict__ X, int64_t S, const float* __restrict__ K,
               const double* __restrict__ dchi, const double* __restrict__ dpart, int nsplit,
               double* __restrict__ out, int mode, double scale) {
  const int nff = d.nff, nff2 = nff * nff, nq = d.nq;
  const int l = blockIdx.x;
  extern __shared__ float fsm[];
  float* Vs = fsm;              // [3][nff2]
  float* Ch = Vs + 3 * nff2;    // [2][nff2]
  float* Wm = Ch + 2 * nff2;    // [nff2]
  float* T1 = Wm + nff2;        // [3][nff2]
  float* T2 = T1 + 3 * nff2;    // [3][nff2]
  for (int w = threadIdx.x; w < 3 * nff2; w += blockDim.x) {
    const int ch = w / nff2, mn = w % nff2;
    const float bare = (mn == 0) ? (float)d.U : 0.0f;
    const float own = (float)X[(size_t)ch * S + (size_t)l * nff2 + mn];
    const float kk = K ? K[((size_t)ch * nq + l) * nff2 + mn] : 0.0f;
    Vs[w] = bare + (ch == 0 ? -own : own) + kk;
  }
  if (mode == 0) {
    __syncthreads();
    for (int w = threadIdx.x; w < 3 * nff2; w += blockDim.x)
      out[(size_t)(w / nff2) * S + (size_t)l * nff2 + w % nff2] = (double)Vs[w];
    return;
  }
  for (int w = threadIdx.x; w < 2 * nff2; w += blockDim.x) {
    const int ch = w / nff2, mn = w % nff2;
    double v;
    if (nsplit == 1) {
      v = dchi[(size_t)ch * S + (size_t)l * nff2 + mn];
    } else {
      v = 0.0;
      for (int s2 = 0; s2 < nsplit; ++s2) v += dpart[(((size_t)s2 * 2 + ch) * nq + l) * nff2 + mn];
    }
    Ch[w] = (float)v;
  }
  __syncthreads();
  const float* VP = Vs;
  const float* VC = Vs + nff2;
  const float* VD = Vs + 2 * nff2;
  for (int w = threadIdx.x; w < nff2; w += blockDim.x) Wm[w] = 2.0f * VD[w] - VC[w];
  __syncthreads();
  for (int w = threadIdx.x; w < 3 * nff2; w += blockDim.x) {
    const int which = w / nff2, m = (w % nff2) / nff, n = w % nff;
    const float* A = Ch + (which == 0 ? 0 : nff2) + m * nff;
    const float* B = which == 0 ? VP : (which == 1 ? VC : Wm);
    float v = 0.0f;
    for (int k = 0; k < nff; ++k) v = fmaf(A[k], B[k * nff + n], v);
    T1[w] = v;
  }
  __syncthreads();
  for (int w = threadIdx.x; w < 3 * nff2; w += blockDim.x) {
    const int which = w / nff2, m = (w % nff2) / nff, n = w % nff;
    const float* A = (which == 0 ? VP : (which == 1 ? VC : Wm)) + m * nff;
    const float* B = T1 + which * nff2;
    float v = 0.0f;
    for (int k = 0; k < nff; ++k) v = fmaf(A[k], B[k * nff + n], v);
    T2[w] = v;
  }
  __syncthreads();
  for (int w = threadIdx.x; w < nff2; w += blockDim.x) {
    const size_t o = (size_t)l * nff2 + w;
    out[o] = scale * (double)T2[w];
    out[(size_t)S + o] = -scale * (double)T2[nff2 + w];
    out[2 * (size_t)S + o] = 0.5 * scale * ((double)T2[2 * nff2 + w] - (double)T2[nff2 + w]);
  }
}

// ----------------------------------------------------------- ODE helpers
struct SlopeSet {
  const double* k[7];
  double coef[7];
};

__global__ void k_axpy_stage(const double* __restrict__ X, SlopeSet ks, int nk, double h,
                             double* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int j = 0; j < nk; ++j) acc = fma(ks.coef[j], ks.k[j][i], acc);
    out[i] = fma(h, acc, X[i]);
  }
}

// max |x| as the ordered bit pattern of a non-negative double (NaN sorts
// above +inf, so a non-finite state is seen)
__global__ void k_maxabs(const double* __restrict__ X, int64_t n, unsigned long long* word) {
  __shared__ unsigned long long red[256];
  unsigned long long m = 0ull;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    unsigned long long b = (unsigned long long)__double_as_longlong(fabs(X[i]));
    if (X[i] != X[i]) b = 0x7ff8000000000000ull;
    m = b > m ? b : m;
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && red[threadIdx.x + s] > red[threadIdx.x])
      red[threadIdx.x] = red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(word, red[0]);
}

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Partial sums of ((h sum_j e_j k_j) / (atol + rtol max(|y0|,|y5|)))^2 per
// block, in a fixed tree order (deterministic).
__global__ void k_errnorm(const double* __restrict__ y0, const double* __restrict__ y5,
                          SlopeSet ks, int nk, double h, double rtol, double atol, int64_t n,
                          double* red_out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double e = 0.0;
    for (int j = 0; j < nk; ++j) e = fma(ks.coef[j], ks.k[j][i], e);
    e *= h;
    const double sc = atol + rtol * fmax(fabs(y0[i]), fabs(y5[i]));
    const double r = e / sc;
    acc = fma(r, r, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) red_out[blockIdx.x] = red[0];
}

}  // namespace

// ------------------------------------------------------------- launchers
LoopGeom loop_geometry(const DevTables& d) {
  // Split the half fine grid of every transfer momentum into nsplit row blocks
  // of lk * nchunk threads until about 8 waves per SIMD are in flight, keeping
  // at least 4 rows per thread and at most kBubThreads threads per block.
  const int rows = d.lk / 2 + 1;
  const int64_t target = (int64_t)256 * 4 * 8 * 64;   // lanes for ~8 waves per SIMD
  int nsplit = 1, nchunk = 1;
  for (;;) {
    const int64_t lanes = (int64_t)d.nq * d.lk * nsplit * nchunk;
    if (lanes >= target) break;
    if (d.lk * (nchunk + 1) <= kBubThreads && rows / (nsplit * (nchunk + 1)) >= 4) {
      ++nchunk;
    } else if (nsplit < 16 && rows / ((nsplit + 1) * nchunk) >= 4) {
      ++nsplit;
    } else {
      break;
    }
  }
  LoopGeom g;
  g.nsplit = nsplit;
  g.nchunk = nchunk;
  g.threads = ((d.lk * nchunk + 63) / 64) * 64;
  const int nrmax = (rows + nsplit - 1) / nsplit;
  const int NH = 2 * d.smax + 1, nout = 2 * d.nsh;
  int nseg = g.threads / nout;
  if (nseg < 1) nseg = 1;
  g.smem = sizeof(double) * ((size_t)2 * nrmax + (size_t)nrmax * NH + (size_t)d.lk * 2 * NH +
                             (size_t)nseg * nout);
  return g;
}

void launch_loops(const DevTables& d, double T, double* dchi, int64_t S, double* dpart,
                  bool sum_slices, hipStream_t s) {
  const LoopGeom g = loop_geometry(d);
  const dim3 grid((unsigned)(d.nq * g.nsplit));
  switch (d.smax) {
    case 0:
      hipLaunchKernelGGL(k_loops_f64<0>, grid, dim3(g.threads), g.smem, s, d, T, g.nsplit, g.nchunk,
                         dchi, S, dpart);
      break;
    case 2:
      hipLaunchKernelGGL(k_loops_f64<2>, grid, dim3(g.threads), g.smem, s, d, T, g.nsplit, g.nchunk,
                         dchi, S, dpart);
      break;
    default:
      hipLaunchKernelGGL(k_loops_f64<4>, grid, dim3(g.threads), g.smem, s, d, T, g.nsplit, g.nchunk,
                         dchi, S, dpart);
      break;
  }
  if (sum_slices && g.nsplit > 1) {
    const int nff2 = d.nff * d.nff;
    const int64_t n = (int64_t)2 * d.nq * nff2;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_chi_sum, dim3(blocks), dim3(256), 0, s, dpart, g.nsplit, d.nq, nff2, dchi, S);
  }
}

void launch_project_front(const DevTables& d, const double* X, int64_t S, double* xt, double* yb,
                          double* g2, uint32_t flags, hipStream_t s) {
  if (flags & TUFRG_NO_CROSS) return;
  const int nff2 = d.nff * d.nff;
  const int ncols = 3 * nff2;
  if (d.nq * ncols >= 2000000) {
    dim3 g1((ncols + 63) / 64, (d.ncol + 7) / 8);
    hipLaunchKernelGGL((k_dft_fwd<8, 8>), g1, dim3(512), 0, s, d.eph, d.nq, d.ncol, X, S, nff2, xt);
  } else {
    dim3 g1((ncols + 63) / 64, (d.ncol + 3) / 4);
    hipLaunchKernelGGL((k_dft_fwd<4, 16>), g1, dim3(1024), 0, s, d.eph, d.nq, d.ncol, X, S, nff2, xt);
  }
  const int nv = 2 * d.nsh - 1;
  const int total = 3 * nv * nff2;
  hipLaunchKernelGGL(k_bond_basis, dim3((total + 255) / 256), dim3(256), 0, s, d, xt, yb);
  const size_t sm_mid = sizeof(double) * 4 * (size_t)nff2;
  hipLaunchKernelGGL(k_gather_g2, dim3(d.nsh, 3), dim3(256), sm_mid, s, d, yb, g2);
}

void launch_project_back(const DevTables& d, const double* X, int64_t S, const double* g2,
                         const double* dchi, const double* dpart, double* out, int mode,
                         uint32_t flags, double scale, hipStream_t s) {
  const int nff2 = d.nff * d.nff;
  const int nsplit = loop_geometry(d).nsplit;
  const int cross = (flags & TUFRG_NO_CROSS) ? 0 : 1;
  auto sm_bytes = [&](int l) {
    return sizeof(double) * ((size_t)l * d.ncol + (size_t)l * 3 * nff2 + 9 * (size_t)nff2);
  };
  // momenta per block: two on large grids (halves the reads of g2), one
  // otherwise; always within 64 KB of LDS
  int lt = d.nq >= 1024 ? 2 : 1;
  while (lt > 1 && sm_bytes(lt) > 65536) --lt;
  hipLaunchKernelGGL(k_proj_back, dim3((d.nq + lt - 1) / lt), dim3(256), sm_bytes(lt), s, d, X, S,
                     g2, dchi, dpart, nsplit, out, mode, cross, scale, lt);
}

size_t loop_smem_mixed(const DevTables& d, const LoopGeom& g) {
  const int rows = d.lk / 2 + 1, nrmax = (rows + g.nsplit - 1) / g.nsplit;
  const int NH = 2 * d.smax + 1, nout = 2 * d.nsh;
  int nseg = g.threads / nout;
  if (nseg < 1) nseg = 1;
  return sizeof(double) * ((size_t)2 * nrmax + (size_t)d.lk * 2 * NH + (size_t)nseg * nout) +
         sizeof(float) * (((size_t)nrmax * NH + 1) & ~(size_t)1);
}

void launch_loops_mixed(const DevTables& d, double T, double* dchi, int64_t S, double* dpart,
                        bool sum_slices, hipStream_t s) {
  const LoopGeom g = loop_geometry(d);
  const size_t sm = loop_smem_mixed(d, g);
  const dim3 grid((unsigned)(d.nq * g.nsplit));
  switch (d.smax) {
    case 0:
      hipLaunchKernelGGL(k_loops_mixed<0>, grid, dim3(g.threads), sm, s, d, T, g.nsplit, g.nchunk,
                         dchi, S, dpart);
      break;
    case 2:
      hipLaunchKernelGGL(k_loops_mixed<2>, grid, dim3(g.threads), sm, s, d, T, g.nsplit, g.nchunk,
                         dchi, S, dpart);
      break;
    default:
      hipLaunchKernelGGL(k_loops_mixed<4>, grid, dim3(g.threads), sm, s, d, T, g.nsplit, g.nchunk,
                         dchi, S, dpart);
      break;
  }
  if (sum_slices && g.nsplit > 1) {
    const int nff2 = d.nff * d.nff;
    const int64_t n = (int64_t)2 * d.nq * nff2;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_chi_sum, dim3(blocks), dim3(256), 0, s, dpart, g.nsplit, d.nq, nff2, dchi, S);
  }
}

void launch_project_front_mixed(const DevTables& d, const double* X, int64_t S, double* xt,
                                double* yb, double* g2, uint32_t flags, hipStream_t s) {
  if (flags & TUFRG_NO_CROSS) return;
  const int nff2 = d.nff * d.nff;
  dim3 g1((d.ncol + 15) / 16, (3 * nff2 + 15) / 16);
  hipLaunchKernelGGL(k_dft_fwd_mfma, g1, dim3(256), 0, s, d.eph_hi, d.eph_lo, d.nq, d.ncol, X, S,
                     nff2, xt);
  const int nv = 2 * d.nsh - 1;
  const int total = 3 * nv * nff2;
  hipLaunchKernelGGL(k_bond_basis, dim3((total + 255) / 256), dim3(256), 0, s, d, xt, yb);
  const size_t sm_mid = sizeof(double) * 4 * (size_t)nff2;
  hipLaunchKernelGGL(k_gather_g2, dim3(d.nsh, 3), dim3(256), sm_mid, s, d, yb, g2);
}

void launch_inverse_mixed(const DevTables& d, const double* g2, float* K, uint32_t flags,
                          hipStream_t s) {
  if (flags & TUFRG_NO_CROSS) return;
  const int nff2 = d.nff * d.nff;
  dim3 g((d.nq + 15) / 16, (3 * nff2 + 63) / 64);
  hipLaunchKernelGGL(k_dft_inv_mfma, g, dim3(256), 0, s, d.eph_hi, d.eph_lo, d.nq, d.ncol, g2, nff2,
                     K);
}

void launch_products_mixed(const DevTables& d, const double* X, int64_t S, const float* K,
                           const double* dchi, const double* dpart, double* out, int mode,
                           uint32_t flags, double scale, hipStream_t s) {
  const int nff2 = d.nff * d.nff;
  const int nsplit = loop_geometry(d).nsplit;
  const float* Kp = (flags & TUFRG_NO_CROSS) ? nullptr : K;
  hipLaunchKernelGGL(k_products_f32, dim3(d.nq), dim3(256), sizeof(float) * 12 * (size_t)nff2, s, d,
                     X, S, Kp, dchi, dpart, nsplit, out, mode, scale);
}

void launch_axpy_stage(const double* X, const double* const* k, const double* coef, int nk,
                       double h, double* out, int64_t n, hipStream_t s) {
  SlopeSet ks{};
  for (int j = 0; j < nk; ++j) {
    ks.k[j] = k[j];
    ks.coef[j] = coef[j];
  }
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_axpy_stage, dim3(blocks), dim3(256), 0, s, X, ks, nk, h, out, n);
}

void launch_maxabs(const double* X, int64_t n, unsigned long long* word, hipStream_t s) {
  int blocks = (int)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_maxabs, dim3(blocks), dim3(256), 0, s, X, n, word);
}

void launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
}

void launch_errnorm(const double* y0, const double* y5, const double* const* k, const double* e,
                    int nk, double h, double rtol, double atol, int64_t n, double* red, int nred,
                    hipStream_t s) {
  SlopeSet ks{};
  for (int j = 0; j < nk; ++j) {
    ks.k[j] = k[j];
    ks.coef[j] = e[j];
  }
  hipLaunchKernelGGL(k_errnorm, dim3(nred), dim3(256), 0, s, y0, y5, ks, nk, h, rtol, atol, n,
                     red);
}

}  // namespace tufrg
