// Internal structures of the TUfRG library (host side and kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tufrg.h"

namespace tufrg {

using cplx = std::complex<double>;

// ---------------------------------------------------------------- tables
// Scale-independent data of one point, built once on the host (Sec. 2.5:
// the Kronecker-delta overlaps and Fourier phases do not depend on the
// flow scale).
struct HostTables {
  tufrg_point p{};
  int nff = 0, nq = 0, lk = 0;
  int nshell = 0;                 // shells + 1
  int shell_start[6] = {0};       // form factors and bonds of shell s: [start_s, start_{s+1})
  int rmax = 0;                   // largest bond component
  int smax = 0;                   // largest harmonic component (2 rmax)
  std::vector<int> bx, by;        // bond vectors [nff]
  std::vector<int> parity, irrep; // per form factor; irrep 0..4 = A1,B1,B2,A2,E
  std::vector<cplx> c;            // c[m*nff + b]: f_m(k) = sum_b c_mb exp(-i k.R_b)
  // harmonic set Hs = bonds + bonds (N_S vectors) and its half set Hh
  // (representatives with Sx > 0 or Sx == 0 && Sy >= 0; Hh[0] = (0,0))
  std::vector<int> hx, hy;        // half set [nsh]
  int nsh = 0;                    // N_S' = (N_S + 1)/2
  int ncol = 0;                   // 2 nsh - 1 real harmonic columns (cos, then sin without 0)
  // loops: chi_mn = sum_j Ebub[mn*nsh + j] ghat(S'_j)
  std::vector<double> ebub;       // [nff*nff][nsh]
  // loops: per-px harmonics cos(n px), n = 0..smax, sin(n px), n = 1..smax,
  // per-py weighted harmonics w(py) cos(n py), w(py) sin(n py) for py in [0, Lk/2]
  std::vector<double> pxtab;      // [Lk][2*smax+1]
  std::vector<double> pytab;      // [Lk/2+1][2*smax+1]
  // loops: cos(p_j + q_i/2), cos(p_j - q_i/2) for one axis, [Lq][Lk][2]
  std::vector<double> cshift;
  // projections: phase table E[u][k] = cos(u.S'_k/2) (k < nsh), sin(u.S'_{k-nsh+1}/2)
  std::vector<double> eph;        // [nq][ncol]
  // projections: entry lists per (out channel, V in full set index, A, B)
  // rows = 3 * nsh_full2 * nff * nff where V runs over the half set and its
  // negatives: vfull index v in [0, 2 nsh - 1): v < nsh -> +S'_v, else -S'_{v-nsh+1}
  std::vector<int32_t> mrow;      // CSR row pointers [rows + 1]
  std::vector<int32_t> ment;      // packed entries (see pack_entry)
  int64_t flops_loops = 0, flops_proj = 0, flops_prod = 0;
};

// packed gather entry: input channel (2 bits), bonds b1, b2 (5 bits each),
// harmonic index v in the full list [+S'_0..+S'_{nsh-1}, -S'_1..-S'_{nsh-1}]
// (7 bits), negative sign (1 bit)
inline int32_t pack_entry(int in, int b1, int b2, int v, int neg) {
  return in | (b1 << 2) | (b2 << 7) | (v << 12) | (neg << 19);
}

std::string build_tables(const tufrg_point& p, HostTables& t);   // "" on success
int nff_of_shells(int shells);

// ---------------------------------------------------------- device side
struct DevTables {
  int nff, nq, lq, lk, nsh, ncol, smax;
  double t, tp, mu, U;
  double* cre;   // [nff*nff]
  double* cim;
  int* shell_start;       // [nshell+1]
  int* shell_of;          // [nff]
  double* ebub;  // [nff*nff*nsh]
  double* pxtab; // [lk][2 smax + 1]
  double* pytab; // [lk/2+1][2 smax + 1]
  double* cshift; // [lq][lk][2]: cos(p_j + q_i/2), cos(p_j - q_i/2) per axis
  double* eph;   // [nq][ncol]
  unsigned short* eph_hi;  // BF16 split of eph (mixed precision): eph ~ hi + lo
  unsigned short* eph_lo;
  int32_t* mrow;
  int32_t* ment;
  int32_t* hx;   // half set [nsh]
  int32_t* hy;
  int nshell;
};

struct Workspace {
  double* xt;    // forward transform [3][ncol][nff^2] (largest point)
  double* yb;    // bond-basis transform [2 (re, im)][3][2 nsh - 1][nff^2]
  double* g2;    // inverse-transform coefficients [3][ncol][nff^2]
  double* dpart; // loop slices [nsplit][2][Nq][nff^2] (largest point)
  float* kinv;   // mixed precision: inverse transform K [3][Nq][nff^2] (largest point)
  double* dchi;  // loops [2][S]
  double* stage; // RK stage state [3][S]
  double* k[7];  // RK slopes [3][S] each
  double* ytmp;  // [3][S]
  double* red;   // reduction scratch (doubles)
  unsigned long long* umax; // max-abs words per point
};

}  // namespace tufrg

struct tufrg_ctx {
  std::vector<tufrg::HostTables> host;
  std::vector<tufrg::DevTables> dev;
  std::vector<int64_t> off;   // element offset of each point within a channel
  int64_t S = 0;              // total elements per channel
  tufrg_options opt{};
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;      // loops run here, concurrently with the projections
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  tufrg::Workspace ws{};
  std::vector<void*> allocations;
  std::string err;
  int device = 0;
};

namespace tufrg {
// kernel launchers (kernels.hip); all asynchronous on `s`
// Loop launch geometry of one point: nsplit blocks per transfer momentum, each
// with lk * nchunk threads (rounded up to whole waves).
struct LoopGeom {
  int nsplit, nchunk, threads;
  size_t smem;
};
LoopGeom loop_geometry(const DevTables& d);
// loops at temperature T.  With one split per momentum they land in dchi (this
// point's block in [2][S]); otherwise in the slices dpart[nsplit][2][Nq][nff^2],
// which are added into dchi when sum_slices is set (else the consumer adds them)
void launch_loops(const DevTables& d, double T, double* dchi, int64_t S, double* dpart,
                  bool sum_slices, hipStream_t s);
// projection front end (depends on X only): forward transform, bond basis,
// gather into the inverse-transform coefficients g2
void launch_project_front(const DevTables& d, const double* X, int64_t S, double* xt, double* yb,
                          double* g2, uint32_t flags, hipStream_t s);
// projection back end: mode 0 -> out = V; mode 1 -> out = scale * dX/dT with the
// loops from dchi (one split) or the slices dpart
void launch_project_back(const DevTables& d, const double* X, int64_t S, const double* g2,
                         const double* dchi, const double* dpart, double* out, int mode,
                         uint32_t flags, double scale, hipStream_t s);
// mixed precision (TUFRG_MIXED): FP32 loops, BF16-split MFMA transforms, FP32 products
void launch_loops_mixed(const DevTables& d, double T, double* dchi, int64_t S, double* dpart,
                        bool sum_slices, hipStream_t s);
void launch_project_front_mixed(const DevTables& d, const double* X, int64_t S, double* xt,
                                double* yb, double* g2, uint32_t flags, hipStream_t s);
void launch_inverse_mixed(const DevTables& d, const double* g2, float* K, uint32_t flags,
                          hipStream_t s);
void launch_products_mixed(const DevTables& d, const double* X, int64_t S, const float* K,
                           const double* dchi, const double* dpart, double* out, int mode,
                           uint32_t flags, double scale, hipStream_t s);
size_t loop_smem_mixed(const DevTables& d, const LoopGeom& g);
void launch_axpy_stage(const double* X, const double* const* k, const double* coef, int nk,
                       double h, double* out, int64_t n, hipStream_t s);
void launch_maxabs(const double* X, int64_t n, unsigned long long* word, hipStream_t s);
void launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t s);
void launch_errnorm(const double* y0, const double* y5, const double* const* k, const double* e,
                    int nk, double h, double rtol, double atol, int64_t n, double* red,
                    int nred, hipStream_t s);
}  // namespace tufrg
