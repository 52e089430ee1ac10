// Internal structures of the TUfRG library (host side and kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tufrg.h"

struct tufrg_mlp;

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
  std::vector<int32_t> pairs;     // canonical bond pair of each half-set harmonic [nsh][4]
  // point-group reduction: representatives of the transfer momenta and, per
  // (q, harmonic j), the representative's slot, harmonic and sign (pack_sym)
  int nirr = 0;
  std::vector<int32_t> irr;       // [nirr] flat q of each representative (increasing)
  std::vector<int32_t> symmap;    // [nq][nsh]
  // orbits for symmetric states: X(q) = T X(r) T^T with T a signed permutation
  // of the form factors (pack_perm entries of transform tr, [ntr][nff]);
  // members of representative slot s: orb_q/orb_tr[orb_start[s] .. orb_start[s+1])
  int ntr = 0;
  std::vector<int32_t> tperm;     // [ntr][nff]
  std::vector<int32_t> orb_start; // [nirr + 1]
  std::vector<int32_t> orb_q;     // [nq]
  std::vector<int32_t> orb_tr;    // [nq]
  int nsh = 0;                    // N_S' = (N_S + 1)/2
  int ncol = 0;                   // 2 nsh - 1 real harmonic columns (cos, then sin without 0)
  // loops: chi_mn = sum_j Ebub[mn*nsh + j] ghat(S'_j)
  std::vector<double> ebub;       // [nff*nff][nsh]
  // loops: per-px harmonics cos(n px), n = 0..smax, sin(n px), n = 1..smax,
  // per-py weighted harmonics w(py) cos(n py), w(py) sin(n py) for py in [0, Lk/2]
  std::vector<double> pxtab;      // [Lk][2*smax+1]
  std::vector<double> pytab;      // [Lk/2+1][2*smax+1]
  // loops: cos(p_j + q_i/2), cos(p_j - q_i/2) per axis value, [nx][Lk][2]
  // (x components) and [ny][Lk][2] (y components; the same table on the
  // uniform grid), and per momentum the two axis indices (ix << 16 | iy)
  std::vector<double> cshift, cshift_y;
  std::vector<int32_t> qax;
  // transfer momenta (coordinates) and N_q times their quadrature weights
  // (1 on the uniform grid; the cells' area fractions times N_q on a mesh)
  std::vector<double> qxv, qyv, wq;
  bool mesh = false;
  // projections: phase table E[u][k] = cos(u.S'_k/2) (k < nsh), sin(u.S'_{k-nsh+1}/2)
  std::vector<double> eph;        // [nq][ncol]
  // projections: entry lists per (out channel, V in full set index, A, B)
  // rows = 3 * nsh_full2 * nff * nff where V runs over the half set and its
  // negatives: vfull index v in [0, 2 nsh - 1): v < nsh -> +S'_v, else -S'_{v-nsh+1}
  std::vector<int32_t> mrow;      // CSR row pointers [rows + 1]
  std::vector<int32_t> ment;      // packed entries (see pack_entry)
  int64_t flops_loops = 0, flops_proj = 0, flops_prod = 0;
  int64_t flops_loop_kernel = 0;  // the loop kernel alone (flops_loops adds the chi' expansion)
  // the parts of flops_proj: forward transform, bond basis, gather, inverse transform
  int64_t flops_fwd = 0, flops_basis = 0, flops_gather = 0, flops_inv = 0;
};

// packed gather entry: input channel (2 bits), bonds b1, b2 (5 bits each),
// harmonic index v in the full list [+S'_0..+S'_{nsh-1}, -S'_1..-S'_{nsh-1}]
// (7 bits), negative sign (1 bit)
inline int32_t pack_entry(int in, int b1, int b2, int v, int neg) {
  return in | (b1 << 2) | (b2 << 7) | (v << 12) | (neg << 19);
}

// form-factor permutation entry: source form factor (8 bits), negative sign (bit 8)
inline int32_t pack_perm(int n, int neg) { return n | (neg << 8); }

// symmetry map entry: representative slot (16 bits), harmonic (7 bits), sign (1 bit)
inline int32_t pack_sym(int slot, int j, int neg) { return slot | (j << 16) | (neg << 24); }

std::string build_tables(const tufrg_point& p, const tufrg_mesh* mesh, HostTables& t, bool symmetric,
                         bool omega);   // "" on success; mesh null or nq = 0: uniform grid
int nff_of_shells(int shells);

// ---------------------------------------------------------- device side
constexpr int kLoopThreadsMax = 512;   // loop kernel block size bound
constexpr int64_t kFuseMaxState = 1 << 18;  // largest channel state (sum of Nq Nff^2) run in fused launches
constexpr int kSeg = 1024;             // elements per ODE segment item (4 per thread of 256)
constexpr int kShellMax = 8;           // largest form-factor shell (bonds up to |R|^2 = 5)
constexpr int kEpad = 80;              // padded row length of the phase table copy (ncol <= 69)

// Per-point tables and launch parameters as seen by the kernels (device array).
struct DevTables {
  int nff, nq, lq, lk, nsh, ncol, smax, nshell;
  int nsplit, nchunk;     // loop geometry: row slices per momentum, row chunks per column
  int nsu;                // splits of the transfer grid in the FP64 forward transform
  int nirr;               // representatives of the transfer momenta (point-group orbits)
  double t, tp, mu, U;
  int64_t off;            // element offset of the point inside one channel of [3][S] / [2][S]
  int64_t ws_yb, ws_g2, ws_k;   // element offsets into the shared workspace
  int64_t ws_xp;          // offset of the forward-transform partial sums [nsu][ncol][3 nff^2]
  int64_t ws_gh;          // offset of the point's loop-harmonic slices [nsplit][nirr][2][nsh]
  int64_t gh_off;         // offset of the point's harmonics [nq][2][nsh] in harmonic outputs
  double* dense_A;        // dense projection operator [N][N] column-major (N = 3 nq nff^2), or null
  int64_t ws_dp;          // offset of its partial products [dense_splits][N] in the dense workspace
  int dense_splits;       // splits of the operator's columns
  double* cre;            // [nff*nff]
  double* cim;
  int* shell_start;       // [nshell+1]
  int* shell_of;          // [nff]
  double* ebub;           // [nsh][nff*nff] (the host table transposed: coalesced over mn)
  double* pxtab;          // [lk][2 smax + 1]
  double* pytab;          // [lk/2+1][2 smax + 1]
  double* cshift;         // [nx][lk][2]: cos(p_j + q_x/2), cos(p_j - q_x/2) per x value
  double* cshift_y;       // [ny][lk][2]: the same per y value (= cshift on the uniform grid)
  double* eph;            // [nq][ncol]
  double* ephp;           // [nq][kEpad]: eph padded with zero columns
  // BF16 splits of the phase table (mixed precision: E ~ hi + lo), zero-padded
  unsigned short* ephq_hi; // forward transform: [ceil(nq/16)*4][kEpad][4], quads of momenta
  unsigned short* ephq_lo;
  unsigned short* ephr_hi; // inverse transform: [ceil(nq/64)*64][kEpad]
  unsigned short* ephr_lo;
  int32_t* hx;            // half set [nsh]
  int32_t* hy;
  int32_t* pairs;         // canonical bond pairs [nsh][4]
  int32_t* irr;           // [nirr] flat q of each representative
  int32_t* symmap;        // [nq][nsh] pack_sym(slot, harmonic, sign)
  int32_t* tperm;         // [ntr][nff] pack_perm(source, sign): X(q)_mn = s_m s_n X(r)_{pi(m) pi(n)}
  int32_t* orb_start;     // [nirr + 1] orbit members of each representative slot
  int32_t* orb_q;         // [nq] flat q of each member
  int32_t* orb_tr;        // [nq] its transform
};

// Kernel-side view of one launch: tables, temperatures, stop flags, workspace.
struct Batch {
  const DevTables* pts;   // device array [npts]
  int64_t S;              // channel stride of [3][S] / [2][S] arrays
  const double* Tp;       // per-point temperatures (device)
  const int* frozen;      // per-point stop flags (device) or null
  double* dchi;           // loops [2][S]
  double* xp;             // forward-transform partial sums
  double* yb;             // bond-basis transforms
  double* g2;             // inverse-transform coefficients
  float* kinv;            // inverse transforms (mixed precision)
  double* kinv64;         // inverse transforms (FP64)
  double* ghat;           // loop-harmonic slices (all points, at ws_gh)
  double* dense_ws;       // partial products of the dense projection operator (or null)
  const int* item_count;  // loops: when set, only the first *item_count items run
  int loop_threads;       // threads of the loop geometry (fixes the loops' summation order)
  int wedge;              // symmetric states: inverse transform and products at the orbit
                          // representatives, the increments copied to every orbit member
  DevTables pt0;          // copy of pts[0] (single-point launches read their descriptor
                          // from the kernel arguments: one dependent load fewer)
};

struct ItemRange {
  int begin = 0, n = 0;
};

// Item ranges of one launch set (all points, or one point)
struct Ranges {
  ItemRange loop, exp, fwd, basis, gather, inv, prod, seg;
  ItemRange exp_w;   // loop expansion at the orbit representatives (symmetric states)
  ItemRange dpart, dsum;   // dense projection operator: partial products, their sums
  // the product items by N_ff (contiguous runs of prod): one launch each, with
  // the shared memory of its own N_ff, so that small matrices are not held to
  // the occupancy of the largest
  int nprod_cls = 0;
  ItemRange prod_cls[5];
  int prod_cls_nff[5];
  // the forward-transform items by harmonic tile count KT (contiguous runs of
  // fwd): one launch each, compiled for that KT
  int nfwd_cls = 0;
  ItemRange fwd_cls[5];
  int fwd_cls_kt[5];
};

// Where a fused loops + transform launch takes the temperatures of its
// points: mode 0 reads the per-point array as set before the launch; mode 1
// uses the values v[i] for points p0 + i (i < n <= 64); mode 2 takes the RK4
// stage temperature Ttab[4 step + stage] for every point.  Block 0 of the
// launch also stores them into the per-point array Tp for later kernels.
// Mode 3 takes T = exp(s[p] + c h[p]) from the device arrays of the adaptive
// flow (stage c of the point's current step).
struct TArg {
  int mode, p0, n, npts;
  double* Tp;
  const double* Ttab;
  const int* step;
  int stage;
  const double* s;
  const double* h;
  double c;
  double v[64];
};

// The next stage of an explicit Runge-Kutta step, formed by the kernel that
// writes a slope, element by element as the slope is written:
// out = X + h_p sum_{j < nk} coef_j k_j, where k_{nk-1} is the slope being
// written (its value is taken from the kernel, not read back) and h_p is
// hp[p] (the adaptive flow) or h.  The same operations in the same order as
// the stand-alone stage combination.  nk = 0: no next stage.
struct StageNext {
  const double* X;
  const double* k[7];
  double coef[7];
  double* out;
  const double* hp;
  double h;
  int nk;
};

// Device state of the adaptive (Dormand-Prince) flow, one entry per point.
struct DpState {
  double s, h;            // current scale s = ln T and the step of the next attempt
  double s0, m0, s1, m1;  // the last two accepted (s, max|X|)
  double err;             // error norm of the last attempt
  int status;             // 0 while flowing, else a TUFRG_FLOW_* status
  int n_acc, n_att;       // accepted and attempted steps
  int accept;             // the last attempt was accepted
};

// Device item tables and launch shapes shared by all launches of a context.
struct Launch {
  Batch b;
  const int4* loop_items;
  const int4* exp_items;
  const int4* expw_items; // loop expansion at the representatives (symmetric states) or null
  const int4* fwd_items;
  const int4* inv_items;
  const int4* basis_items;
  const int4* gather_items;
  const int2* gather_ent;  // gather rows' entries: absolute yb offsets (re, im; im < 0 negates)
  int gather_cap;          // entries per gather row (padded with re = -1)
  const int4* prod_items;
  const int4* seg_items;
  const int4* dpart_items;  // dense projection: (p, row tile, column split)
  const int4* dsum_items;   // (p, row tile)
  bool dense = false;       // projections by the dense operator (TUFRG_DENSE_PROJECTION)
  int loop_threads, loop_blocks, smax_max;
  int fwd_kt;             // forward transform: 16-row harmonic tiles (1, 2, 3 or 5)
  int inv_lt;             // inverse transform: 16-momentum tiles per item (1, 2 or 4)
  int front_threads;      // block of the forward transform and of the loops + transform launch
  bool fused;             // right-hand side in fused launches on one stream (small contexts)
  size_t fwd_smem;        // forward transform: dynamic LDS
  size_t front_smem;      // loops + transform launch: dynamic LDS
  bool loop_persistent;   // loop kernel: persistent work queue, or one block per item
  size_t loop_smem, prod_smem;
  bool omega = false;     // the scale is the Omega cutoff at T = 0 (temperatures hold Om)
  bool one_point = false; // the context has one point: kernels take p = 0 without the item's
  bool loop_unroll = false;  // loop kernel: two FP64 rows in flight (when the launch needs no
                             // more blocks per CU than that form's occupancy allows)
};

// Surrogate state of a single-point context (device pointers and settings).
struct SurState {
  double tol;                 // relative tolerance of the ensemble and residual checks
  int stride;                 // one momentum in `stride` is checked per call, rotating
  int* phase;                 // [1] current check phase
  int* state;                 // [nirr] fallback flags of the representatives
  int* need;                  // [nirr] exact kernel this call
  int* fail;                  // [nirr] failed check this call
  double* pred;               // [nirr][2][nsh] predicted harmonics
  double* fin;                // [nirr][2][nsh] harmonics used this call
  int4* items;                // [nirr * nsplit] loop items of the exact representatives
  int* count;                 // [1] number of those items
  unsigned long long* stats;  // [3] exact, queried representatives, failed checks (cumulative)
};

void launch_loops(const Launch& L, const ItemRange& r, int* queue, bool mixed, hipStream_t s);
// chi' of every momentum from the loop harmonics of the representatives:
// from the slices in b.ghat (fin == null), or from fin [nirr][2][nsh] of a
// single-point context
void launch_chi_expand(const Launch& L, const ItemRange& r, const double* fin, double* dchi,
                       hipStream_t s);
void launch_front(const Launch& L, const Ranges& r, const double* X, bool mixed, hipStream_t s);
// the projections' cross terms K (inverse-transform output) by the dense operator
void launch_dense(const Launch& L, const Ranges& r, const double* X, hipStream_t s);
void launch_set_unit(double* X, int64_t prev, int64_t cur, hipStream_t s);
void launch_fwd(const Launch& L, const Ranges& r, const double* X, bool mixed, hipStream_t s);
void launch_gather_inv(const Launch& L, const Ranges& r, bool mixed, hipStream_t s);
// the parts of launch_front one at a time (bond basis, gather, inverse transform)
void launch_basis(const Launch& L, const Ranges& r, hipStream_t s);
void launch_gather(const Launch& L, const Ranges& r, hipStream_t s);
void launch_inv(const Launch& L, const Ranges& r, bool mixed, hipStream_t s);
void launch_loops_fwd(const Launch& L, const Ranges& r, const double* X, bool mixed, bool cross,
                      const TArg& ta, hipStream_t s);
void launch_expand_basis(const Launch& L, const Ranges& r, double* dchi, bool cross, hipStream_t s);
// sn (or null): the next stage formed where the products write dX (mode 1)
void launch_back(const Launch& L, const Ranges& r, const double* X, double* out, int mode,
                 bool cross, bool scale_T, bool mixed, hipStream_t s, const StageNext* sn = nullptr);
// hp (device, per point) or null: the step of point p is hp[p] (the adaptive
// flow) instead of h
void launch_axpy(const Launch& L, const ItemRange& r, const double* X, const double* const* k,
                 const double* coef, int nk, double h, double* out, bool skip_frozen, hipStream_t s,
                 const double* hp = nullptr);
void launch_maxabs(const Launch& L, const ItemRange& r, const double* X, unsigned long long* words,
                   hipStream_t s);
// per point, the smallest local flat index whose |X| has the bit pattern
// words[p] (atomic minimum into first[p], which starts at INT_MAX)
void launch_first_max(const Launch& L, const ItemRange& r, const double* X, const unsigned long long* words,
                      int* first, hipStream_t s);
// the last Dormand-Prince stage: y5, the error partial sums and max|y5| per point
void launch_dp_final(const Launch& L, const ItemRange& r, const double* y0, const double* const* k,
                     const double* b5, const double* e, double h, double rtol, double atol, double* y5,
                     double* red, unsigned long long* max_words, hipStream_t s, const double* hp = nullptr);
// the adaptive flow's step control of every point (one block per point) and
// the acceptance of its new state (y = y5 and k0 = k6 where accepted)
struct DpControl {
  DpState* st;
  int* frozen;
  const int2* seg;        // per point: first error partial sum and their count
  const double* n_el;     // per point: elements of the state (3 Nq Nff^2)
  const double* red;      // error partial sums of the attempt
  unsigned long long* max_words;
  double* s_arr;          // per point s and h, read by the next attempt's kernels
  double* h_arr;
  double s_end, xmax;
  int max_steps, npts;
  int* status_out;        // mapped host memory or null: each point's status after the attempt
};
void launch_dp_control(const DpControl& c, hipStream_t s);
// y = y5 and k0 = k6 where the attempt was accepted, then the first stage of
// the next attempt, stage1 = y + h_p (a10 k0), for every point still flowing
void launch_dp_accept(const Launch& L, const ItemRange& r, const DpState* st, const double* y5, const double* k6,
                      double* y, double* k0, double a10, const double* h_arr, double* stage1, hipStream_t s);
void launch_set_T_sh(double* Tp, int npts, const double* s_arr, const double* h_arr, double c, hipStream_t s);
void launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t s);
// per-point largest deviation of X from the C4v covariance law (items (p, slot))
void launch_sym_defect(const Launch& L, const int2* items, int n, const double* X, unsigned long long* words,
                       hipStream_t s);
void launch_fill_i32(int* p, int n, int v, hipStream_t s);
void launch_set_T(double* Tp, int npts, const double* Ttab, const int* step, int stage,
                  hipStream_t s);
void launch_set_T_values(double* Tp, const double* T_host, int n, hipStream_t s);
void launch_step_end(unsigned long long* words, int npts, int* frozen, double* hist, int* step,
                     int nsteps, double xmax, hipStream_t s, int* status_out = nullptr);
const void* loop_kernel_symbol(int smax_max, bool mixed, bool omega, bool unroll);
void launch_ghat_sum(const Launch& L, int p, const DevTables& d, double* out, hipStream_t s);
void launch_sur_dataset(const Launch& L, int npts, int64_t n, uint64_t seed, float* x, float* y,
                        int32_t* idx, hipStream_t s);
void launch_surrogate_front(const Launch& L, int p, const DevTables& d, float* x, hipStream_t s);
void launch_surrogate_decide(const Launch& L, int p, const DevTables& d, const float* ya, const float* yb,
                             const SurState& st, hipStream_t s);
void launch_surrogate_finish(const Launch& L, int p, const DevTables& d, const SurState& st, hipStream_t s);
// forward pass of an MLP on stream s (rows in chunks of the net's max_rows)
void mlp_forward_on(tufrg_mlp* net, const float* x, float* y, int64_t rows, hipStream_t s);
int mlp_width(const tufrg_mlp* net, int i);   // widths[i]; i = -1: the last
int mlp_max_rows(const tufrg_mlp* net);

}  // namespace tufrg

struct tufrg_ctx {
  std::vector<tufrg::HostTables> host;
  std::vector<tufrg::DevTables> dev;       // host copy of the device array
  std::vector<int64_t> off;                // element offset of each point within a channel
  int64_t S = 0;                           // total elements per channel
  tufrg_options opt{};
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;              // loops run here, concurrently with the projections
  hipStream_t gs = nullptr;                // capture and replay stream of the graph-driven flow
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_gs = nullptr;
  hipEvent_t ev_att[2] = {nullptr, nullptr}; // the adaptive flow's attempts, alternating
  tufrg::Launch L{};
  tufrg::Ranges all;                       // item ranges of all points
  std::vector<tufrg::Ranges> per_point;    // item ranges of each point
  // device buffers owned by the context
  double* Tp = nullptr;                    // per-point temperatures
  int* frozen = nullptr;                   // per-point stop flags
  int* first_max = nullptr;                // per-point first index of max|X| (classification)
  int* queue = nullptr;                    // loop-kernel work queue: next item, finished blocks
  bool flow_ready = false;                 // flow state buffers allocated (first tufrg_flow)
  double* stage = nullptr;                 // RK stage states [3][S] (two, alternating)
  double* stage2 = nullptr;
  double* kk[7] = {nullptr};               // RK slopes [3][S]
  double* ytmp = nullptr;                  // [3][S]
  double* red = nullptr;                   // reduction scratch
  double* red_host = nullptr;              // pinned copy of red
  int nred = 0;
  unsigned long long* umax = nullptr;      // per-point max words
  unsigned long long* umax_host = nullptr; // pinned
  int* flow_status_host = nullptr;         // pinned, mapped: per-point stop words of a flow
  int* flow_status_dev = nullptr;          // its device address
  double* Ttab = nullptr;                  // RK4 stage temperatures [nsteps][4]
  double* hist = nullptr;                  // max|X| history [nsteps+1][npts]
  int* step = nullptr;                     // device step counter
  int ttab_cap = 0;
  bool loop_persistent = false;            // launch form of the loop kernel
  double* ghat = nullptr;                  // loop-harmonic slices of the representatives
  int64_t ghat_len = 0, ghat_sum_len = 0;  // slice and summed lengths over all points
  // attached surrogate (single-point contexts)
  tufrg_mlp* sur_a = nullptr;
  tufrg_mlp* sur_b = nullptr;
  tufrg::SurState sur{};
  float* sur_x = nullptr;                  // [nq * nsh][9] features
  float* sur_ya = nullptr;                 // [nq * nsh][4] predictions of each network
  float* sur_yb = nullptr;
  std::vector<void*> sur_allocations;
  std::vector<void*> allocations;          // freed by tufrg_free
  std::vector<void*> geometry_allocations; // item tables and slices; rebuilt by the autotuner
  std::string err;
  int device = 0;
  // workspace totals (elements) of the step calls, for the no-allocation entry point
  int64_t ws_total_xp = 0, ws_total_yb = 0, ws_total_g2 = 0, ws_total_k = 0;
  void* scratch = nullptr;                 // device address of the static scratch on ctx->device
  tufrg::DpState* dp_state = nullptr;             // adaptive flow: per-point state (device)
  double* dp_sh = nullptr;                 // [2][npts] s and h of every point (device)
  int2* dp_seg = nullptr;                  // [npts] first error partial sum and count
  double* dp_nel = nullptr;                // [npts] state elements 3 Nq Nff^2
  int2* sym_items = nullptr;               // (point, representative slot) of every orbit
  int n_sym_items = 0;
  unsigned long long* sym_words = nullptr; // per-point covariance defect words
};
