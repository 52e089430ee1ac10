// C ABI of the TUfRG library: context, validation, tables and workspace, the
// work-item tables that let one launch cover any set of points, the step
// calls, the loop-geometry autotuner and the ODE flow driver (batched RK4 with
// device-side stopping and optional HIP-graph replay; per-point Dormand-Prince).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "tufrg_internal.h"

using namespace tufrg;

// Static device scratch of the allocation-free right-hand side
// (tufrg_rhs_noalloc): its workspace lives here instead of in the context's
// allocations.  Each device the library runs on holds its own copy until the
// process ends.  In host code `scratch` only names the symbol: its device
// address on the current device comes from hipGetSymbolAddress.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

thread_local std::string g_last_error = "";

tufrg_status fail(tufrg_ctx* ctx, tufrg_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  g_last_error = msg;
  return st;
}

#define HIP_TRY(ctx, expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(ctx, TUFRG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define ST_TRY(expr)               \
  do {                             \
    tufrg_status s_ = (expr);      \
    if (s_ != TUFRG_OK) return s_; \
  } while (0)

// device allocation of `count` elements recorded in `list` (freed with it)
template <class T>
tufrg_status dalloc(tufrg_ctx* ctx, size_t count, T** out, std::vector<void*>& list) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(count * sizeof(T), 16)) != hipSuccess)
    return fail(ctx, TUFRG_ENOMEM, "hipMalloc failed (" + std::to_string(count * sizeof(T)) + " bytes)");
  list.push_back(p);
  *out = static_cast<T*>(p);
  return TUFRG_OK;
}

template <class T>
tufrg_status upload(tufrg_ctx* ctx, const std::vector<T>& v, T** out, std::vector<void*>& list) {
  ST_TRY(dalloc(ctx, std::max<size_t>(v.size(), 1), out, list));
  if (!v.empty()) HIP_TRY(ctx, hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return TUFRG_OK;
}

// ------------------------------------------------------- BF16 split (host)
// round-to-nearest-even BF16 bits of a float, and the hi/lo split of a double
unsigned short bf16_bits(float f) {
  unsigned int u;
  std::memcpy(&u, &f, sizeof u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
float bf16_value(unsigned short h) {
  unsigned int u = ((unsigned int)h) << 16;
  float f;
  std::memcpy(&f, &u, sizeof f);
  return f;
}
void split_table(const std::vector<double>& x, std::vector<unsigned short>& hi,
                 std::vector<unsigned short>& lo) {
  hi.resize(x.size());
  lo.resize(x.size());
  for (size_t i = 0; i < x.size(); ++i) {
    const float f = (float)x[i];
    hi[i] = bf16_bits(f);
    lo[i] = bf16_bits(f - bf16_value(hi[i]));
  }
}

// Device address of `scratch` on device dev (the current device), resolved
// once per device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

hipError_t resolve_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

constexpr double kSymmetryTol = 1e-12;   // relative covariance defect accepted as symmetric
constexpr int64_t kDenseMaxN = 8192;      // largest 3 Nq Nff^2 of the dense projection operator (512 MiB)
constexpr int kDenseColsHost = 64;        // its column splits (the kernel's kDenseCols)

double word_to_double(unsigned long long w) {
  double d;
  std::memcpy(&d, &w, sizeof d);
  return d;
}

// ------------------------------------------------------- loop geometry
int round64(int x) { return ((x + 63) / 64) * 64; }

// LDS bytes of the loop kernel for point d in blocks of `threads` threads
size_t loop_smem_of(const DevTables& d, int threads) {
  const int rows = d.lk / 2 + 1, nrmax = (rows + d.nsplit - 1) / d.nsplit;
  const int NH = 2 * d.smax + 1, nout = 2 * d.nsh;
  int nseg = threads / nout;
  if (nseg < 1) nseg = 1;
  return sizeof(double) *
         ((size_t)2 * nrmax + (size_t)nrmax * NH + (size_t)d.lk * 3 * NH + (size_t)nseg * nout);
}

// Default loop geometry: two row slices (separate work items) per
// representative transfer momentum when the half fine grid has at least 16
// rows, then the fewest row chunks (threads of one column) that put about two
// waves per SIMD in flight and leave at most 16 rows per thread, with at most
// kLoopThreadsMax threads per block and at least 2 rows per thread.  (Fitted
// to the autotuner's choices; TUFRG_AUTOTUNE searches the full range.)
void default_geometry(DevTables& d) {
  const int rows = d.lk / 2 + 1;
  const int64_t target_waves = (int64_t)256 * 4 * 2;
  const int nsplit = rows >= 16 ? 2 : 1;
  auto waves = [&](int nc) { return (int64_t)d.nirr * nsplit * ((d.lk * nc + 63) / 64); };
  int nchunk = 1;
  while (d.lk * (nchunk + 1) <= kLoopThreadsMax && rows / (nsplit * (nchunk + 1)) >= 2 &&
         (waves(nchunk) < target_waves || rows / (nsplit * nchunk) > 16))
    ++nchunk;
  d.nsplit = nsplit;
  d.nchunk = nchunk;
}

// ------------------------------------------------------------ item tables
struct HostItems {
  std::vector<int4> loop, exp, expw, fwd, basis, gather, inv, prod, seg, dpart, dsum;
  std::vector<int2> gent;   // gather rows' entries, gather_cap per row
};

template <class F>
void mark(std::vector<int4>& v, ItemRange& rg, F fill) {
  rg.begin = (int)v.size();
  fill(v);
  rg.n = (int)v.size() - rg.begin;
}

// The work items of point p for every kernel, appended to h; r receives the
// point's ranges.  Item layouts are those documented at each kernel.
// Inverse-transform rows and product items: every momentum, or with symmetric
// states (wedge) one representative per orbit (items carry its slot).
int inv_rows_of(const DevTables& d, bool wedge) { return wedge ? d.nirr : d.nq; }

void add_point_items(const DevTables& d, const HostTables& t, int p, int inv_lt, int fwd_cols, bool wedge,
                     int gcap, bool split_basis, HostItems& h, Ranges& r) {
  const int nff2 = d.nff * d.nff, nv = 2 * d.nsh - 1;
  const int nrow = inv_rows_of(d, wedge);
  mark(h.exp, r.exp, [&](std::vector<int4>& v) {
    for (int rt = 0; rt < (2 * d.nq + 31) / 32; ++rt)
      for (int ct = 0; ct < (nff2 + 63) / 64; ++ct) v.push_back(make_int4(p, rt, ct, 0));
  });
  // symmetric states: chi' at the representatives only (rows (channel, slot),
  // item.w = 1), which is all the products read
  if (wedge)
    mark(h.expw, r.exp_w, [&](std::vector<int4>& v) {
      for (int rt = 0; rt < (2 * d.nirr + 31) / 32; ++rt)
        for (int ct = 0; ct < (nff2 + 63) / 64; ++ct) v.push_back(make_int4(p, rt, ct, 1));
    });
  mark(h.fwd, r.fwd, [&](std::vector<int4>& v) {
    for (int sp = 0; sp < d.nsu; ++sp)
      for (int c = 0; c < (3 * nff2 + fwd_cols - 1) / fwd_cols; ++c) v.push_back(make_int4(p, c, sp, 0));
  });
  mark(h.inv, r.inv, [&](std::vector<int4>& v) {
    for (int lt = 0; lt < (nrow + 16 * inv_lt - 1) / (16 * inv_lt); ++lt)
      for (int c = 0; c < (3 * nff2 + 63) / 64; ++c) v.push_back(make_int4(p, lt, c, 0));
  });
  // bond-basis items (p, harmonic, r0, r1): with split_basis (the fused
  // launches of small contexts, whose basis blocks are fewer than the CUs) the
  // rows in two groups of whole shells, cut at the shell boundary closest to
  // the middle (three shells or more), so that the launch has twice the
  // blocks; otherwise all rows in one item (measured: the split made the
  // two-stream right-hand side at 48x48, N_ff = 21 slower in the mixed form)
  mark(h.basis, r.basis, [&](std::vector<int4>& v) {
    int cut = d.nff;
    if (split_basis && d.nshell >= 3) {
      for (int s = 1; s < d.nshell; ++s)
        if (std::abs(2 * t.shell_start[s] - d.nff) < std::abs(2 * cut - d.nff)) cut = t.shell_start[s];
    }
    for (int b = 0; b < 3 * nv; ++b) {
      v.push_back(make_int4(p, b, 0, cut));
      if (cut < d.nff) v.push_back(make_int4(p, b, cut, d.nff));
    }
  });
  // gather items (p, packed block, -, first entry): the block's harmonic j,
  // output channel X and shell pair (start and size of each) packed into y,
  // and its rows' entries (gcap per row, in the entry lists' order) as
  // absolute offsets into yb, so that the kernel reaches yb in two loads
  mark(h.gather, r.gather, [&](std::vector<int4>& v) {
    const int ns = d.nshell, nv2 = 2 * d.nsh - 1, ybim = 3 * nv2 * nff2;
    for (int j = 0; j < d.nsh; ++j)
      for (int x = 0; x < 3 * ns * ns; ++x) {
        const int X = x / (ns * ns), sm = x / ns % ns, sn = x % ns;
        const int a0 = t.shell_start[sm], na = t.shell_start[sm + 1] - a0;
        const int b0 = t.shell_start[sn], nb = t.shell_start[sn + 1] - b0;
        const int nvl = j == 0 ? 1 : 2, nab = na * nb;
        const int packed = j | (X << 8) | (na << 10) | (nb << 14) | (a0 << 18) | (b0 << 23);
        v.push_back(make_int4(p, packed, 0, (int)h.gent.size()));
        for (int w = 0; w < nvl * nab; ++w) {
          const int vi = w / nab, rr = w % nab, vf = vi == 0 ? j : d.nsh - 1 + j;
          const size_t row = ((size_t)X * nv2 + vf) * nff2 + (size_t)(a0 + rr / nb) * d.nff + b0 + rr % nb;
          int k = 0;
          for (int e = t.mrow[row]; e < t.mrow[row + 1]; ++e, ++k) {
            const int32_t pk = t.ment[(size_t)e];
            const int in = pk & 3, b1 = (pk >> 2) & 31, b2 = (pk >> 7) & 31, vv = (pk >> 12) & 127;
            const int o = (int)d.ws_yb + ((in * nv2 + vv) * nff2 + b1 * d.nff + b2);
            const int im = o + ybim;
            h.gent.push_back(make_int2(o, ((pk >> 19) & 1) ? -(im + 1) : im));
          }
          for (; k < gcap; ++k) h.gent.push_back(make_int2(-1, 0));
        }
      }
  });
  mark(h.prod, r.prod, [&](std::vector<int4>& v) {
    if (wedge)
      for (int sl = 0; sl < d.nirr; ++sl) v.push_back(make_int4(p, t.irr[(size_t)sl], sl, 0));
    else
      for (int l = 0; l < d.nq; ++l) v.push_back(make_int4(p, l, 0, 0));
  });
  mark(h.seg, r.seg, [&](std::vector<int4>& v) {
    const int chunks = (d.nq * nff2 + kSeg - 1) / kSeg;
    for (int c = 0; c < 3; ++c)
      for (int k = 0; k < chunks; ++k) v.push_back(make_int4(p, c, k, 0));
  });
  // dense projection operator: (p, tile of 256 rows, column split), (p, tile)
  if (d.dense_A) {
    const int tiles = (3 * d.nq * nff2 + 255) / 256;
    mark(h.dpart, r.dpart, [&](std::vector<int4>& v) {
      for (int s2 = 0; s2 < d.dense_splits; ++s2)
        for (int rt = 0; rt < tiles; ++rt) v.push_back(make_int4(p, rt, s2, 0));
    });
    mark(h.dsum, r.dsum, [&](std::vector<int4>& v) {
      for (int rt = 0; rt < tiles; ++rt) v.push_back(make_int4(p, rt, 0, 0));
    });
  }
}

// harmonic tiles of 16 rows the forward transform of point d needs (the
// kernel is compiled for 1, 2, 3 and 5)
int fwd_kt_of(const DevTables& d) {
  const int k = (d.ncol + 15) / 16;
  return k <= 3 ? k : 5;
}

// loop items of one point: one per (representative momentum, row slice),
// (p, slot * nsplit + split, flat q of the representative, its axis indices
// ix << 16 | iy into the shifted-cosine tables)
void add_loop_items(const DevTables& d, const HostTables& t, int p, std::vector<int4>& v, ItemRange& r) {
  mark(v, r, [&](std::vector<int4>& w) {
    for (int b = 0; b < d.nirr * d.nsplit; ++b) {
      const int q = t.irr[b / d.nsplit];
      w.push_back(make_int4(p, b, q, t.qax[(size_t)q]));
    }
  });
}

bool mixed_of(const tufrg_ctx* ctx) { return ctx->opt.precision == TUFRG_MIXED; }
bool cross_of(const tufrg_ctx* ctx) { return !(ctx->opt.flags & TUFRG_NO_CROSS); }
bool omega_of(const tufrg_ctx* ctx) { return (ctx->opt.flags & TUFRG_OMEGA_CUTOFF) != 0; }

// Item tables, slice buffers, launch shapes and the device table array from
// the current per-point geometry (replaces those of an earlier build).
tufrg_status build_launch(tufrg_ctx* ctx) {
  const int npts = (int)ctx->dev.size();
  const bool mixed = mixed_of(ctx);
  if (!ctx->geometry_allocations.empty()) {
    HIP_TRY(ctx, hipDeviceSynchronize());
    for (void* p : ctx->geometry_allocations) (void)hipFree(p);
    ctx->geometry_allocations.clear();
  }
  HostItems h;
  ctx->per_point.assign(npts, Ranges());
  // Loop items of costlier points first: the persistent loop kernel takes
  // items in table order, so the longest tasks start first.
  std::vector<int> order(npts);
  std::iota(order.begin(), order.end(), 0);
  auto cost = [&](int p) {
    const DevTables& d = ctx->dev[p];
    return (double)d.lk * (d.lk / 2 + 1) / d.nsplit * (2 * d.smax + 5);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  for (int p : order) add_loop_items(ctx->dev[p], ctx->host[p], p, h.loop, ctx->per_point[p].loop);
  const bool wedge = (ctx->opt.flags & TUFRG_SYMMETRIC_STATE) != 0;
  // entries per gather row: the longest row of any point
  int gcap = 1;
  for (const HostTables& t : ctx->host)
    for (size_t r = 0; r + 1 < t.mrow.size(); ++r) gcap = std::max(gcap, t.mrow[r + 1] - t.mrow[r]);
  for (const DevTables& d : ctx->dev)   // gather entries hold yb offsets as int
    if (d.ws_yb + (int64_t)6 * (2 * d.nsh - 1) * d.nff * d.nff > (int64_t)INT32_MAX)
      return fail(ctx, TUFRG_EINVAL, "bond-basis workspace beyond 2^31 elements");
  // inverse-transform momentum tile: the largest of 64, 32, 16 that still
  // gives the launch 512 items
  int64_t inv_items[3] = {0, 0, 0};
  for (const DevTables& d : ctx->dev)
    for (int i = 0; i < 3; ++i)
      inv_items[i] += (int64_t)((inv_rows_of(d, wedge) + (16 << i) - 1) / (16 << i)) * ((3 * d.nff * d.nff + 63) / 64);
  const int inv_lt = inv_items[2] >= 512 ? 4 : (inv_items[1] >= 512 ? 2 : 1);
  // loop block (the largest point's loop geometry).  Small problems are
  // bound by launch and synchronisation cost: there the loops share launches
  // with the projections on one stream (the forward transform then runs in
  // blocks of the loops' size, 16 columns per wave); larger ones overlap the
  // two on two streams.
  int threads = 64;
  for (const DevTables& d : ctx->dev) threads = std::max(threads, round64(d.lk * d.nchunk));
  const bool fused = ctx->S <= kFuseMaxState && !ctx->loop_persistent && !(ctx->opt.flags & TUFRG_NO_FUSE);
  const int front_threads = fused ? std::max(threads, 256) : 256, fwd_cols = 16 * (front_threads / 64);
  // points in decreasing N_ff, so that the product items of one N_ff are contiguous
  std::vector<int> by_nff(npts);
  std::iota(by_nff.begin(), by_nff.end(), 0);
  std::stable_sort(by_nff.begin(), by_nff.end(), [&](int x, int y) { return ctx->dev[x].nff > ctx->dev[y].nff; });
  for (int p : by_nff) {
    Ranges& rp = ctx->per_point[p];
    add_point_items(ctx->dev[p], ctx->host[p], p, inv_lt, fwd_cols, wedge, gcap, fused, h, rp);
    rp.nprod_cls = 1;
    rp.prod_cls[0] = rp.prod;
    rp.prod_cls_nff[0] = ctx->dev[p].nff;
    rp.nfwd_cls = 1;
    rp.fwd_cls[0] = rp.fwd;
    rp.fwd_cls_kt[0] = fwd_kt_of(ctx->dev[p]);
  }
  int smax_max = 0;
  size_t lsm = 0, psm = 0;
  int kpt = 1;
  int64_t gh = 0, ghs = 0;
  for (int p = 0; p < npts; ++p) {
    DevTables& d = ctx->dev[p];
    smax_max = std::max(smax_max, d.smax);
    const int nff2 = d.nff * d.nff;
    psm = std::max(psm, sizeof(double) * 10 * (size_t)nff2);
    kpt = std::max(kpt, (d.ncol + 15) / 16);
    d.ws_gh = gh;
    gh += (int64_t)d.nsplit * d.nirr * 2 * d.nsh;
    d.gh_off = ghs;
    ghs += (int64_t)d.nq * 2 * d.nsh;
  }
  ctx->ghat_len = gh;
  ctx->ghat_sum_len = ghs;
  for (int p = 0; p < npts; ++p) lsm = std::max(lsm, loop_smem_of(ctx->dev[p], threads));
  const int fwd_kt = kpt <= 3 ? kpt : 5;   // the largest fwd_kt_of over the points
  // forward transform LDS: FP64 chunks of 32 momenta [32][16 KT + 2] + [32][cols + 2];
  // split precision: hi and lo quads [8][16 KT] + [8][cols] (8 bytes each)
  const size_t fsm = mixed ? (size_t)16 * 8 * (16 * fwd_kt + fwd_cols)
                           : sizeof(double) * 32 * ((size_t)(16 * fwd_kt + 2) + (size_t)(fwd_cols + 2));
  int dev_smem = 0;
  (void)hipDeviceGetAttribute(&dev_smem, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device);
  if (dev_smem > 0 && (lsm > (size_t)dev_smem || psm > (size_t)dev_smem || fsm > (size_t)dev_smem))
    return fail(ctx, TUFRG_EINVAL, "grids too large for the shared memory of one block");
  auto whole = [](const std::vector<int4>& v) {
    ItemRange r;
    r.n = (int)v.size();
    return r;
  };
  Ranges& all = ctx->all;
  all.loop = whole(h.loop); all.exp = whole(h.exp); all.exp_w = whole(h.expw); all.fwd = whole(h.fwd);
  all.basis = whole(h.basis); all.gather = whole(h.gather);
  all.inv = whole(h.inv); all.prod = whole(h.prod);
  all.seg = whole(h.seg);
  all.dpart = whole(h.dpart);
  all.dsum = whole(h.dsum);
  all.nfwd_cls = 0;
  for (int p : by_nff) {
    const ItemRange& fr = ctx->per_point[p].fwd;
    const int kt = fwd_kt_of(ctx->dev[p]);
    if (all.nfwd_cls > 0 && all.fwd_cls_kt[all.nfwd_cls - 1] == kt) {
      all.fwd_cls[all.nfwd_cls - 1].n = fr.begin + fr.n - all.fwd_cls[all.nfwd_cls - 1].begin;
    } else {
      all.fwd_cls[all.nfwd_cls] = fr;
      all.fwd_cls_kt[all.nfwd_cls] = kt;
      ++all.nfwd_cls;
    }
  }
  all.nprod_cls = 0;
  for (int p : by_nff) {
    const ItemRange& pr = ctx->per_point[p].prod;
    const int nff = ctx->dev[p].nff;
    if (all.nprod_cls > 0 && all.prod_cls_nff[all.nprod_cls - 1] == nff) {
      all.prod_cls[all.nprod_cls - 1].n = pr.begin + pr.n - all.prod_cls[all.nprod_cls - 1].begin;
    } else {
      all.prod_cls[all.nprod_cls] = pr;
      all.prod_cls_nff[all.nprod_cls] = nff;
      ++all.nprod_cls;
    }
  }
  Launch& L = ctx->L;
  std::vector<void*>& g = ctx->geometry_allocations;
  int4* t = nullptr;
  ST_TRY(upload(ctx, h.loop, &t, g)); L.loop_items = t;
  ST_TRY(upload(ctx, h.exp, &t, g)); L.exp_items = t;
  L.expw_items = nullptr;
  if (!h.expw.empty()) {
    ST_TRY(upload(ctx, h.expw, &t, g));
    L.expw_items = t;
  }
  ST_TRY(upload(ctx, h.fwd, &t, g)); L.fwd_items = t;
  ST_TRY(upload(ctx, h.inv, &t, g)); L.inv_items = t;
  ST_TRY(upload(ctx, h.basis, &t, g)); L.basis_items = t;
  ST_TRY(upload(ctx, h.gather, &t, g)); L.gather_items = t;
  {
    int2* ge = nullptr;
    ST_TRY(upload(ctx, h.gent, &ge, g));
    L.gather_ent = ge;
    L.gather_cap = gcap;
  }
  ST_TRY(upload(ctx, h.prod, &t, g)); L.prod_items = t;
  ST_TRY(upload(ctx, h.seg, &t, g)); L.seg_items = t;
  ST_TRY(upload(ctx, h.dpart, &t, g)); L.dpart_items = t;
  ST_TRY(upload(ctx, h.dsum, &t, g)); L.dsum_items = t;
  ST_TRY(dalloc(ctx, (size_t)std::max<int64_t>(gh, 1), &L.b.ghat, g));
  ctx->ghat = L.b.ghat;
  DevTables* dp = nullptr;
  ST_TRY(upload(ctx, ctx->dev, &dp, g));
  L.b.pts = dp;
  L.b.pt0 = ctx->dev[0];
  L.b.S = ctx->S;
  L.b.Tp = ctx->Tp;
  L.b.frozen = nullptr;
  L.smax_max = smax_max;
  L.loop_threads = threads;
  L.loop_smem = lsm;
  L.prod_smem = psm;
  L.fwd_kt = fwd_kt;
  L.inv_lt = inv_lt;
  L.front_threads = front_threads;
  L.fused = fused;
  L.fwd_smem = fsm;
  L.front_smem = std::max(lsm, fsm);
  L.b.loop_threads = threads;
  L.b.wedge = wedge ? 1 : 0;
  L.one_point = npts == 1;
  L.omega = omega_of(ctx);
  // blocks of the loop kernel per CU in each form; the form with two rows in
  // flight when the items need no more blocks per CU than it allows
  int cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
  if (cus < 1) cus = 1;
  auto per_cu_of = [&](bool unroll) {
    int n = 0;
    const void* k = loop_kernel_symbol(smax_max, mixed, omega_of(ctx), unroll);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, threads, lsm) != hipSuccess || n < 1)
      n = 1;
    return n;
  };
  const int per_cu_unroll = per_cu_of(true);
  const int nloop = (int)h.loop.size();
  L.loop_unroll = !ctx->loop_persistent && (nloop + cus - 1) / cus <= per_cu_unroll;
  // persistent loop grid: every CU filled to the kernel's occupancy
  const int per_cu = L.loop_unroll ? per_cu_unroll : per_cu_of(false);
  L.loop_blocks = cus * per_cu;
  L.loop_persistent = ctx->loop_persistent;
  return TUFRG_OK;
}

// Largest relative deviation of X from the C4v covariance law over the
// points (max|X(q) - T X(r) T^T| / max|X| per point; 0 for X = 0).
// Synchronises the stream.
tufrg_status symmetry_defect(tufrg_ctx* ctx, const double* X, double* rel) {
  const int npts = (int)ctx->dev.size();
  launch_fill_u64(ctx->sym_words, npts, 0ull, ctx->stream);
  launch_fill_u64(ctx->umax, npts, 0ull, ctx->stream);
  launch_sym_defect(ctx->L, ctx->sym_items, ctx->n_sym_items, X, ctx->sym_words, ctx->stream);
  launch_maxabs(ctx->L, ctx->all.seg, X, ctx->umax, ctx->stream);
  std::vector<unsigned long long> dw(npts), mw(npts);
  HIP_TRY(ctx, hipMemcpyAsync(dw.data(), ctx->sym_words, sizeof(unsigned long long) * npts, hipMemcpyDeviceToHost,
                              ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(mw.data(), ctx->umax, sizeof(unsigned long long) * npts, hipMemcpyDeviceToHost,
                              ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  double worst = 0.0;
  for (int p = 0; p < npts; ++p) {
    const double dv = word_to_double(dw[p]), mv = word_to_double(mw[p]);
    const double r = (dv == 0.0) ? 0.0 : dv / mv;
    if (!(r <= worst)) worst = r;   // NaN propagates
  }
  *rel = worst;
  return TUFRG_OK;
}

// ------------------------------------------------------------ RHS driver
// One right-hand side over the item ranges r on stream ms: out = dX/dT, or
// T dX/dT (= dX/ds) when scale_T.  The loops depend on T only and run on the
// side stream, concurrently with the X-dependent front end of the
// projections; the back end (V and the products) joins both.
// Loops through the attached surrogate (single-point context): predicted
// harmonics of the representatives, exact loop kernel on those that need it,
// the check and fallback bookkeeping, and chi' of every momentum into dchi.
void surrogate_loops(tufrg_ctx* ctx, const Launch& L, double* dchi, hipStream_t s) {
  const DevTables& d = ctx->dev[0];
  const int64_t rows = (int64_t)d.nirr * d.nsh;
  launch_surrogate_front(L, 0, d, ctx->sur_x, s);
  mlp_forward_on(ctx->sur_a, ctx->sur_x, ctx->sur_ya, rows, s);
  // one network: its prediction is compared with itself (no disagreement),
  // so acceptance rests on the rotating check and the fallback flags
  const float* yb = ctx->sur_ya;
  if (ctx->sur_b) {
    mlp_forward_on(ctx->sur_b, ctx->sur_x, ctx->sur_yb, rows, s);
    yb = ctx->sur_yb;
  }
  launch_surrogate_decide(L, 0, d, ctx->sur_ya, yb, ctx->sur, s);
  Launch Lg = L;
  Lg.b.item_count = ctx->sur.count;
  Lg.loop_items = ctx->sur.items;
  ItemRange r;
  r.n = d.nirr * d.nsplit;
  launch_loops(Lg, r, ctx->queue, false, s);
  launch_surrogate_finish(L, 0, d, ctx->sur, s);
  launch_chi_expand(L, ctx->all.exp, ctx->sur.fin, dchi, s);
}

// Loops of the ranges r into dchi: the loop kernel on the representatives,
// then chi' of every momentum (or the surrogate path when attached).
void loops_launch(tufrg_ctx* ctx, const Launch& L, const Ranges& r, double* dchi, hipStream_t s) {
  if (ctx->sur_a) {
    surrogate_loops(ctx, L, dchi, s);
    return;
  }
  launch_loops(L, r.loop, ctx->queue, mixed_of(ctx), s);
  launch_chi_expand(L, r.exp, nullptr, dchi, s);
}

// The temperatures of one right-hand side: host values for points p0 .. p0+n-1,
// or (host == nullptr) the RK4 stage temperature Ttab[4 step + stage] of every
// point, read on the device.
// With sh set: T = exp(s[p] + c h[p]) of the adaptive flow's device state
// (stage c of every point's current step).
struct TSource {
  const double* host;
  int p0, n;
  int stage;
  const double* s = nullptr;
  const double* h = nullptr;
  double c = 0.0;
};

// Stores the temperatures into the per-point array on stream s.
void set_T_launch(tufrg_ctx* ctx, const TSource& ts, hipStream_t s) {
  if (ts.host) launch_set_T_values(ctx->Tp + ts.p0, ts.host, ts.n, s);
  else if (ts.s) launch_set_T_sh(ctx->Tp, (int)ctx->dev.size(), ts.s, ts.h, ts.c, s);
  else launch_set_T(ctx->Tp, (int)ctx->dev.size(), ctx->Ttab, ctx->step, ts.stage, s);
}

// One right-hand side on stream ms.  The loops and the projections are
// independent until the products, so they share launches on one stream:
// (loops + forward transform), (loop expansion + bond basis), gather,
// inverse transform, products, when the context is small enough for launch
// costs to dominate (Launch::fused).  Otherwise, and with the surrogate, the
// loops run on the side stream (fork and join by events) alongside the
// whole projection chain.
// same_T: the right-hand side issued just before this one on the context
// took the same temperatures (two stages at the same s: RK4's second and
// third, RK4's first and the last of the step before, Dormand-Prince's sixth
// and seventh), so its loop
// expansion, still in dchi, is used again and the loop and expansion work is
// not issued (the loops read only T; the bits are those of a fresh
// evaluation).  Not with the surrogate, whose checks count its calls.
void rhs_launch(tufrg_ctx* ctx, const Launch& L0, const Ranges& r0, const double* X, double* out,
                bool scale_T, hipStream_t ms, const TSource& ts, const StageNext* sn = nullptr,
                bool same_T = false) {
  const bool mixed = mixed_of(ctx), cross = cross_of(ctx);
  // symmetric states: the loop expansion at the representatives only
  Launch L = L0;
  Ranges r = r0;
  if (L0.b.wedge && L0.expw_items) {
    L.exp_items = L0.expw_items;
    r.exp = r0.exp_w;
  }
  const bool reuse = same_T && !ctx->sur_a && !(ctx->opt.flags & TUFRG_NO_LOOP_REUSE);
  if (reuse) {
    r.loop.n = 0;
    r.exp.n = 0;
  }
  if (!ctx->sur_a && L.fused) {
    // the fused launch takes the temperatures itself (and stores them for the
    // products), except for host values of more than 64 points
    TArg ta{};
    ta.Tp = ctx->Tp;
    ta.npts = (int)ctx->dev.size();
    if (ts.host && ts.n <= 64) {
      ta.mode = 1;
      ta.p0 = ts.p0;
      ta.n = ts.n;
      for (int i = 0; i < ts.n; ++i) ta.v[i] = ts.host[i];
    } else if (!ts.host && ts.s) {
      ta.mode = 3;
      ta.s = ts.s;
      ta.h = ts.h;
      ta.c = ts.c;
    } else if (!ts.host) {
      ta.mode = 2;
      ta.Ttab = ctx->Ttab;
      ta.step = ctx->step;
      ta.stage = ts.stage;
    } else {
      set_T_launch(ctx, ts, ms);
    }
    // with the dense projection operator the loops share no launch with the
    // forward transform: the cross terms come from one operator product
    const bool factored = cross && !L.dense;
    launch_loops_fwd(L, r, X, mixed, factored, ta, ms);
    launch_expand_basis(L, r, L.b.dchi, factored, ms);
    if (factored) launch_gather_inv(L, r, mixed, ms);
    else if (cross) launch_dense(L, r, X, ms);
    launch_back(L, r, X, out, 1, cross, scale_T, mixed, ms, sn);
    return;
  }
  if (reuse) {
    if (cross && L.dense) launch_dense(L, r, X, ms);
    else if (cross) launch_front(L, r, X, mixed, ms);
    launch_back(L, r, X, out, 1, cross, scale_T, mixed, ms, sn);
    return;
  }
  // fork and join: errors of these calls are read with hipGetLastError by every caller
  (void)hipEventRecord(ctx->ev_fork, ms);
  (void)hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0);
  set_T_launch(ctx, ts, ctx->side);
  loops_launch(ctx, L, r, L.b.dchi, ctx->side);
  (void)hipEventRecord(ctx->ev_join, ctx->side);
  if (cross && L.dense) launch_dense(L, r, X, ms);
  else if (cross) launch_front(L, r, X, mixed, ms);
  (void)hipStreamWaitEvent(ms, ctx->ev_join, 0);
  launch_back(L, r, X, out, 1, cross, scale_T, mixed, ms, sn);
}

// V of every point (eqns. proj_VP/VC/VD) on the context's stream.
void project_launch(tufrg_ctx* ctx, const double* X, double* V) {
  const bool mixed = mixed_of(ctx), cross = cross_of(ctx);
  if (cross && ctx->L.dense) launch_dense(ctx->L, ctx->all, X, ctx->stream);
  else if (cross) launch_front(ctx->L, ctx->all, X, mixed, ctx->stream);
  launch_back(ctx->L, ctx->all, X, V, 0, cross, false, mixed, ctx->stream);
}

// max |V| of every point's projected couplings at the state X (V in the
// flow's stage buffer) into res[p].max_abs_V.  Synchronises the stream.
tufrg_status flow_max_abs_V(tufrg_ctx* ctx, const double* X, tufrg_flow_result* res) {
  const int npts = (int)ctx->dev.size();
  project_launch(ctx, X, ctx->stage);
  launch_fill_u64(ctx->umax, npts, 0ull, ctx->stream);
  launch_maxabs(ctx->L, ctx->all.seg, ctx->stage, ctx->umax, ctx->stream);
  std::vector<unsigned long long> w(npts);
  HIP_TRY(ctx, hipMemcpyAsync(w.data(), ctx->umax, sizeof(unsigned long long) * npts, hipMemcpyDeviceToHost,
                              ctx->stream));
  launch_fill_u64(ctx->umax, npts, 0ull, ctx->stream);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int p = 0; p < npts; ++p) res[p].max_abs_V = word_to_double(w[p]);
  return TUFRG_OK;
}

// The flows' per-point stop words in pinned, mapped host memory: the step
// kernels write them, so that the host can follow a flow without
// synchronising the stream (allocated on the first flow, kept until
// tufrg_free).
tufrg_status ensure_status_words(tufrg_ctx* ctx) {
  if (ctx->flow_status_host) return TUFRG_OK;
  void* hp = nullptr;
  void* dp = nullptr;
  if (hipHostMalloc(&hp, sizeof(int) * ctx->dev.size(), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
    return fail(ctx, TUFRG_ENOMEM, "pinned host allocation failed");
  ctx->flow_status_host = static_cast<int*>(hp);
  if (hipHostGetDevicePointer(&dp, hp, 0) != hipSuccess)
    return fail(ctx, TUFRG_EHIP, "no device address for the mapped status words");
  ctx->flow_status_dev = static_cast<int*>(dp);
  return TUFRG_OK;
}

tufrg_status ensure_flow_buffers(tufrg_ctx* ctx) {
  if (ctx->flow_ready) return TUFRG_OK;
  const size_t s3 = 3 * (size_t)ctx->S;
  ST_TRY(dalloc(ctx, s3, &ctx->stage, ctx->allocations));
  ST_TRY(dalloc(ctx, s3, &ctx->stage2, ctx->allocations));
  ST_TRY(dalloc(ctx, s3, &ctx->ytmp, ctx->allocations));
  for (int i = 0; i < 7; ++i) ST_TRY(dalloc(ctx, s3, &ctx->kk[i], ctx->allocations));
  ctx->flow_ready = true;
  return TUFRG_OK;
}

tufrg_status check_temperatures(tufrg_ctx* ctx, const double* T_host) {
  for (size_t p = 0; p < ctx->dev.size(); ++p)
    if (!(T_host[p] > 0.0) || !std::isfinite(T_host[p]))
      return fail(ctx, TUFRG_EINVAL, "T must be finite and > 0 (point " + std::to_string(p) + ")");
  return TUFRG_OK;
}

// The dense projection operator of every point (precomputed projection data,
// Sec. 2.5 and the stored projection tensors of the appendix on symmetries):
// column j of A is the projections' cross terms K of the unit state e_j,
// computed by the factored path, so that afterwards one operator product
// replaces the forward transform, bond basis, gather and inverse transform.
tufrg_status build_dense(tufrg_ctx* ctx) {
  double* Xp = nullptr;
  const size_t n3 = 3 * (size_t)ctx->S;
  if (hipMalloc(&Xp, n3 * sizeof(double)) != hipSuccess) return fail(ctx, TUFRG_ENOMEM, "dense operator probe");
  hipError_t e = hipMemsetAsync(Xp, 0, n3 * sizeof(double), ctx->stream);
  int64_t prev = -1;
  for (size_t p = 0; p < ctx->dev.size() && e == hipSuccess; ++p) {
    const DevTables& d = ctx->dev[p];
    const int64_t nqn = (int64_t)d.nq * d.nff * d.nff, N = 3 * nqn;
    for (int64_t j = 0; j < N && e == hipSuccess; ++j) {
      const int64_t cur = (j / nqn) * ctx->S + d.off + j % nqn;
      launch_set_unit(Xp, prev, cur, ctx->stream);
      prev = cur;
      launch_front(ctx->L, ctx->per_point[p], Xp, false, ctx->stream);
      e = hipMemcpyAsync(d.dense_A + j * N, ctx->L.b.kinv64 + d.ws_k, (size_t)N * sizeof(double),
                         hipMemcpyDeviceToDevice, ctx->stream);
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = hipGetLastError();
  (void)hipFree(Xp);
  if (e != hipSuccess) return fail(ctx, TUFRG_EHIP, std::string("dense operator: ") + hipGetErrorString(e));
  ctx->L.dense = true;
  return TUFRG_OK;
}

// ------------------------------------------------------------ autotuner
// Times every candidate loop geometry (row slices x row chunks) of each
// distinct point shape in launches of that point alone and keeps the fastest.
std::string tune_key(const DevTables& d, int precision) {
  char k[128];
  std::snprintf(k, sizeof k, "gfx950_nq%d_nirr%d_lk%d_nff%d_prec%d", d.nq, d.nirr, d.lk, d.nff, precision);
  return k;
}

tufrg_status autotune(tufrg_ctx* ctx) {
  const int npts = (int)ctx->dev.size();
  const bool mixed = mixed_of(ctx);
  std::map<std::string, std::pair<int, int>> known;
  const char* path = std::getenv("TUFRG_TUNE_CACHE");
  if (path) {
    std::ifstream in(path);
    std::string k;
    int a, b;
    while (in >> k >> a >> b)
      if (a >= 1 && b >= 1) known[k] = {a, b};
  }
  std::vector<double> T(npts, 0.05);
  launch_set_T_values(ctx->Tp, T.data(), npts, ctx->stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  std::map<std::string, std::pair<int, int>> fresh;
  tufrg_status st = TUFRG_OK;
  for (int p = 0; p < npts && !st; ++p) {
    DevTables& d = ctx->dev[p];
    const std::string key = tune_key(d, ctx->opt.precision);
    const int rows = d.lk / 2 + 1;
    auto fits = [&](int ns, int nc) { return d.lk * nc <= kLoopThreadsMax && rows / (ns * nc) >= 2; };
    std::pair<int, int> prior{0, 0};
    if (known.count(key)) prior = known[key];
    else if (fresh.count(key)) prior = fresh[key];
    if (prior.first > 0 && fits(prior.first, prior.second)) {
      d.nsplit = prior.first;
      d.nchunk = prior.second;
      continue;
    }
    double best = 1e300;
    int bs = d.nsplit, bc = d.nchunk;
    for (int ns = 1; ns <= 16 && !st; ns *= 2)
      for (int nc = 1; nc <= 8 && !st; ++nc) {
        if (!fits(ns, nc)) continue;
        d.nsplit = ns;
        d.nchunk = nc;
        if ((st = build_launch(ctx))) break;
        const ItemRange r = ctx->per_point[p].loop;
        for (int w = 0; w < 2; ++w) launch_loops(ctx->L, r, ctx->queue, mixed, ctx->stream);
        const int reps = 5;
        float ms = 0.f;
        if (hipEventRecord(e0, ctx->stream) != hipSuccess) { st = fail(ctx, TUFRG_EHIP, "event"); break; }
        for (int w = 0; w < reps; ++w) launch_loops(ctx->L, r, ctx->queue, mixed, ctx->stream);
        if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          st = fail(ctx, TUFRG_EHIP, "autotuner timing failed");
          break;
        }
        if (ms < best) {
          best = ms;
          bs = ns;
          bc = nc;
        }
      }
    d.nsplit = bs;
    d.nchunk = bc;
    fresh[key] = {bs, bc};
  }
  // Batches: the shapes were timed alone (latency); with many items in flight
  // fewer, longer blocks can serve the whole launch better.  Time every
  // point's row slices divided by 1, 2, 4, 8 on the whole batch and keep the
  // fastest (cached under the batch's multiset of shapes).
  if (!st && npts > 1) {
    std::vector<std::string> shapes;
    for (int p = 0; p < npts; ++p) shapes.push_back(tune_key(ctx->dev[p], ctx->opt.precision));
    std::sort(shapes.begin(), shapes.end());
    uint64_t hsh = 1469598103934665603ull;   // FNV-1a over the sorted shape keys
    for (const std::string& k : shapes)
      for (unsigned char c : k + ";") hsh = (hsh ^ c) * 1099511628211ull;
    char bk[64];
    std::snprintf(bk, sizeof bk, "batch_%016llx", (unsigned long long)hsh);
    std::vector<int> ns0(npts);
    for (int p = 0; p < npts; ++p) ns0[p] = ctx->dev[p].nsplit;
    auto apply = [&](int f) {
      for (int p = 0; p < npts; ++p) ctx->dev[p].nsplit = std::max(1, ns0[p] / f);
    };
    int best_f = 1;
    if (known.count(bk)) {
      best_f = known[bk].first;
    } else {
      double best = 1e300;
      for (int f = 1; f <= 8 && !st; f *= 2) {
        if (f > 1 && std::all_of(ns0.begin(), ns0.end(), [&](int n) { return n / (f / 2) <= 1; })) break;
        apply(f);
        if ((st = build_launch(ctx))) break;
        for (int w = 0; w < 2; ++w) launch_loops(ctx->L, ctx->all.loop, ctx->queue, mixed, ctx->stream);
        const int reps = 5;
        float ms = 0.f;
        if (hipEventRecord(e0, ctx->stream) != hipSuccess) { st = fail(ctx, TUFRG_EHIP, "event"); break; }
        for (int w = 0; w < reps; ++w) launch_loops(ctx->L, ctx->all.loop, ctx->queue, mixed, ctx->stream);
        if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          st = fail(ctx, TUFRG_EHIP, "autotuner timing failed");
          break;
        }
        if (ms < best) {
          best = ms;
          best_f = f;
        }
      }
      fresh[bk] = {best_f, 1};
    }
    apply(best_f);
  }
  // launch form of the whole batch: one block per item, or the persistent queue
  if (!st) st = build_launch(ctx);
  double form_ms[2] = {0.0, 0.0};
  for (int f = 0; f < 2 && !st; ++f) {
    ctx->L.loop_persistent = (f == 1);
    for (int w = 0; w < 2; ++w) launch_loops(ctx->L, ctx->all.loop, ctx->queue, mixed, ctx->stream);
    const int reps = 5;
    float ms = 0.f;
    if (hipEventRecord(e0, ctx->stream) != hipSuccess) { st = fail(ctx, TUFRG_EHIP, "event"); break; }
    for (int w = 0; w < reps; ++w) launch_loops(ctx->L, ctx->all.loop, ctx->queue, mixed, ctx->stream);
    if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(ctx, TUFRG_EHIP, "autotuner timing failed");
      break;
    }
    form_ms[f] = ms;
  }
  ctx->loop_persistent = !st && form_ms[1] < form_ms[0];
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  if (path && !fresh.empty()) {
    std::ofstream out(path, std::ios::app);
    for (auto& kv : fresh)
      if (!known.count(kv.first)) out << kv.first << " " << kv.second.first << " " << kv.second.second << "\n";
  }
  return build_launch(ctx);
}

}  // namespace

// ================================================================== C ABI
extern "C" {

tufrg_status tufrg_init(const tufrg_point* pts, int32_t npts, const tufrg_options* opt, void* stream,
                        tufrg_ctx** out) {
  return tufrg_init_mesh(pts, nullptr, npts, opt, stream, out);
}

tufrg_status tufrg_init_mesh(const tufrg_point* pts, const tufrg_mesh* meshes, int32_t npts,
                             const tufrg_options* opt, void* stream, tufrg_ctx** out) {
  if (!out) return fail(nullptr, TUFRG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!pts || npts <= 0) return fail(nullptr, TUFRG_EINVAL, "need at least one point");
  tufrg_options o{};
  if (opt) o = *opt;
  if (o.precision != TUFRG_FP64 && o.precision != TUFRG_MIXED)
    return fail(nullptr, TUFRG_EINVAL, "precision must be TUFRG_FP64 or TUFRG_MIXED");
  if (o.flags & ~(uint32_t)(TUFRG_NO_CROSS | TUFRG_AUTOTUNE | TUFRG_LOOP_QUEUE | TUFRG_NO_SYMMETRY |
                            TUFRG_NO_FUSE | TUFRG_OMEGA_CUTOFF | TUFRG_SYMMETRIC_STATE | TUFRG_DENSE_PROJECTION |
                            TUFRG_NO_LOOP_REUSE))
    return fail(nullptr, TUFRG_EINVAL, "unknown flag bits");
  if ((o.flags & TUFRG_DENSE_PROJECTION) && (o.precision != TUFRG_FP64 || (o.flags & TUFRG_SYMMETRIC_STATE)))
    return fail(nullptr, TUFRG_EUNSUPPORTED, "the dense projection operator serves FP64 per-momentum contexts");
  auto* ctx = new tufrg_ctx();
  ctx->opt = o;
  ctx->stream = static_cast<hipStream_t>(stream);
  ctx->loop_persistent = (o.flags & TUFRG_LOOP_QUEUE) != 0;
  ctx->host.resize(npts);
  ctx->off.resize(npts);
  ctx->dev.assign(npts, DevTables());
  int64_t S = 0, ws_yb = 0, ws_g2 = 0, ws_k = 0, ws_xp = 0;
  for (int p = 0; p < npts; ++p) {
    const tufrg_mesh* mp = meshes && meshes[p].nq != 0 ? &meshes[p] : nullptr;
    std::string e = build_tables(pts[p], mp, ctx->host[p], !(o.flags & TUFRG_NO_SYMMETRY),
                                 (o.flags & TUFRG_OMEGA_CUTOFF) != 0);
    if (e.empty() && mp && (o.flags & TUFRG_SYMMETRIC_STATE)) {
      delete ctx;
      return fail(nullptr, TUFRG_EUNSUPPORTED, "point " + std::to_string(p) +
                                                   ": symmetric states need the uniform transfer grid");
    }
    if (e.empty() && ctx->host[p].lk > kLoopThreadsMax)
      e = "Lk must be <= " + std::to_string(kLoopThreadsMax);
    for (int sh = 0; e.empty() && sh < ctx->host[p].nshell; ++sh)
      if (ctx->host[p].shell_start[sh + 1] - ctx->host[p].shell_start[sh] > kShellMax)
        e = "form-factor shell larger than " + std::to_string(kShellMax);
    if (!e.empty()) {
      delete ctx;
      return fail(nullptr, TUFRG_EINVAL, "point " + std::to_string(p) + ": " + e);
    }
    const HostTables& t = ctx->host[p];
    DevTables& d = ctx->dev[p];
    std::memset(&d, 0, sizeof d);
    d.nff = t.nff; d.nq = t.nq; d.lq = t.p.Lq; d.lk = t.lk; d.nsh = t.nsh; d.ncol = t.ncol;
    d.smax = t.smax; d.nshell = t.nshell; d.nirr = t.nirr;
    d.t = t.p.t; d.tp = t.p.tp; d.mu = t.p.mu; d.U = t.p.U;
    default_geometry(d);
    // splits of the transfer grid in the forward transform: about 512 work
    // items per point, at least 64 momenta per split (every split writes a
    // full partial sum that the next kernel reads again, so fewer, longer
    // splits where the point is small)
    const int nff2 = t.nff * t.nff;
    const int ctiles = (3 * nff2 + 63) / 64;
    d.nsu = std::max(1, std::min(512 / ctiles, t.nq / 64));
    d.off = S;
    ctx->off[p] = S;
    S += (int64_t)t.nq * nff2;
    d.ws_g2 = ws_g2;
    ws_g2 += (int64_t)3 * t.ncol * nff2;
    d.ws_yb = ws_yb;
    ws_yb += (int64_t)2 * 3 * (2 * t.nsh - 1) * nff2;
    d.ws_k = ws_k;
    ws_k += (int64_t)3 * t.nq * nff2;
    d.ws_xp = ws_xp;
    ws_xp += (int64_t)d.nsu * t.ncol * 3 * nff2;
  }
  ctx->S = S;
  // first device call: every argument has been validated
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return fail(nullptr, TUFRG_EHIP, "no HIP device");
  }
  ctx->ws_total_xp = ws_xp;
  ctx->ws_total_yb = ws_yb;
  ctx->ws_total_g2 = ws_g2;
  ctx->ws_total_k = ws_k;
  {
    // the static scratch of this device (used by tufrg_rhs_noalloc only)
    const hipError_t e = resolve_scratch(ctx->device, &ctx->scratch);
    if (e != hipSuccess) {
      delete ctx;
      return fail(nullptr, TUFRG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
  }
  auto bad = [&](tufrg_status st) {
    std::string m = ctx->err;
    tufrg_free(ctx);
    return fail(nullptr, st, m);
  };
  std::vector<void*>& A = ctx->allocations;
  for (int p = 0; p < npts; ++p) {
    const HostTables& t = ctx->host[p];
    DevTables& d = ctx->dev[p];
    std::vector<double> cre(t.c.size()), cim(t.c.size());
    for (size_t i = 0; i < t.c.size(); ++i) {
      cre[i] = t.c[i].real();
      cim[i] = t.c[i].imag();
    }
    std::vector<int> ss(t.shell_start, t.shell_start + t.nshell + 1);
    std::vector<int> so(t.nff);
    for (int s = 0; s < t.nshell; ++s)
      for (int m = t.shell_start[s]; m < t.shell_start[s + 1]; ++m) so[m] = s;
    std::vector<int32_t> hx(t.hx.begin(), t.hx.end()), hy(t.hy.begin(), t.hy.end());
    std::vector<double> ebub_t(t.ebub.size());
    for (int mn = 0; mn < t.nff * t.nff; ++mn)
      for (int j = 0; j < t.nsh; ++j) ebub_t[(size_t)j * t.nff * t.nff + mn] = t.ebub[(size_t)mn * t.nsh + j];
    // the forward transform's copy of the phase table carries N_q times the
    // quadrature weight of each momentum (exactly 1 on the uniform grid; the
    // bond-basis kernel divides the sums by N_q); the inverse transform's
    // tables are the plain phases
    std::vector<double> ephp((size_t)t.nq * kEpad, 0.0), ephu((size_t)t.nq * kEpad, 0.0);
    for (int u = 0; u < t.nq; ++u)
      for (int k = 0; k < t.ncol; ++k) {
        ephu[(size_t)u * kEpad + k] = t.eph[(size_t)u * t.ncol + k];
        ephp[(size_t)u * kEpad + k] = t.wq[u] * t.eph[(size_t)u * t.ncol + k];
      }
    // BF16 splits of the phase table in the two layouts of the mixed transforms
    std::vector<unsigned short> ehi, elo, uhi, ulo;
    split_table(ephp, ehi, elo);
    split_table(ephu, uhi, ulo);
    const size_t nq16 = (size_t)(t.nq + 15) / 16 * 16, nq64 = (size_t)(t.nq + 63) / 64 * 64;
    std::vector<unsigned short> qhi(nq16 * kEpad, 0), qlo(nq16 * kEpad, 0);
    std::vector<unsigned short> rhi(nq64 * kEpad, 0), rlo(nq64 * kEpad, 0);
    for (int u = 0; u < t.nq; ++u)
      for (int k = 0; k < kEpad; ++k) {
        const size_t src = (size_t)u * kEpad + k, q = ((size_t)(u / 4) * kEpad + k) * 4 + u % 4;
        qhi[q] = ehi[src];
        qlo[q] = elo[src];
        rhi[src] = uhi[src];
        rlo[src] = ulo[src];
      }
    tufrg_status st;
    if ((st = upload(ctx, cre, &d.cre, A)) || (st = upload(ctx, cim, &d.cim, A)) ||
        (st = upload(ctx, ss, &d.shell_start, A)) || (st = upload(ctx, so, &d.shell_of, A)) ||
        (st = upload(ctx, ebub_t, &d.ebub, A)) || (st = upload(ctx, t.pxtab, &d.pxtab, A)) ||
        (st = upload(ctx, t.pytab, &d.pytab, A)) || (st = upload(ctx, t.eph, &d.eph, A)) ||
        (st = upload(ctx, ephp, &d.ephp, A)) ||
        (st = upload(ctx, t.cshift, &d.cshift, A)) || (st = upload(ctx, qhi, &d.ephq_hi, A)) ||
        (!t.cshift_y.empty() && (st = upload(ctx, t.cshift_y, &d.cshift_y, A))) ||
        (st = upload(ctx, qlo, &d.ephq_lo, A)) || (st = upload(ctx, rhi, &d.ephr_hi, A)) ||
        (st = upload(ctx, rlo, &d.ephr_lo, A)) || (st = upload(ctx, hx, &d.hx, A)) ||
        (st = upload(ctx, hy, &d.hy, A)) || (st = upload(ctx, t.pairs, &d.pairs, A)) ||
        (st = upload(ctx, t.irr, &d.irr, A)) || (st = upload(ctx, t.symmap, &d.symmap, A)) ||
        (st = upload(ctx, t.tperm, &d.tperm, A)) || (st = upload(ctx, t.orb_start, &d.orb_start, A)) ||
        (st = upload(ctx, t.orb_q, &d.orb_q, A)) || (st = upload(ctx, t.orb_tr, &d.orb_tr, A)))
      return bad(st);
    if (t.cshift_y.empty()) d.cshift_y = d.cshift;   // the uniform grid: one table for both axes
  }
  // workspace, state buffers and control words
  Batch& B = ctx->L.b;
  tufrg_status st = TUFRG_OK;
  if (!st) st = dalloc(ctx, 2 * (size_t)S, &B.dchi, A);
  if (!st) st = dalloc(ctx, (size_t)std::max<int64_t>(ws_yb, 1), &B.yb, A);
  if (!st) st = dalloc(ctx, (size_t)std::max<int64_t>(ws_g2, 1), &B.g2, A);
  B.kinv = nullptr;
  if (!st && o.precision == TUFRG_MIXED) st = dalloc(ctx, (size_t)std::max<int64_t>(ws_k, 1), &B.kinv, A);
  if (!st && o.precision != TUFRG_MIXED) st = dalloc(ctx, (size_t)std::max<int64_t>(ws_k, 1), &B.kinv64, A);
  if (!st) st = dalloc(ctx, (size_t)std::max<int64_t>(ws_xp, 1), &B.xp, A);
  B.dense_ws = nullptr;
  if (!st && (o.flags & TUFRG_DENSE_PROJECTION)) {
    // the dense operator of every point (filled below) and the partial sums
    int64_t wsd = 0;
    for (int p = 0; p < npts && !st; ++p) {
      DevTables& d = ctx->dev[p];
      const int64_t N = 3 * (int64_t)d.nq * d.nff * d.nff;
      if (N > kDenseMaxN) {
        st = fail(ctx, TUFRG_EINVAL, "point " + std::to_string(p) + ": the dense projection operator needs 3 Nq Nff^2 <= " +
                                         std::to_string(kDenseMaxN) + " (it stores (3 Nq Nff^2)^2 doubles)");
        break;
      }
      st = dalloc(ctx, (size_t)(N * N), &d.dense_A, A);
      d.dense_splits = (int)((N + kDenseColsHost - 1) / kDenseColsHost);
      d.ws_dp = wsd;
      wsd += (int64_t)d.dense_splits * N;
    }
    if (!st) st = dalloc(ctx, (size_t)std::max<int64_t>(wsd, 1), &B.dense_ws, A);
  }
  if (!st) st = dalloc(ctx, (size_t)npts, &ctx->Tp, A);
  if (!st) st = dalloc(ctx, (size_t)npts, &ctx->frozen, A);
  if (!st) st = dalloc(ctx, (size_t)npts, &ctx->first_max, A);
  if (!st) st = dalloc(ctx, 2, &ctx->queue, A);
  if (!st) st = dalloc(ctx, (size_t)npts, &ctx->umax, A);
  if (!st) st = dalloc(ctx, 1, &ctx->step, A);
  if (!st) st = dalloc(ctx, (size_t)npts, &ctx->sym_words, A);
  if (!st) {
    std::vector<int2> si;
    for (int p = 0; p < npts; ++p)
      for (int sl = 0; sl < ctx->host[p].nirr; ++sl) si.push_back(make_int2(p, sl));
    ctx->n_sym_items = (int)si.size();
    st = upload(ctx, si, &ctx->sym_items, A);
  }
  if (st) return bad(st);
  if (hipHostMalloc((void**)&ctx->umax_host, sizeof(unsigned long long) * npts, 0) != hipSuccess)
    return bad(fail(ctx, TUFRG_ENOMEM, "pinned host allocation failed"));
  // side and graph streams (default priority) and the fork/join events
  if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&ctx->gs, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_gs, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_att[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_att[1], hipEventDisableTiming) != hipSuccess)
    return bad(fail(ctx, TUFRG_EHIP, "stream or event creation failed"));
  // loop-kernel work queue: zero once, then reset by every launch at its end
  launch_fill_i32(ctx->queue, 2, 0, ctx->stream);
  // item tables and launch shapes, tuned on request
  st = build_launch(ctx);
  if (!st && (o.flags & TUFRG_AUTOTUNE)) st = autotune(ctx);
  if (!st && (o.flags & TUFRG_DENSE_PROJECTION)) st = build_dense(ctx);
  if (st) return bad(st);
  if (hipDeviceSynchronize() != hipSuccess)
    return bad(fail(ctx, TUFRG_EHIP, "device synchronize failed after init"));
  *out = ctx;
  return TUFRG_OK;
}

tufrg_status tufrg_layout(const tufrg_ctx* ctx, int32_t point, int64_t* offset, int32_t* Nq,
                          int32_t* Nff, int64_t* total) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (point < 0 || point >= (int)ctx->host.size())
    return fail(const_cast<tufrg_ctx*>(ctx), TUFRG_EINVAL, "point out of range");
  if (offset) *offset = ctx->off[point];
  if (Nq) *Nq = ctx->host[point].nq;
  if (Nff) *Nff = ctx->host[point].nff;
  if (total) *total = ctx->S;
  return TUFRG_OK;
}

tufrg_status tufrg_geometry(const tufrg_ctx* ctx, int32_t point, int32_t* nsplit, int32_t* nchunk,
                            int32_t* threads, int32_t* persistent) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (point < 0 || point >= (int)ctx->dev.size())
    return fail(const_cast<tufrg_ctx*>(ctx), TUFRG_EINVAL, "point out of range");
  if (nsplit) *nsplit = ctx->dev[point].nsplit;
  if (nchunk) *nchunk = ctx->dev[point].nchunk;
  if (threads) *threads = ctx->L.loop_threads;
  if (persistent) *persistent = ctx->L.loop_persistent ? 1 : 0;
  return TUFRG_OK;
}

tufrg_status tufrg_bubbles(tufrg_ctx* ctx, const double* T_host, double* dchi) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (!T_host || !dchi) return fail(ctx, TUFRG_EINVAL, "NULL argument");
  ST_TRY(check_temperatures(ctx, T_host));
  launch_set_T_values(ctx->Tp, T_host, (int)ctx->dev.size(), ctx->stream);
  loops_launch(ctx, ctx->L, ctx->all, dchi, ctx->stream);
  HIP_TRY(ctx, hipGetLastError());
  return TUFRG_OK;
}

tufrg_status tufrg_project(tufrg_ctx* ctx, const double* X, double* V) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (!X || !V) return fail(ctx, TUFRG_EINVAL, "NULL argument");
  if (X == V) return fail(ctx, TUFRG_EINVAL, "X and V must not alias");
  project_launch(ctx, X, V);
  HIP_TRY(ctx, hipGetLastError());
  return TUFRG_OK;
}

tufrg_status tufrg_rhs(tufrg_ctx* ctx, const double* T_host, const double* X, double* dXdT) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (!T_host || !X || !dXdT) return fail(ctx, TUFRG_EINVAL, "NULL argument");
  if (X == dXdT) return fail(ctx, TUFRG_EINVAL, "X and dXdT must not alias");
  ST_TRY(check_temperatures(ctx, T_host));
  rhs_launch(ctx, ctx->L, ctx->all, X, dXdT, false, ctx->stream,
             TSource{T_host, 0, (int)ctx->dev.size(), 0});
  HIP_TRY(ctx, hipGetLastError());
  return TUFRG_OK;
}

tufrg_status tufrg_rhs_noalloc(tufrg_ctx* ctx, const double* T_host, const double* X, double* dXdT) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (!T_host || !X || !dXdT) return fail(ctx, TUFRG_EINVAL, "NULL argument");
  if (X == dXdT) return fail(ctx, TUFRG_EINVAL, "X and dXdT must not alias");
  if (ctx->sur_a) return fail(ctx, TUFRG_EUNSUPPORTED, "the allocation-free right-hand side has no surrogate path");
  if (!ctx->scratch) return fail(ctx, TUFRG_EHIP, "static scratch not resolved on this device");
  ST_TRY(check_temperatures(ctx, T_host));
  // workspace regions inside the static scratch (doubles, 256-byte aligned):
  // loops, forward-transform splits, bond basis, inverse-transform
  // coefficients, inverse transforms (FP32 in mixed precision), loop harmonics
  auto up = [](int64_t n) { return (n + 31) / 32 * 32; };
  const bool mixed = mixed_of(ctx);
  const int64_t n_k = mixed ? (ctx->ws_total_k + 1) / 2 : ctx->ws_total_k;
  const int64_t parts[6] = {2 * ctx->S, ctx->ws_total_xp, ctx->ws_total_yb, ctx->ws_total_g2, n_k, ctx->ghat_len};
  int64_t off[6], need = 0;
  for (int i = 0; i < 6; ++i) {
    off[i] = need;
    need += up(std::max<int64_t>(parts[i], 1));
  }
  const int64_t cap = (int64_t)(kScratchBytes / sizeof(double));
  if (need > cap)
    return fail(ctx, TUFRG_EINVAL, "workspace of " + std::to_string(need * 8) + " bytes exceeds the " +
                                       std::to_string(kScratchBytes) + "-byte static scratch");
  double* base = static_cast<double*>(ctx->scratch);
  Launch L = ctx->L;
  L.b.dchi = base + off[0];
  L.b.xp = base + off[1];
  L.b.yb = base + off[2];
  L.b.g2 = base + off[3];
  if (mixed) {
    L.b.kinv = reinterpret_cast<float*>(base + off[4]);
    L.b.kinv64 = nullptr;
  } else {
    L.b.kinv = nullptr;
    L.b.kinv64 = base + off[4];
  }
  L.b.ghat = base + off[5];
  rhs_launch(ctx, L, ctx->all, X, dXdT, false, ctx->stream, TSource{T_host, 0, (int)ctx->dev.size(), 0});
  HIP_TRY(ctx, hipGetLastError());
  return TUFRG_OK;
}

tufrg_status tufrg_harmonics(const tufrg_ctx* ctx, int32_t point, int32_t* n, int32_t* table,
                             int64_t* offset) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (point < 0 || point >= (int)ctx->dev.size())
    return fail(const_cast<tufrg_ctx*>(ctx), TUFRG_EINVAL, "point out of range");
  const HostTables& t = ctx->host[point];
  if (n) *n = t.nsh;
  if (offset) *offset = ctx->dev[point].gh_off;
  if (table)
    for (int j = 0; j < t.nsh; ++j) {
      table[6 * j + 0] = t.hx[j];
      table[6 * j + 1] = t.hy[j];
      for (int k = 0; k < 4; ++k) table[6 * j + 2 + k] = t.pairs[4 * j + k];
    }
  return TUFRG_OK;
}

tufrg_status tufrg_loop_harmonics(tufrg_ctx* ctx, const double* T_host, double* ghat) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (!T_host || !ghat) return fail(ctx, TUFRG_EINVAL, "NULL argument");
  if (mixed_of(ctx)) return fail(ctx, TUFRG_EUNSUPPORTED, "loop harmonics are computed in FP64 contexts");
  ST_TRY(check_temperatures(ctx, T_host));
  launch_set_T_values(ctx->Tp, T_host, (int)ctx->dev.size(), ctx->stream);
  const Launch& L = ctx->L;
  launch_loops(L, ctx->all.loop, ctx->queue, false, ctx->stream);
  for (size_t p = 0; p < ctx->dev.size(); ++p) launch_ghat_sum(L, (int)p, ctx->dev[p], ghat, ctx->stream);
  HIP_TRY(ctx, hipGetLastError());
  return TUFRG_OK;
}

tufrg_status tufrg_surrogate_dataset(tufrg_ctx* ctx, const double* T_host, int64_t n, uint64_t seed,
                                     float* x, float* y, int32_t* idx) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (!T_host || !x || !y) return fail(ctx, TUFRG_EINVAL, "NULL argument");
  if (n < 0) return fail(ctx, TUFRG_EINVAL, "n must be >= 0");
  if (mixed_of(ctx)) return fail(ctx, TUFRG_EUNSUPPORTED, "training labels come from FP64 contexts");
  if (omega_of(ctx)) return fail(ctx, TUFRG_EUNSUPPORTED, "the surrogate serves the temperature flow");
  for (const HostTables& t : ctx->host)
    if (t.mesh) return fail(ctx, TUFRG_EUNSUPPORTED, "the surrogate serves the uniform transfer grid");
  ST_TRY(check_temperatures(ctx, T_host));
  launch_set_T_values(ctx->Tp, T_host, (int)ctx->dev.size(), ctx->stream);
  const Launch& L = ctx->L;
  launch_loops(L, ctx->all.loop, ctx->queue, false, ctx->stream);
  launch_sur_dataset(L, (int)ctx->dev.size(), n, seed, x, y, idx, ctx->stream);
  HIP_TRY(ctx, hipGetLastError());
  return TUFRG_OK;
}

tufrg_status tufrg_surrogate_attach(tufrg_ctx* ctx, tufrg_mlp* a, tufrg_mlp* b, double tol,
                                    int32_t check_stride) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->side));
  for (void* p : ctx->sur_allocations) (void)hipFree(p);
  ctx->sur_allocations.clear();
  ctx->sur_a = ctx->sur_b = nullptr;
  if (!a && !b) return TUFRG_OK;
  if (!a) return fail(ctx, TUFRG_EINVAL, "attach network a (b optional), or none to detach");
  if (ctx->dev.size() != 1) return fail(ctx, TUFRG_EUNSUPPORTED, "the surrogate serves single-point contexts");
  if (mixed_of(ctx)) return fail(ctx, TUFRG_EUNSUPPORTED, "the surrogate serves FP64 contexts");
  if (omega_of(ctx)) return fail(ctx, TUFRG_EUNSUPPORTED, "the surrogate serves the temperature flow");
  if (ctx->host[0].mesh) return fail(ctx, TUFRG_EUNSUPPORTED, "the surrogate serves the uniform transfer grid");
  for (tufrg_mlp* m : {a, b})
    if (m && (mlp_width(m, 0) != 9 || mlp_width(m, -1) != 4))
      return fail(ctx, TUFRG_EINVAL, "surrogate networks map 9 features to 4 targets");
  if (!(tol > 0.0) || check_stride < 1) return fail(ctx, TUFRG_EINVAL, "need tol > 0 and check_stride >= 1");
  const DevTables& d = ctx->dev[0];
  const size_t rows = (size_t)d.nirr * d.nsh, nh = (size_t)d.nirr * 2 * d.nsh;
  std::vector<void*>& g = ctx->sur_allocations;
  SurState& st = ctx->sur;
  st = SurState();
  st.tol = tol;
  st.stride = check_stride;
  ST_TRY(dalloc(ctx, rows * 9, &ctx->sur_x, g));
  ST_TRY(dalloc(ctx, rows * 4, &ctx->sur_ya, g));
  if (b) ST_TRY(dalloc(ctx, rows * 4, &ctx->sur_yb, g));
  ST_TRY(dalloc(ctx, 1, &st.phase, g));
  ST_TRY(dalloc(ctx, (size_t)d.nirr, &st.state, g));
  ST_TRY(dalloc(ctx, (size_t)d.nirr, &st.need, g));
  ST_TRY(dalloc(ctx, (size_t)d.nirr, &st.fail, g));
  ST_TRY(dalloc(ctx, nh, &st.pred, g));
  ST_TRY(dalloc(ctx, nh, &st.fin, g));
  ST_TRY(dalloc(ctx, (size_t)d.nirr * d.nsplit, &st.items, g));
  ST_TRY(dalloc(ctx, 1, &st.count, g));
  ST_TRY(dalloc(ctx, 3, &st.stats, g));
  launch_fill_i32(st.phase, 1, 0, ctx->stream);
  launch_fill_i32(st.state, d.nirr, 0, ctx->stream);
  launch_fill_u64(st.stats, 3, 0ull, ctx->stream);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  ctx->sur_a = a;
  ctx->sur_b = b;
  return TUFRG_OK;
}

tufrg_status tufrg_surrogate_stats(tufrg_ctx* ctx, int64_t out[3]) {
  if (!ctx || !out) return fail(ctx, TUFRG_EINVAL, "NULL argument");
  if (!ctx->sur_a) return fail(ctx, TUFRG_EINVAL, "no surrogate attached");
  unsigned long long v[3];
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  HIP_TRY(ctx, hipMemcpy(v, ctx->sur.stats, sizeof v, hipMemcpyDeviceToHost));
  for (int i = 0; i < 3; ++i) out[i] = (int64_t)v[i];
  return TUFRG_OK;
}

tufrg_status tufrg_loop_kernel_time(tufrg_ctx* ctx, const double* T_host, int32_t reps, double* us,
                                    double* flops) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (!T_host || !us || reps < 1) return fail(ctx, TUFRG_EINVAL, "need T_host, us and reps >= 1");
  ST_TRY(check_temperatures(ctx, T_host));
  launch_set_T_values(ctx->Tp, T_host, (int)ctx->dev.size(), ctx->stream);
  const bool mixed = mixed_of(ctx);
  launch_loops(ctx->L, ctx->all.loop, ctx->queue, mixed, ctx->stream);   // warm-up
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  hipError_t e = hipEventRecord(e0, ctx->stream);
  for (int i = 0; i < reps && e == hipSuccess; ++i) launch_loops(ctx->L, ctx->all.loop, ctx->queue, mixed, ctx->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(ctx, TUFRG_EHIP, std::string("loop kernel timing: ") + hipGetErrorString(e));
  *us = 1e3 * (double)ms / reps;
  if (flops) {
    *flops = 0.0;
    for (const HostTables& t : ctx->host) *flops += (double)t.flops_loop_kernel;
  }
  return TUFRG_OK;
}

tufrg_status tufrg_kernel_times(tufrg_ctx* ctx, const double* T_host, const double* X, double* dXdT,
                                int32_t reps, double us[5], double flops[5]) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (!T_host || !X || !dXdT || !us || reps < 1) return fail(ctx, TUFRG_EINVAL, "need T_host, X, dXdT, us and reps >= 1");
  if (X == dXdT) return fail(ctx, TUFRG_EINVAL, "X and dXdT must not alias");
  if (ctx->sur_a) return fail(ctx, TUFRG_EUNSUPPORTED, "kernel timing is not available with a surrogate attached");
  if (ctx->L.dense || !cross_of(ctx))
    return fail(ctx, TUFRG_EUNSUPPORTED, "kernel timing needs the factored projections (no dense operator, no NO_CROSS)");
  ST_TRY(check_temperatures(ctx, T_host));
  hipStream_t s = ctx->stream;
  const bool mixed = mixed_of(ctx);
  const Launch& L = ctx->L;
  const Ranges& r = ctx->all;
  // one right-hand side leaves every stage's input in the workspace
  rhs_launch(ctx, L, r, X, dXdT, false, s, TSource{T_host, 0, (int)ctx->dev.size(), 0});
  HIP_TRY(ctx, hipGetLastError());
  // each stage's reps launches are captured in a HIP graph on the context's
  // capture stream (ordered after the caller's) and replayed, so that the
  // time is the GPU's (kernels and the gaps between them), not the host's
  // launch rate
  hipStream_t gs = ctx->gs;
  HIP_TRY(ctx, hipEventRecord(ctx->ev_gs, s));
  HIP_TRY(ctx, hipStreamWaitEvent(gs, ctx->ev_gs, 0));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(ctx, hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  for (int i = 0; i < 5 && e == hipSuccess; ++i) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    e = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      for (int k = 0; k < reps; ++k) {
        switch (i) {
          case 0: launch_fwd(L, r, X, mixed, gs); break;
          case 1: launch_basis(L, r, gs); break;
          case 2: launch_gather(L, r, gs); break;
          case 3: launch_inv(L, r, mixed, gs); break;
          default: launch_back(L, r, X, dXdT, 1, true, false, mixed, gs); break;
        }
      }
      e = hipStreamEndCapture(gs, &graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(exec, gs);   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, gs);
    if (e == hipSuccess) e = hipGraphLaunch(exec, gs);
    if (e == hipSuccess) e = hipEventRecord(e1, gs);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    us[i] = 1e3 * (double)ms / reps;
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
  if (e1) (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e0);
  if (e != hipSuccess) return fail(ctx, TUFRG_EHIP, std::string("kernel timing: ") + hipGetErrorString(e));
  HIP_TRY(ctx, hipGetLastError());
  if (flops) {
    for (int i = 0; i < 5; ++i) flops[i] = 0.0;
    const bool wedge = L.b.wedge != 0;
    for (const HostTables& t : ctx->host) {
      // with symmetric states the inverse transform and the products run at
      // the orbit representatives only
      const double rows = wedge ? (double)t.nirr / t.nq : 1.0;
      flops[0] += (double)t.flops_fwd;
      flops[1] += (double)t.flops_basis;
      flops[2] += (double)t.flops_gather;
      flops[3] += (double)t.flops_inv * rows;
      flops[4] += (double)t.flops_prod * rows;
    }
  }
  return TUFRG_OK;
}

tufrg_status tufrg_symmetry_defect(tufrg_ctx* ctx, const double* X, double* rel) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (!X || !rel) return fail(ctx, TUFRG_EINVAL, "NULL argument");
  return symmetry_defect(ctx, X, rel);
}

tufrg_status tufrg_sync(tufrg_ctx* ctx) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  HIP_TRY(ctx, hipGetLastError());
  return TUFRG_OK;
}

tufrg_status tufrg_flop_count(const tufrg_ctx* ctx, double out[3]) {
  if (!ctx || !out) return fail(nullptr, TUFRG_EINVAL, "NULL argument");
  out[0] = out[1] = out[2] = 0.0;
  for (const HostTables& t : ctx->host) {
    out[0] += (double)t.flops_loops;
    out[1] += (double)t.flops_proj;
    out[2] += (double)t.flops_prod;
  }
  return TUFRG_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ flow
namespace {

// Cyclic Jacobi eigenvalue iteration for a small real symmetric matrix.
void jacobi_eig(std::vector<double> a, int n, std::vector<double>& w, std::vector<double>& v) {
  v.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += a[(size_t)i * n + j] * a[(size_t)i * n + j];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = a[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
          a[(size_t)k * n + p] = c * akp - s * akq;
          a[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
          a[(size_t)p * n + k] = c * apk - s * aqk;
          a[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
          v[(size_t)k * n + p] = c * vkp - s * vkq;
          v[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
}

// irrep of the leading eigenvector of the form-factor matrix src = X(ch, q)
// that holds the largest |X_mn(q)| (channel and momentum found on the device)
void classify(const HostTables& t, int ch, int q, const double* src /*[nff][nff]*/, tufrg_flow_result* r) {
  const int nff = t.nff, nff2 = nff * nff;
  std::vector<double> m((size_t)nff2);
  for (int i = 0; i < nff; ++i)
    for (int j = 0; j < nff; ++j) m[(size_t)i * nff + j] = 0.5 * (src[i * nff + j] + src[j * nff + i]);
  std::vector<double> w, v;
  jacobi_eig(m, nff, w, v);
  int lead = 0;
  for (int i = 1; i < nff; ++i)
    if (std::fabs(w[i]) > std::fabs(w[lead])) lead = i;
  double weight[5] = {0, 0, 0, 0, 0};
  for (int k = 0; k < nff; ++k) weight[t.irrep[k]] += v[(size_t)k * nff + lead] * v[(size_t)k * nff + lead];
  int ir = 0;
  for (int i = 1; i < 5; ++i)
    if (weight[i] > weight[ir]) ir = i;
  r->channel = ch;
  r->q_index = q;
  r->irrep = ir;
}

double interp_tc(double s0, double s1, double m0, double m1, double xmax) {
  if (!(m0 > 0.0)) return std::exp(s1);
  double sc = s0 + (std::log(xmax) - std::log(m0)) * (s1 - s0) / (std::log(m1) - std::log(m0));
  return std::exp(sc);
}

// Result of point p: status, counters, and for a divergence Tc by log-linear
// interpolation between the last two accepted steps (s0, m0) -> (s1, m1) and
// the classification of the stopped state X.
tufrg_status finish_point(tufrg_ctx* ctx, int p, const double* X, int status, double s0, double s1,
                          double m0, double m1, double xmax, int64_t n_rhs, int64_t n_steps, int first,
                          hipStream_t ms, tufrg_flow_result* r) {
  std::memset(r, 0, sizeof *r);
  r->status = status;
  r->n_rhs = n_rhs;
  r->n_steps = n_steps;
  r->max_abs_X = m1;
  r->channel = r->q_index = r->irrep = -1;
  r->Tc = 0.0;
  if (status == TUFRG_FLOW_DIVERGED) {
    r->Tc = interp_tc(s0, s1, m0, m1, xmax);
    const HostTables& t = ctx->host[p];
    const int nff2 = t.nff * t.nff;
    if (first < 0 || first >= 3 * t.nq * nff2) return TUFRG_OK;   // no finite maximum: unclassified
    const int ch = first / (t.nq * nff2), q = (first / nff2) % t.nq;
    std::vector<double> m((size_t)nff2);
    HIP_TRY(ctx, hipMemcpyAsync(m.data(), X + ch * ctx->S + ctx->off[p] + (size_t)q * nff2, nff2 * sizeof(double),
                                hipMemcpyDeviceToHost, ms));
    HIP_TRY(ctx, hipStreamSynchronize(ms));
    classify(t, ch, q, m.data(), r);
  }
  return TUFRG_OK;
}

// Per point, the first flat index (channel, q, m, n) of the largest |X| of
// the stopped state, on the device (the classification then copies one
// form-factor matrix per diverged point instead of the state)
tufrg_status locate_maxima(tufrg_ctx* ctx, const double* X, hipStream_t ms, std::vector<int>& first) {
  const int npts = (int)ctx->dev.size();
  launch_fill_u64(ctx->umax, npts, 0ull, ms);
  launch_maxabs(ctx->L, ctx->all.seg, X, ctx->umax, ms);
  launch_fill_i32(ctx->first_max, npts, INT_MAX, ms);
  launch_first_max(ctx->L, ctx->all.seg, X, ctx->umax, ctx->first_max, ms);
  first.assign(npts, INT_MAX);
  HIP_TRY(ctx, hipMemcpyAsync(first.data(), ctx->first_max, sizeof(int) * npts, hipMemcpyDeviceToHost, ms));
  HIP_TRY(ctx, hipStreamSynchronize(ms));
  return TUFRG_OK;
}

// One RK4 step of every point still flowing, in s = ln T: stage temperatures
// from the device table at the device step counter, slopes dX/ds, the update
// (stopped points untouched), per-point max|X| and the device-side stop test.
// The third stage takes the second's loops (same temperature); with
// reuse_first (every step after a flow's first) the first stage takes the
// loops of the step before's last stage, whose table temperature exp(s0 +
// (i + 1) h) is bit for bit the first stage's of step i + 1.
void rk4_step(tufrg_ctx* ctx, const Launch& L, double* X, double h, double xmax, int nsteps,
              hipStream_t ms, bool reuse_first) {
  double* const* k = ctx->kk;
  const int npts = (int)ctx->dev.size();
  const double half[1] = {0.5}, one[1] = {1.0};
  const double fin[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
  const Ranges& r = ctx->all;
  auto stage_T = [](int stage) { return TSource{nullptr, 0, 0, stage}; };
  if (!L.fused) {
    // large contexts: the stage combinations as streaming kernels of their own
    rhs_launch(ctx, L, r, X, k[0], true, ms, stage_T(0), nullptr, reuse_first);
    launch_axpy(L, r.seg, X, &k[0], half, 1, h, ctx->stage, true, ms);
    rhs_launch(ctx, L, r, ctx->stage, k[1], true, ms, stage_T(1));
    launch_axpy(L, r.seg, X, &k[1], half, 1, h, ctx->stage, true, ms);
    rhs_launch(ctx, L, r, ctx->stage, k[2], true, ms, stage_T(2), nullptr, true);
    launch_axpy(L, r.seg, X, &k[2], one, 1, h, ctx->stage, true, ms);
    rhs_launch(ctx, L, r, ctx->stage, k[3], true, ms, stage_T(3));
    launch_axpy(L, r.seg, X, k, fin, 4, h, X, true, ms);
    launch_maxabs(L, r.seg, X, ctx->umax, ms);
    launch_step_end(ctx->umax, npts, ctx->frozen, ctx->hist, ctx->step, nsteps, xmax, ms, ctx->flow_status_dev);
    return;
  }
  // small (launch-bound) contexts: each stage combination is formed by the
  // products of the slope before it (X + h/2 k1, X + h/2 k2, X + h k3 in
  // alternating buffers, then the update of X in place)
  auto next = [&](double* dst, const double* coef, int nk, double* const* ks) {
    StageNext sn{};
    sn.X = X;
    for (int j = 0; j < nk; ++j) {
      sn.k[j] = ks[j];
      sn.coef[j] = coef[j];
    }
    sn.out = dst;
    sn.h = h;
    sn.nk = nk;
    return sn;
  };
  double* st[2] = {ctx->stage, ctx->stage2};
  const StageNext n1 = next(st[0], half, 1, &k[0]), n2 = next(st[1], half, 1, &k[1]);
  const StageNext n3 = next(st[0], one, 1, &k[2]), n4 = next(X, fin, 4, k);
  rhs_launch(ctx, L, r, X, k[0], true, ms, stage_T(0), &n1, reuse_first);
  rhs_launch(ctx, L, r, st[0], k[1], true, ms, stage_T(1), &n2);
  rhs_launch(ctx, L, r, st[1], k[2], true, ms, stage_T(2), &n3, true);
  rhs_launch(ctx, L, r, st[0], k[3], true, ms, stage_T(3), &n4);
  launch_maxabs(L, r.seg, X, ctx->umax, ms);
  launch_step_end(ctx->umax, npts, ctx->frozen, ctx->hist, ctx->step, nsteps, xmax, ms, ctx->flow_status_dev);
}

tufrg_status flow_rk4_all(tufrg_ctx* ctx, const tufrg_flow_opts* o, double* X, tufrg_flow_result* res) {
  const int npts = (int)ctx->dev.size();
  const int nsteps = o->nsteps;
  const double s0 = std::log(o->T0);
  const double h = (std::log(o->Tmin) - s0) / nsteps;
  // stage temperatures of every step (one spare row read by nothing) and the
  // max|X| history
  if (ctx->ttab_cap < nsteps) {
    ST_TRY(dalloc(ctx, (size_t)4 * (nsteps + 1), &ctx->Ttab, ctx->allocations));
    ST_TRY(dalloc(ctx, (size_t)(nsteps + 2) * npts, &ctx->hist, ctx->allocations));
    ctx->ttab_cap = nsteps;
  }
  std::vector<double> tt((size_t)4 * (nsteps + 1), 0.0);
  for (int i = 0; i < nsteps; ++i) {
    const double s = s0 + i * h;
    tt[4 * i + 0] = std::exp(s);
    tt[4 * i + 1] = std::exp(s + 0.5 * h);
    tt[4 * i + 2] = std::exp(s + 0.5 * h);
    tt[4 * i + 3] = std::exp(s0 + (i + 1) * h);
  }
  for (int j = 0; j < 4; ++j) tt[4 * nsteps + j] = tt[4 * (nsteps - 1) + 3];
  // graph replay runs on the context's own capture stream, ordered after the
  // caller's stream
  hipStream_t ms = ctx->stream;
  if (o->use_graph) {
    ms = ctx->gs;
    HIP_TRY(ctx, hipEventRecord(ctx->ev_gs, ctx->stream));
    HIP_TRY(ctx, hipStreamWaitEvent(ms, ctx->ev_gs, 0));
  }
  HIP_TRY(ctx, hipMemcpyAsync(ctx->Ttab, tt.data(), tt.size() * sizeof(double), hipMemcpyHostToDevice, ms));
  launch_fill_i32(ctx->frozen, npts, 0, ms);
  launch_fill_i32(ctx->step, 1, 0, ms);
  launch_fill_u64(ctx->umax, npts, 0ull, ms);
  ST_TRY(ensure_status_words(ctx));
  for (int p = 0; p < npts; ++p) ctx->flow_status_host[p] = 0;
  Launch Lf = ctx->L;
  Lf.b.frozen = ctx->frozen;
  launch_maxabs(Lf, ctx->all.seg, X, ctx->umax, ms);
  HIP_TRY(ctx, hipMemcpyAsync(ctx->umax_host, ctx->umax, sizeof(unsigned long long) * npts,
                              hipMemcpyDeviceToHost, ms));
  launch_fill_u64(ctx->umax, npts, 0ull, ms);
  HIP_TRY(ctx, hipStreamSynchronize(ms));
  std::vector<double> m0(npts);
  for (int p = 0; p < npts; ++p) m0[p] = word_to_double(ctx->umax_host[p]);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto cleanup = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  };
  // the graph holds a step after the first (its first stage takes the loops
  // of the step before); the first step is issued directly
  if (o->use_graph) {
    HIP_TRY(ctx, hipStreamBeginCapture(ms, hipStreamCaptureModeThreadLocal));
    rk4_step(ctx, Lf, X, h, o->Xmax, nsteps, ms, true);
    hipError_t e = hipStreamEndCapture(ms, &graph);
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      cleanup();
      return fail(ctx, TUFRG_EHIP, std::string("graph capture of the RK4 step: ") + hipGetErrorString(e));
    }
  }
  // steps are issued one ahead of the host's view (as the adaptive flow's
  // attempts): after issuing step n the host waits for step n - 1 and reads
  // the points' stop words, which the step-end kernel writes into mapped host
  // memory; once every point has stopped, the one step issued after that
  // runs as a no-op
  int done = 0;
  auto issue = [&]() -> hipError_t {
    if (exec && done > 0) {
      const hipError_t e = hipGraphLaunch(exec, ms);
      if (e != hipSuccess) return e;
    } else {
      rk4_step(ctx, Lf, X, h, o->Xmax, nsteps, ms, done > 0);
    }
    return hipEventRecord(ctx->ev_att[done++ & 1], ms);
  };
  hipError_t e = issue();
  while (e == hipSuccess) {
    const bool more = done < nsteps;
    if (more) e = issue();
    if (e != hipSuccess) break;
    e = hipEventSynchronize(ctx->ev_att[(done - (more ? 2 : 1)) & 1]);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) break;
    bool all_done = true;
    const volatile int* hs = ctx->flow_status_host;
    for (int p = 0; p < npts && all_done; ++p) all_done = hs[p] != 0;
    if (all_done || !more) break;
  }
  std::vector<int> frozen(npts, 0);
  if (e == hipSuccess)
    e = hipMemcpyAsync(frozen.data(), ctx->frozen, sizeof(int) * npts, hipMemcpyDeviceToHost, ms);
  if (e == hipSuccess) e = hipStreamSynchronize(ms);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    cleanup();
    return fail(ctx, TUFRG_EHIP, std::string("RK4 flow: ") + hipGetErrorString(e));
  }
  cleanup();
  std::vector<double> hist((size_t)(done + 1) * npts);
  HIP_TRY(ctx, hipMemcpyAsync(hist.data(), ctx->hist, hist.size() * sizeof(double), hipMemcpyDeviceToHost, ms));
  HIP_TRY(ctx, hipStreamSynchronize(ms));
  for (int p = 0; p < npts; ++p) hist[p] = m0[p];
  std::vector<int> first;
  ST_TRY(locate_maxima(ctx, X, ms, first));
  for (int p = 0; p < npts; ++p) {
    const int f = frozen[p];
    const int last = f ? f : done;
    const double mlast = hist[(size_t)last * npts + p];
    const double mprev = hist[(size_t)(last - 1) * npts + p];
    int status = TUFRG_FLOW_REACHED_TMIN;
    if (f) status = std::isfinite(mlast) ? TUFRG_FLOW_DIVERGED : TUFRG_FLOW_NONFINITE;
    ST_TRY(finish_point(ctx, p, X, status, s0 + (last - 1) * h, s0 + last * h, mprev, mlast, o->Xmax,
                        4 * (int64_t)last, last, first[p], ms, &res[p]));
  }
  return TUFRG_OK;
}

// Dormand-Prince 5(4) tableau (Dormand & Prince 1980)
const double kDpC[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
const double kDpA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84},
};
const double kDpB5[7] = {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0.0};
const double kDpB4[7] = {5179.0 / 57600, 0.0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200,
                         187.0 / 2100, 1.0 / 40};

// The adaptive flow of every point at once, with the step control on the
// device (Dormand-Prince 5(4) in s = ln T, the rules of the flow options, the
// oracle's): one attempted step of all points is six stage combinations and
// right-hand sides, the fifth-order state with the error norm's partial sums
// and max|y5|, the control kernel (accept or reject, next step, stop) and the
// acceptance copy (y = y5, k0 = k6).  Each point has its own s and h in device
// memory; the kernels read them, so the attempt can be captured in a HIP
// graph and replayed.  A point that has stopped is skipped by every kernel.
// The host follows the points' status words one attempt behind the stream.
tufrg_status flow_dopri5_all(tufrg_ctx* ctx, const tufrg_flow_opts* o, double* X, tufrg_flow_result* res) {
  const int npts = (int)ctx->dev.size();
  double* k[7];
  for (int i = 0; i < 7; ++i) k[i] = ctx->kk[i];
  double* y5 = ctx->ytmp;
  const Ranges& r = ctx->all;
  if (ctx->nred < r.seg.n) {
    ST_TRY(dalloc(ctx, (size_t)r.seg.n, &ctx->red, ctx->allocations));
    ctx->nred = r.seg.n;
  }
  if (!ctx->dp_state) {
    ST_TRY(dalloc(ctx, (size_t)npts, &ctx->dp_state, ctx->allocations));
    ST_TRY(dalloc(ctx, (size_t)2 * npts, &ctx->dp_sh, ctx->allocations));
    std::vector<int2> seg(npts);
    std::vector<double> nel(npts);
    for (int p = 0; p < npts; ++p) {
      seg[p] = make_int2(ctx->per_point[p].seg.begin, ctx->per_point[p].seg.n);
      nel[p] = 3.0 * (double)ctx->host[p].nq * ctx->host[p].nff * ctx->host[p].nff;
    }
    ST_TRY(upload(ctx, seg, &ctx->dp_seg, ctx->allocations));
    ST_TRY(upload(ctx, nel, &ctx->dp_nel, ctx->allocations));
  }
  ST_TRY(ensure_status_words(ctx));
  const double s0 = std::log(o->T0), s_end = std::log(o->Tmin);
  const double h0 = (o->h0 != 0.0) ? o->h0 : (s_end - s0) / 200.0;
  const int max_steps = o->max_steps > 0 ? o->max_steps : 100000;
  hipStream_t ms = ctx->stream;
  if (o->use_graph) {
    ms = ctx->gs;
    HIP_TRY(ctx, hipEventRecord(ctx->ev_gs, ctx->stream));
    HIP_TRY(ctx, hipStreamWaitEvent(ms, ctx->ev_gs, 0));
  }
  // initial state: max|X| of every point, s, h (clipped) and the first slope
  launch_fill_i32(ctx->frozen, npts, 0, ms);
  launch_fill_u64(ctx->umax, npts, 0ull, ms);
  launch_maxabs(ctx->L, r.seg, X, ctx->umax, ms);
  std::vector<unsigned long long> mw(npts);
  HIP_TRY(ctx, hipMemcpyAsync(mw.data(), ctx->umax, sizeof(unsigned long long) * npts, hipMemcpyDeviceToHost, ms));
  launch_fill_u64(ctx->umax, npts, 0ull, ms);
  HIP_TRY(ctx, hipStreamSynchronize(ms));
  std::vector<DpState> st0(npts);
  std::vector<double> sh(2 * (size_t)npts);
  for (int p = 0; p < npts; ++p) {
    DpState& q = st0[p];
    std::memset(&q, 0, sizeof q);
    q.s = s0;
    q.h = (s0 + h0 < s_end) ? s_end - s0 : h0;
    q.s0 = q.s1 = s0;
    q.m0 = q.m1 = word_to_double(mw[p]);
    sh[p] = q.s;
    sh[npts + p] = q.h;
  }
  HIP_TRY(ctx, hipMemcpyAsync(ctx->dp_state, st0.data(), sizeof(DpState) * npts, hipMemcpyHostToDevice, ms));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->dp_sh, sh.data(), sizeof(double) * 2 * npts, hipMemcpyHostToDevice, ms));
  double* s_arr = ctx->dp_sh;
  double* h_arr = ctx->dp_sh + npts;
  Launch Lf = ctx->L;
  Lf.b.frozen = ctx->frozen;
  auto stage_T = [&](double c) {
    TSource ts{nullptr, 0, 0, 0};
    ts.s = s_arr;
    ts.h = h_arr;
    ts.c = c;
    return ts;
  };
  rhs_launch(ctx, Lf, r, X, k[0], true, ms, stage_T(0.0));
  // stage i of an attempt lives in stg[i & 1]; the acceptance kernel forms
  // stage 1 of the next attempt, and in small (launch-bound) contexts the
  // products of stage i form stage i + 1 (i < 6), in large ones streaming
  // stage kernels of their own
  double* stg[2] = {ctx->stage, ctx->stage2};
  const bool fuse_stages = Lf.fused;
  launch_axpy(Lf, r.seg, X, k, kDpA[1], 1, 0.0, stg[1], true, ms, h_arr);
  double e[7];
  for (int j = 0; j < 7; ++j) e[j] = kDpB5[j] - kDpB4[j];
  DpControl dc{};
  dc.st = ctx->dp_state;
  dc.frozen = ctx->frozen;
  dc.seg = ctx->dp_seg;
  dc.n_el = ctx->dp_nel;
  dc.red = ctx->red;
  dc.max_words = ctx->umax;
  dc.s_arr = s_arr;
  dc.h_arr = h_arr;
  dc.s_end = s_end;
  dc.xmax = o->Xmax;
  dc.max_steps = max_steps;
  dc.npts = npts;
  dc.status_out = ctx->flow_status_dev;
  for (int p = 0; p < npts; ++p) ctx->flow_status_host[p] = 0;
  auto attempt = [&]() {
    for (int i = 1; i < 7; ++i) {
      if (i > 1 && !fuse_stages) launch_axpy(Lf, r.seg, X, k, kDpA[i], i, 0.0, stg[i & 1], true, ms, h_arr);
      StageNext sn{};
      if (i < 6 && fuse_stages) {
        sn.X = X;
        for (int j = 0; j <= i; ++j) {
          sn.k[j] = k[j];
          sn.coef[j] = kDpA[i + 1][j];
        }
        sn.out = stg[(i + 1) & 1];
        sn.hp = h_arr;
        sn.nk = i + 1;
      }
      rhs_launch(ctx, Lf, r, stg[i & 1], k[i], true, ms, stage_T(kDpC[i]), sn.nk > 0 ? &sn : nullptr,
                 kDpC[i] == kDpC[i - 1]);
    }
    launch_dp_final(Lf, r.seg, X, k, kDpB5, e, 0.0, o->rtol, o->atol, y5, ctx->red, ctx->umax, ms, h_arr);
    launch_dp_control(dc, ms);
    launch_dp_accept(Lf, r.seg, ctx->dp_state, y5, k[6], X, k[0], kDpA[1][0], h_arr, stg[1], ms);
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto cleanup = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  };
  if (o->use_graph) {
    HIP_TRY(ctx, hipStreamBeginCapture(ms, hipStreamCaptureModeThreadLocal));
    attempt();
    hipError_t ge = hipStreamEndCapture(ms, &graph);
    if (ge == hipSuccess) ge = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ge != hipSuccess) {
      cleanup();
      return fail(ctx, TUFRG_EHIP, std::string("graph capture of the adaptive step: ") + hipGetErrorString(ge));
    }
  }
  // attempts are issued one ahead of the host's view: after issuing attempt n
  // the host waits for attempt n - 1 and reads the points' status words (the
  // control kernel writes them to mapped host memory), so the stream always
  // holds the next attempt and never drains mid-flow; once every point has
  // stopped, the one attempt issued after that runs as a no-op (its kernels
  // skip stopped points).  max_steps bounds the attempts of every point on
  // the device; the count here is only a backstop.
  int attempted = 0;
  auto issue = [&]() -> hipError_t {
    if (exec) {
      const hipError_t ge = hipGraphLaunch(exec, ms);
      if (ge != hipSuccess) return ge;
    } else {
      attempt();
    }
    return hipEventRecord(ctx->ev_att[attempted++ & 1], ms);
  };
  hipError_t ge = issue();
  while (ge == hipSuccess) {
    const bool more = attempted <= max_steps;
    if (more) ge = issue();
    if (ge != hipSuccess) break;
    ge = hipEventSynchronize(ctx->ev_att[(attempted - (more ? 2 : 1)) & 1]);
    if (ge == hipSuccess) ge = hipGetLastError();
    if (ge != hipSuccess) break;
    bool all_done = true;
    const volatile int* hs = ctx->flow_status_host;
    for (int p = 0; p < npts && all_done; ++p) all_done = hs[p] != 0;
    if (all_done || !more) break;
  }
  std::vector<DpState> stv(npts);
  if (ge == hipSuccess)
    ge = hipMemcpyAsync(stv.data(), ctx->dp_state, sizeof(DpState) * npts, hipMemcpyDeviceToHost, ms);
  if (ge == hipSuccess) ge = hipStreamSynchronize(ms);
  if (ge == hipSuccess) ge = hipGetLastError();
  if (ge != hipSuccess) {
    cleanup();
    return fail(ctx, TUFRG_EHIP, std::string("adaptive flow: ") + hipGetErrorString(ge));
  }
  cleanup();
  std::vector<int> first;
  ST_TRY(locate_maxima(ctx, X, ms, first));
  for (int p = 0; p < npts; ++p) {
    const DpState& q = stv[p];
    const int status = q.status != 0 ? q.status : TUFRG_FLOW_MAX_STEPS;
    ST_TRY(finish_point(ctx, p, X, status, q.s0, q.s1, q.m0, q.m1, o->Xmax, 1 + 6 * (int64_t)q.n_att, q.n_acc,
                        first[p], ms, &res[p]));
  }
  return TUFRG_OK;
}

}  // namespace

extern "C" {

tufrg_status tufrg_flow(tufrg_ctx* ctx, const tufrg_flow_opts* o, double* X, tufrg_flow_result* res) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (!o || !X || !res) return fail(ctx, TUFRG_EINVAL, "NULL argument");
  if (!(o->T0 > 0.0) || !(o->Tmin > 0.0) || !(o->Tmin < o->T0) || !(o->Xmax > 0.0))
    return fail(ctx, TUFRG_EINVAL, "need T0 > Tmin > 0 and Xmax > 0");
  if (o->scheme != TUFRG_RK4_LOG && o->scheme != TUFRG_DOPRI5_LOG)
    return fail(ctx, TUFRG_EINVAL, "unknown scheme");
  if (ctx->opt.flags & TUFRG_SYMMETRIC_STATE) {
    double rel = 0.0;
    ST_TRY(symmetry_defect(ctx, X, &rel));
    if (!(rel <= kSymmetryTol))
      return fail(ctx, TUFRG_EINVAL, "initial state is not C4v-symmetric (relative defect " + std::to_string(rel) +
                                         "); symmetric-state contexts need symmetric states");
  }
  ST_TRY(ensure_flow_buffers(ctx));
  if (o->scheme == TUFRG_RK4_LOG) {
    if (o->nsteps <= 0) return fail(ctx, TUFRG_EINVAL, "nsteps must be > 0");
    ST_TRY(flow_rk4_all(ctx, o, X, res));
  } else if (o->scheme == TUFRG_DOPRI5_LOG) {
    if (!(o->rtol > 0.0) || !(o->atol > 0.0)) return fail(ctx, TUFRG_EINVAL, "rtol, atol must be > 0");
    if (!(o->h0 <= 0.0)) return fail(ctx, TUFRG_EINVAL, "h0 must be 0 (default) or negative (towards Tmin)");
    if (o->max_steps < 0) return fail(ctx, TUFRG_EINVAL, "max_steps must be >= 0");
    ST_TRY(flow_dopri5_all(ctx, o, X, res));
  } else {
    return fail(ctx, TUFRG_EINVAL, "unknown scheme");
  }
  ST_TRY(flow_max_abs_V(ctx, X, res));
  for (size_t p = 0; p < ctx->dev.size(); ++p)
    if (res[p].status == TUFRG_FLOW_NONFINITE)
      return fail(ctx, TUFRG_ENONFINITE, "flow state of point " + std::to_string(p) + " became non-finite");
  return TUFRG_OK;
}

void tufrg_free(tufrg_ctx* ctx) {
  if (!ctx) return;
  if (!ctx->allocations.empty() || !ctx->geometry_allocations.empty() || !ctx->sur_allocations.empty())
    (void)hipDeviceSynchronize();
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  if (ctx->gs) (void)hipStreamDestroy(ctx->gs);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->ev_gs) (void)hipEventDestroy(ctx->ev_gs);
  for (hipEvent_t e : ctx->ev_att)
    if (e) (void)hipEventDestroy(e);
  if (ctx->umax_host) (void)hipHostFree(ctx->umax_host);
  if (ctx->flow_status_host) (void)hipHostFree(ctx->flow_status_host);
  if (ctx->red_host) (void)hipHostFree(ctx->red_host);
  for (void* p : ctx->sur_allocations) (void)hipFree(p);
  for (void* p : ctx->geometry_allocations) (void)hipFree(p);
  for (void* p : ctx->allocations) (void)hipFree(p);
  delete ctx;
}

const char* tufrg_last_error(const tufrg_ctx* ctx) {
  if (ctx) return ctx->err.c_str();
  return g_last_error.c_str();
}

}  // extern "C"
