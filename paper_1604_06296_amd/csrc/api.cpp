// C ABI of the TUfRG library: context, validation, workspace, step calls and
// the ODE flow driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "tufrg_internal.h"

using namespace tufrg;

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

template <class T>
tufrg_status upload(tufrg_ctx* ctx, const std::vector<T>& v, T** out) {
  *out = nullptr;
  size_t bytes = std::max<size_t>(sizeof(T), v.size() * sizeof(T));
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(ctx, TUFRG_ENOMEM, "hipMalloc failed (tables)");
  ctx->allocations.push_back(p);
  if (!v.empty()) HIP_TRY(ctx, hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  *out = static_cast<T*>(p);
  return TUFRG_OK;
}

tufrg_status dalloc(tufrg_ctx* ctx, size_t bytes, void** out) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(bytes, 8)) != hipSuccess)
    return fail(ctx, TUFRG_ENOMEM, "hipMalloc failed (workspace)");
  ctx->allocations.push_back(p);
  *out = p;
  return TUFRG_OK;
}

#define ST_TRY(expr)                      \
  do {                                    \
    tufrg_status s_ = (expr);             \
    if (s_ != TUFRG_OK) return s_;        \
  } while (0)

// One right-hand side of point p: out = scale * dX/dT at temperature T.
// The loops depend on T only and run on the side stream, concurrently with
// the X-dependent front end of the projections on the main stream; the back
// end (inverse transform, V, products) joins both.
void rhs_point(tufrg_ctx* ctx, int p, double T, const double* X, double* out, double scale) {
  const DevTables& d = ctx->dev[p];
  const int64_t off = ctx->off[p];
  if (ctx->opt.precision == TUFRG_MIXED) {
    hipEventRecord(ctx->ev_fork, ctx->stream);
    hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0);
    launch_loops_mixed(d, T, ctx->ws.dchi + off, ctx->S, ctx->ws.dpart, false, ctx->side);
    hipEventRecord(ctx->ev_join, ctx->side);
    launch_project_front_mixed(d, X + off, ctx->S, ctx->ws.xt, ctx->ws.yb, ctx->ws.g2,
                               ctx->opt.flags, ctx->stream);
    launch_inverse_mixed(d, ctx->ws.g2, ctx->ws.kinv, ctx->opt.flags, ctx->stream);
    hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0);
    launch_products_mixed(d, X + off, ctx->S, ctx->ws.kinv, ctx->ws.dchi + off, ctx->ws.dpart,
                          out + off, 1, ctx->opt.flags, scale, ctx->stream);
    return;
  }
  hipEventRecord(ctx->ev_fork, ctx->stream);
  hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0);
  launch_loops(d, T, ctx->ws.dchi + off, ctx->S, ctx->ws.dpart, false, ctx->side);
  hipEventRecord(ctx->ev_join, ctx->side);
  launch_project_front(d, X + off, ctx->S, ctx->ws.xt, ctx->ws.yb, ctx->ws.g2, ctx->opt.flags,
                       ctx->stream);
  hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0);
  launch_project_back(d, X + off, ctx->S, ctx->ws.g2, ctx->ws.dchi + off, ctx->ws.dpart, out + off,
                      1, ctx->opt.flags, scale, ctx->stream);
}

// ----------------------------------------------------- classification
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

// channel, momentum and irrep of the largest |X_mn(q)| (first in flat order)
void classify(const HostTables& t, const std::vector<double>& x /*[3][nq][nff][nff]*/,
              tufrg_flow_result* r) {
  const int nff = t.nff, nff2 = nff * nff;
  size_t best = 0;
  double bv = -1.0;
  for (size_t i = 0; i < x.size(); ++i)
    if (std::fabs(x[i]) > bv) { bv = std::fabs(x[i]); best = i; }
  const int ch = (int)(best / ((size_t)t.nq * nff2));
  const int q = (int)((best / nff2) % t.nq);
  std::vector<double> m((size_t)nff2);
  const double* src = x.data() + ((size_t)ch * t.nq + q) * nff2;
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

double word_to_double(unsigned long long w) {
  double d;
  std::memcpy(&d, &w, sizeof d);
  return d;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

tufrg_status tufrg_init(const tufrg_point* pts, int32_t npts, const tufrg_options* opt, void* stream,
                        tufrg_ctx** out) {
  if (!out) return fail(nullptr, TUFRG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!pts || npts <= 0) return fail(nullptr, TUFRG_EINVAL, "need at least one point");
  tufrg_options o{};
  if (opt) o = *opt;
  if (o.precision != TUFRG_FP64 && o.precision != TUFRG_MIXED)
    return fail(nullptr, TUFRG_EINVAL, "precision must be TUFRG_FP64 or TUFRG_MIXED");
  if (o.flags & ~(uint32_t)TUFRG_NO_CROSS) return fail(nullptr, TUFRG_EINVAL, "unknown flag bits");
  auto* ctx = new tufrg_ctx();
  ctx->opt = o;
  ctx->stream = static_cast<hipStream_t>(stream);
  ctx->host.resize(npts);
  ctx->off.resize(npts);
  int64_t S = 0;
  size_t max_xt = 8, max_yb = 8, max_gp = 8, max_k = 8;
  for (int p = 0; p < npts; ++p) {
    std::string e = build_tables(pts[p], ctx->host[p]);
    if (!e.empty()) {
      delete ctx;
      return fail(nullptr, TUFRG_EINVAL, "point " + std::to_string(p) + ": " + e);
    }
    const HostTables& t = ctx->host[p];
    if (t.lk > 512) {
      delete ctx;
      return fail(nullptr, TUFRG_EINVAL, "point " + std::to_string(p) + ": Lk must be <= 512");
    }
    ctx->off[p] = S;
    S += (int64_t)t.nq * t.nff * t.nff;
    max_xt = std::max(max_xt, (size_t)3 * t.ncol * t.nff * t.nff);
    max_yb = std::max(max_yb, (size_t)2 * 3 * (2 * t.nsh - 1) * t.nff * t.nff);
    max_k = std::max(max_k, (size_t)3 * t.nq * t.nff * t.nff);
  }
  ctx->S = S;
  // device tables (first device call: every argument has been validated)
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return fail(nullptr, TUFRG_EHIP, "no HIP device");
  }
  ctx->dev.resize(npts);
  for (int p = 0; p < npts; ++p) {
    const HostTables& t = ctx->host[p];
    DevTables& d = ctx->dev[p];
    d.nff = t.nff; d.nq = t.nq; d.lq = t.p.Lq; d.lk = t.lk; d.nsh = t.nsh; d.ncol = t.ncol;
    d.smax = t.smax; d.nshell = t.nshell;
    d.t = t.p.t; d.tp = t.p.tp; d.mu = t.p.mu; d.U = t.p.U;
    std::vector<double> cre(t.c.size()), cim(t.c.size());
    for (size_t i = 0; i < t.c.size(); ++i) { cre[i] = t.c[i].real(); cim[i] = t.c[i].imag(); }
    std::vector<int> ss(t.shell_start, t.shell_start + t.nshell + 1);
    std::vector<int> so(t.nff);
    for (int s = 0; s < t.nshell; ++s)
      for (int m = t.shell_start[s]; m < t.shell_start[s + 1]; ++m) so[m] = s;
    std::vector<int32_t> hx(t.hx.begin(), t.hx.end()), hy(t.hy.begin(), t.hy.end());
    std::vector<unsigned short> ehi, elo;
    split_table(t.eph, ehi, elo);
    tufrg_status st;
    if ((st = upload(ctx, cre, &d.cre)) || (st = upload(ctx, cim, &d.cim)) ||
        (st = upload(ctx, ss, &d.shell_start)) || (st = upload(ctx, so, &d.shell_of)) ||
        (st = upload(ctx, t.ebub, &d.ebub)) || (st = upload(ctx, t.pxtab, &d.pxtab)) ||
        (st = upload(ctx, t.pytab, &d.pytab)) || (st = upload(ctx, t.eph, &d.eph)) ||
        (st = upload(ctx, t.cshift, &d.cshift)) || (st = upload(ctx, ehi, &d.eph_hi)) ||
        (st = upload(ctx, elo, &d.eph_lo)) ||
        (st = upload(ctx, t.mrow, &d.mrow)) || (st = upload(ctx, t.ment, &d.ment)) ||
        (st = upload(ctx, hx, &d.hx)) || (st = upload(ctx, hy, &d.hy))) {
      std::string m = ctx->err;
      tufrg_free(ctx);
      return fail(nullptr, st, m);
    }
    int dev_smem = 0;
    hipDeviceGetAttribute(&dev_smem, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device);
    const LoopGeom g = loop_geometry(d);
    if (dev_smem > 0 && g.smem > (size_t)dev_smem) {
      tufrg_free(ctx);
      return fail(nullptr, TUFRG_EINVAL, "point " + std::to_string(p) + ": fine grid too large");
    }
    max_gp = std::max(max_gp, (size_t)g.nsplit * 2 * t.nq * t.nff * t.nff);
  }
  // workspace
  Workspace& w = ctx->ws;
  const size_t b3 = sizeof(double) * 3 * (size_t)S;
  tufrg_status st = TUFRG_OK;
  void* v = nullptr;
  if ((st = dalloc(ctx, sizeof(double) * max_xt, &v))) goto bad;
  w.xt = (double*)v;
  if ((st = dalloc(ctx, sizeof(double) * max_xt, &v))) goto bad;
  w.g2 = (double*)v;
  if ((st = dalloc(ctx, sizeof(double) * max_yb, &v))) goto bad;
  w.yb = (double*)v;
  if ((st = dalloc(ctx, sizeof(double) * max_gp, &v))) goto bad;
  w.dpart = (double*)v;
  if (o.precision == TUFRG_MIXED) {
    if ((st = dalloc(ctx, sizeof(float) * max_k, &v))) goto bad;
    w.kinv = (float*)v;
  }
  if ((st = dalloc(ctx, sizeof(double) * 2 * (size_t)S, &v))) goto bad;
  w.dchi = (double*)v;
  if ((st = dalloc(ctx, b3, &v))) goto bad;
  w.stage = (double*)v;
  if ((st = dalloc(ctx, b3, &v))) goto bad;
  w.ytmp = (double*)v;
  for (int i = 0; i < 7; ++i) {
    if ((st = dalloc(ctx, b3, &v))) goto bad;
    w.k[i] = (double*)v;
  }
  if ((st = dalloc(ctx, sizeof(double) * 1024, &v))) goto bad;
  w.red = (double*)v;
  if ((st = dalloc(ctx, sizeof(unsigned long long) * std::max(npts, 1), &v))) goto bad;
  w.umax = (unsigned long long*)v;
  // side stream (default priority) and the fork/join events of the right-hand side
  if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) != hipSuccess) {
    st = fail(ctx, TUFRG_EHIP, "stream or event creation failed");
    goto bad;
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    st = fail(ctx, TUFRG_EHIP, "device synchronize failed after init");
    goto bad;
  }
  *out = ctx;
  return TUFRG_OK;
bad : {
  std::string m = ctx->err;
  tufrg_free(ctx);
  return fail(nullptr, st, m);
}
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

tufrg_status tufrg_bubbles(tufrg_ctx* ctx, const double* T_host, double* dchi) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (!T_host || !dchi) return fail(ctx, TUFRG_EINVAL, "NULL argument");
  for (size_t p = 0; p < ctx->dev.size(); ++p)
    if (!(T_host[p] > 0.0) || !std::isfinite(T_host[p]))
      return fail(ctx, TUFRG_EINVAL, "T must be finite and > 0");
  for (size_t p = 0; p < ctx->dev.size(); ++p) {
    if (ctx->opt.precision == TUFRG_MIXED)
      launch_loops_mixed(ctx->dev[p], T_host[p], dchi + ctx->off[p], ctx->S, ctx->ws.dpart, true,
                         ctx->stream);
    else
      launch_loops(ctx->dev[p], T_host[p], dchi + ctx->off[p], ctx->S, ctx->ws.dpart, true,
                   ctx->stream);
  }
  HIP_TRY(ctx, hipGetLastError());
  return TUFRG_OK;
}

tufrg_status tufrg_project(tufrg_ctx* ctx, const double* X, double* V) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (!X || !V) return fail(ctx, TUFRG_EINVAL, "NULL argument");
  if (X == V) return fail(ctx, TUFRG_EINVAL, "X and V must not alias");
  for (size_t p = 0; p < ctx->dev.size(); ++p) {
    if (ctx->opt.precision == TUFRG_MIXED) {
      const DevTables& d = ctx->dev[p];
      launch_project_front_mixed(d, X + ctx->off[p], ctx->S, ctx->ws.xt, ctx->ws.yb, ctx->ws.g2,
                                 ctx->opt.flags, ctx->stream);
      launch_inverse_mixed(d, ctx->ws.g2, ctx->ws.kinv, ctx->opt.flags, ctx->stream);
      launch_products_mixed(d, X + ctx->off[p], ctx->S, ctx->ws.kinv, nullptr, nullptr,
                            V + ctx->off[p], 0, ctx->opt.flags, 1.0, ctx->stream);
      continue;
    }
    launch_project_front(ctx->dev[p], X + ctx->off[p], ctx->S, ctx->ws.xt, ctx->ws.yb, ctx->ws.g2,
                         ctx->opt.flags, ctx->stream);
    launch_project_back(ctx->dev[p], X + ctx->off[p], ctx->S, ctx->ws.g2, nullptr, nullptr,
                        V + ctx->off[p], 0, ctx->opt.flags, 1.0, ctx->stream);
  }
  HIP_TRY(ctx, hipGetLastError());
  return TUFRG_OK;
}

tufrg_status tufrg_rhs(tufrg_ctx* ctx, const double* T_host, const double* X, double* dXdT) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (!T_host || !X || !dXdT) return fail(ctx, TUFRG_EINVAL, "NULL argument");
  if (X == dXdT) return fail(ctx, TUFRG_EINVAL, "X and dXdT must not alias");
  for (size_t p = 0; p < ctx->dev.size(); ++p)
    if (!(T_host[p] > 0.0) || !std::isfinite(T_host[p]))
      return fail(ctx, TUFRG_EINVAL, "T must be finite and > 0");
  for (size_t p = 0; p < ctx->dev.size(); ++p) rhs_point(ctx, (int)p, T_host[p], X, dXdT, 1.0);
  HIP_TRY(ctx, hipGetLastError());
  return TUFRG_OK;
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

// ------------------------------------------------------------------ flow
namespace {

struct PointView {
  // a point's three channel blocks inside [3][S] arrays are addressed as
  // ptr + off + c*S; the ODE kernels work on the whole [3][S] range when the
  // context has one point and on per-channel blocks otherwise
  int64_t off, n;
};

// out = X + h * sum_j coef_j k_j over the point's three channel blocks
void axpy_point(tufrg_ctx* ctx, int p, const double* X, double* const* k, const double* coef, int nk,
                double h, double* out) {
  const int64_t off = ctx->off[p], S = ctx->S;
  const HostTables& t = ctx->host[p];
  const int64_t n = (int64_t)t.nq * t.nff * t.nff;
  for (int c = 0; c < 3; ++c) {
    const double* kk[7];
    for (int j = 0; j < nk; ++j) kk[j] = k[j] + c * S + off;
    launch_axpy_stage(X + c * S + off, kk, coef, nk, h, out + c * S + off, n, ctx->stream);
  }
}

tufrg_status maxabs_point(tufrg_ctx* ctx, int p, const double* X, double* result) {
  const int64_t off = ctx->off[p], S = ctx->S;
  const HostTables& t = ctx->host[p];
  const int64_t n = (int64_t)t.nq * t.nff * t.nff;
  launch_fill_u64(ctx->ws.umax + p, 1, 0ull, ctx->stream);
  for (int c = 0; c < 3; ++c) launch_maxabs(X + c * S + off, n, ctx->ws.umax + p, ctx->stream);
  unsigned long long w = 0;
  HIP_TRY(ctx, hipMemcpyAsync(&w, ctx->ws.umax + p, sizeof w, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  *result = word_to_double(w);
  return TUFRG_OK;
}

tufrg_status finish_point(tufrg_ctx* ctx, int p, const double* X, int status,
                          const std::vector<double>& s_hist, const std::vector<double>& m_hist,
                          double xmax, int64_t n_rhs, int64_t n_steps, tufrg_flow_result* r) {
  std::memset(r, 0, sizeof *r);
  r->status = status;
  r->n_rhs = n_rhs;
  r->n_steps = n_steps;
  r->max_abs_X = m_hist.back();
  r->channel = r->q_index = r->irrep = -1;
  r->Tc = 0.0;
  if (status == TUFRG_FLOW_DIVERGED) {
    const size_t k = s_hist.size();
    r->Tc = interp_tc(s_hist[k - 2], s_hist[k - 1], m_hist[k - 2], m_hist[k - 1], xmax);
    const HostTables& t = ctx->host[p];
    const int64_t n = (int64_t)t.nq * t.nff * t.nff;
    std::vector<double> x((size_t)3 * n);
    for (int c = 0; c < 3; ++c)
      HIP_TRY(ctx, hipMemcpy(x.data() + c * n, X + c * ctx->S + ctx->off[p], n * sizeof(double),
                             hipMemcpyDeviceToHost));
    classify(t, x, r);
  }
  return TUFRG_OK;
}

tufrg_status flow_rk4_point(tufrg_ctx* ctx, int p, const tufrg_flow_opts* o, double* X,
                            tufrg_flow_result* r) {
  double* const* k = ctx->ws.k;
  double* stage = ctx->ws.stage;
  const double s0 = std::log(o->T0);
  const double h = (std::log(o->Tmin) - s0) / o->nsteps;
  std::vector<double> s_hist{s0}, m_hist;
  double m;
  ST_TRY(maxabs_point(ctx, p, X, &m));
  m_hist.push_back(m);
  int64_t n_rhs = 0;
  double s = s0;
  const double half[1] = {0.5}, one[1] = {1.0};
  const double fin[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
  for (int step = 0; step < o->nsteps; ++step) {
    double T1 = std::exp(s), Th = std::exp(s + 0.5 * h), T2 = std::exp(s + h);
    rhs_point(ctx, p, T1, X, k[0], T1);
    axpy_point(ctx, p, X, &k[0], half, 1, h, stage);
    rhs_point(ctx, p, Th, stage, k[1], Th);
    axpy_point(ctx, p, X, &k[1], half, 1, h, stage);
    rhs_point(ctx, p, Th, stage, k[2], Th);
    axpy_point(ctx, p, X, &k[2], one, 1, h, stage);
    rhs_point(ctx, p, T2, stage, k[3], T2);
    axpy_point(ctx, p, X, k, fin, 4, h, X);
    n_rhs += 4;
    s = s0 + (step + 1) * h;
    ST_TRY(maxabs_point(ctx, p, X, &m));
    s_hist.push_back(s);
    m_hist.push_back(m);
    if (!std::isfinite(m))
      return finish_point(ctx, p, X, TUFRG_FLOW_NONFINITE, s_hist, m_hist, o->Xmax, n_rhs, step + 1, r);
    if (m > o->Xmax)
      return finish_point(ctx, p, X, TUFRG_FLOW_DIVERGED, s_hist, m_hist, o->Xmax, n_rhs, step + 1, r);
  }
  return finish_point(ctx, p, X, TUFRG_FLOW_REACHED_TMIN, s_hist, m_hist, o->Xmax, n_rhs, o->nsteps, r);
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

tufrg_status flow_dopri5_point(tufrg_ctx* ctx, int p, const tufrg_flow_opts* o, double* X,
                               tufrg_flow_result* r) {
  double* k[7];
  for (int i = 0; i < 7; ++i) k[i] = ctx->ws.k[i];
  double* stage = ctx->ws.stage;
  double* y5 = ctx->ws.ytmp;
  const HostTables& t = ctx->host[p];
  const int64_t n = (int64_t)t.nq * t.nff * t.nff;
  const int nred = 256;
  double s = std::log(o->T0);
  const double s_end = std::log(o->Tmin);
  double h = (o->h0 != 0.0) ? o->h0 : (s_end - s) / 200.0;
  const int max_steps = o->max_steps > 0 ? o->max_steps : 100000;
  std::vector<double> s_hist{s}, m_hist;
  double m;
  ST_TRY(maxabs_point(ctx, p, X, &m));
  m_hist.push_back(m);
  double T = std::exp(s);
  rhs_point(ctx, p, T, X, k[0], T);
  int64_t n_rhs = 1, n_acc = 0;
  std::vector<double> red(nred * 3);
  double e[7];
  for (int j = 0; j < 7; ++j) e[j] = kDpB5[j] - kDpB4[j];
  for (int it = 0; it < max_steps; ++it) {
    if (s + h < s_end) h = s_end - s;
    for (int i = 1; i < 7; ++i) {
      axpy_point(ctx, p, X, k, kDpA[i], i, h, stage);
      const double Ti = std::exp(s + kDpC[i] * h);
      rhs_point(ctx, p, Ti, stage, k[i], Ti);
    }
    n_rhs += 6;
    axpy_point(ctx, p, X, k, kDpB5, 7, h, y5);
    // RMS error norm over the point's 3 n elements
    for (int c = 0; c < 3; ++c) {
      const double* kk[7];
      for (int j = 0; j < 7; ++j) kk[j] = k[j] + c * ctx->S + ctx->off[p];
      launch_errnorm(X + c * ctx->S + ctx->off[p], y5 + c * ctx->S + ctx->off[p], kk, e, 7, h,
                     o->rtol, o->atol, n, ctx->ws.red + c * nred, nred, ctx->stream);
    }
    HIP_TRY(ctx, hipMemcpyAsync(red.data(), ctx->ws.red, sizeof(double) * 3 * nred,
                                hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    double sum = 0.0;
    for (double v : red) sum += v;
    const double err = std::sqrt(sum / (3.0 * (double)n));
    if (!std::isfinite(err)) {
      s_hist.push_back(s + h);
      m_hist.push_back(NAN);
      return finish_point(ctx, p, y5, TUFRG_FLOW_NONFINITE, s_hist, m_hist, o->Xmax, n_rhs, n_acc, r);
    }
    if (err <= 1.0) {
      s = s + h;
      for (int c = 0; c < 3; ++c)
        HIP_TRY(ctx, hipMemcpyAsync(X + c * ctx->S + ctx->off[p], y5 + c * ctx->S + ctx->off[p],
                                    n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
      std::swap(ctx->ws.k[0], ctx->ws.k[6]);
      k[0] = ctx->ws.k[0];
      k[6] = ctx->ws.k[6];
      ++n_acc;
      ST_TRY(maxabs_point(ctx, p, X, &m));
      s_hist.push_back(s);
      m_hist.push_back(m);
      if (m > o->Xmax)
        return finish_point(ctx, p, X, TUFRG_FLOW_DIVERGED, s_hist, m_hist, o->Xmax, n_rhs, n_acc, r);
      if (s <= s_end + 1e-15)
        return finish_point(ctx, p, X, TUFRG_FLOW_REACHED_TMIN, s_hist, m_hist, o->Xmax, n_rhs, n_acc, r);
    }
    const double fac = err == 0.0 ? 5.0 : std::min(5.0, std::max(0.2, 0.9 * std::pow(err, -0.2)));
    h *= fac;
  }
  return finish_point(ctx, p, X, TUFRG_FLOW_REACHED_TMIN, s_hist, m_hist, o->Xmax, n_rhs, n_acc, r);
}

}  // namespace

tufrg_status tufrg_flow(tufrg_ctx* ctx, const tufrg_flow_opts* o, double* X, tufrg_flow_result* res) {
  if (!ctx) return fail(nullptr, TUFRG_EINVAL, "ctx is NULL");
  if (!o || !X || !res) return fail(ctx, TUFRG_EINVAL, "NULL argument");
  if (!(o->T0 > 0.0) || !(o->Tmin > 0.0) || !(o->Tmin < o->T0) || !(o->Xmax > 0.0))
    return fail(ctx, TUFRG_EINVAL, "need T0 > Tmin > 0 and Xmax > 0");
  if (o->scheme == TUFRG_RK4_LOG) {
    if (o->nsteps <= 0) return fail(ctx, TUFRG_EINVAL, "nsteps must be > 0");
  } else if (o->scheme == TUFRG_DOPRI5_LOG) {
    if (!(o->rtol > 0.0) || !(o->atol > 0.0)) return fail(ctx, TUFRG_EINVAL, "rtol, atol must be > 0");
  } else {
    return fail(ctx, TUFRG_EINVAL, "unknown scheme");
  }
  bool nonfinite = false;
  for (size_t p = 0; p < ctx->dev.size(); ++p) {
    tufrg_status st = (o->scheme == TUFRG_RK4_LOG) ? flow_rk4_point(ctx, (int)p, o, X, &res[p])
                                                   : flow_dopri5_point(ctx, (int)p, o, X, &res[p]);
    if (st != TUFRG_OK) return st;
    if (res[p].status == TUFRG_FLOW_NONFINITE) nonfinite = true;
  }
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (nonfinite) return fail(ctx, TUFRG_ENONFINITE, "flow state became non-finite");
  return TUFRG_OK;
}

void tufrg_free(tufrg_ctx* ctx) {
  if (!ctx) return;
  if (!ctx->allocations.empty()) hipStreamSynchronize(ctx->stream);
  if (ctx->side) {
    hipStreamSynchronize(ctx->side);
    hipStreamDestroy(ctx->side);
  }
  if (ctx->ev_fork) hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) hipEventDestroy(ctx->ev_join);
  for (void* p : ctx->allocations) hipFree(p);
  delete ctx;
}

const char* tufrg_last_error(const tufrg_ctx* ctx) {
  if (ctx) return ctx->err.c_str();
  return g_last_error.c_str();
}

}  // extern "C"
