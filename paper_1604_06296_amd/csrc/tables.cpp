// Host-side construction of the scale-independent tables of one point.
//
// Everything here is computed once per point and uploaded at init: the
// reusable projection data (Kronecker-delta overlaps of bonds and Fourier
// phases, Sec. 2.5 and the stored projection tensors of the appendix on
// symmetries) in the compact form of per-harmonic entry lists, and the
// harmonic tables of the loop kernel.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <tuple>

#include "tufrg_internal.h"

namespace tufrg {
namespace {

const double kSqrt2 = 1.4142135623730951;

// A form factor as a sum of coef * cos(k.R) or coef * sin(k.R) terms.
struct Term {
  double coef;
  bool is_sin;
  int rx, ry;
};
struct FF {
  int irrep;  // 0 A1, 1 B1, 2 B2, 3 A2, 4 E
  int parity;
  std::vector<Term> terms;
};

// C4v bond form factors by shell, order A1, B1, B2, A2, E (the table in tufrg.h).
std::vector<std::vector<FF>> form_factor_table() {
  const double h2 = 0.5 * kSqrt2;  // sqrt2 * 1/2
  std::vector<std::vector<FF>> T(5);
  T[0] = {{0, +1, {{1.0, false, 0, 0}}}};
  T[1] = {
      {0, +1, {{1.0, false, 1, 0}, {1.0, false, 0, 1}}},
      {1, +1, {{1.0, false, 1, 0}, {-1.0, false, 0, 1}}},
      {4, -1, {{kSqrt2, true, 1, 0}}},
      {4, -1, {{kSqrt2, true, 0, 1}}},
  };
  // 2 cos x cos y = cos(x+y) + cos(x-y); 2 sin x sin y = cos(x-y) - cos(x+y);
  // 2 sin x cos y = sin(x+y) + sin(x-y); 2 cos x sin y = sin(x+y) - sin(x-y)
  T[2] = {
      {0, +1, {{1.0, false, 1, 1}, {1.0, false, 1, -1}}},
      {2, +1, {{1.0, false, 1, -1}, {-1.0, false, 1, 1}}},
      {4, -1, {{1.0, true, 1, 1}, {1.0, true, 1, -1}}},
      {4, -1, {{1.0, true, 1, 1}, {-1.0, true, 1, -1}}},
  };
  T[3] = {
      {0, +1, {{1.0, false, 2, 0}, {1.0, false, 0, 2}}},
      {1, +1, {{1.0, false, 2, 0}, {-1.0, false, 0, 2}}},
      {4, -1, {{kSqrt2, true, 2, 0}}},
      {4, -1, {{kSqrt2, true, 0, 2}}},
  };
  // sqrt2 cos2x cos y = (sqrt2/2)(cos(2x+y) + cos(2x-y)), etc.
  T[4] = {
      {0, +1, {{h2, false, 2, 1}, {h2, false, 2, -1}, {h2, false, 1, 2}, {h2, false, 1, -2}}},
      {1, +1, {{h2, false, 2, 1}, {h2, false, 2, -1}, {-h2, false, 1, 2}, {-h2, false, 1, -2}}},
      {2, +1, {{h2, false, 2, -1}, {-h2, false, 2, 1}, {h2, false, 1, -2}, {-h2, false, 1, 2}}},
      {3, +1, {{h2, false, 2, -1}, {-h2, false, 2, 1}, {-h2, false, 1, -2}, {h2, false, 1, 2}}},
      {4, -1, {{1.0, true, 2, 1}, {1.0, true, 2, -1}}},    // 2 sin2x cos y
      {4, -1, {{1.0, true, 1, 2}, {-1.0, true, 1, -2}}},   // 2 cos x sin2y
      {4, -1, {{1.0, true, 1, 2}, {1.0, true, 1, -2}}},    // 2 sin x cos2y
      {4, -1, {{1.0, true, 2, 1}, {-1.0, true, 2, -1}}},   // 2 cos2x sin y
  };
  return T;
}

const int kShellBonds[5][8][2] = {
    {{0, 0}},
    {{1, 0}, {-1, 0}, {0, 1}, {0, -1}},
    {{1, 1}, {-1, -1}, {1, -1}, {-1, 1}},
    {{2, 0}, {-2, 0}, {0, 2}, {0, -2}},
    {{2, 1}, {-2, -1}, {2, -1}, {-2, 1}, {1, 2}, {-1, -2}, {1, -2}, {-1, 2}},
};
const int kShellCount[5] = {1, 4, 4, 4, 8};

}  // namespace

int nff_of_shells(int shells) {
  static const int n[5] = {1, 5, 9, 13, 21};
  return (shells >= 0 && shells <= 4) ? n[shells] : -1;
}

std::string build_tables(const tufrg_point& p, const tufrg_mesh* mesh, HostTables& t, bool symmetric,
                         bool omega) {
  char msg[256];
  if (!(p.t > 0.0) || !std::isfinite(p.t)) return "t must be finite and > 0";
  if (!std::isfinite(p.tp) || !std::isfinite(p.mu) || !std::isfinite(p.U))
    return "t', mu and U must be finite";
  if (p.shells < 0 || p.shells > 4) return "shells must be in 0..4";
  t.p = p;
  t.nshell = p.shells + 1;
  t.nff = nff_of_shells(p.shells);
  t.rmax = p.shells == 0 ? 0 : (p.shells <= 2 ? 1 : 2);
  t.smax = 2 * t.rmax;
  if (p.Lq <= 0 || p.Lq % 2 != 0 || p.Lq <= 4 * t.rmax) {
    std::snprintf(msg, sizeof msg, "Lq=%d must be even and > %d for shells=%d", p.Lq,
                  4 * t.rmax, p.shells);
    return msg;
  }
  if (p.Lk < 4 || p.Lk % 2 != 0) {
    std::snprintf(msg, sizeof msg, "Lk=%d must be even and >= 4", p.Lk);
    return msg;
  }
  if ((int64_t)p.Lk * p.Lk > (int64_t)1 << 28) return "Lk too large";
  if (p.Lq > 256) return "Lq must be <= 256";
  t.mesh = mesh != nullptr && mesh->nq != 0;
  if (t.mesh) {
    // a non-uniform transfer mesh: momenta in the zone [-pi, pi)^2, positive
    // weights summing to 1; every momentum is its own orbit representative
    if (mesh->nq < 1 || mesh->nq > 65535) return "mesh nq must be in 1..65535";
    if (!mesh->qx || !mesh->qy || !mesh->w) return "mesh arrays must not be NULL";
    double wsum = 0.0;
    for (int i = 0; i < mesh->nq; ++i) {
      const double x = mesh->qx[i], y = mesh->qy[i], w = mesh->w[i];
      if (!(x >= -M_PI && x < M_PI) || !(y >= -M_PI && y < M_PI)) return "mesh momenta must lie in [-pi, pi)";
      if (!(w > 0.0) || !std::isfinite(w)) return "mesh weights must be finite and > 0";
      wsum += w;
    }
    if (!(std::fabs(wsum - 1.0) <= 1e-12)) return "mesh weights must sum to 1";
    symmetric = false;
    t.nq = mesh->nq;
    t.qxv.assign(mesh->qx, mesh->qx + t.nq);
    t.qyv.assign(mesh->qy, mesh->qy + t.nq);
    t.wq.resize(t.nq);
    for (int i = 0; i < t.nq; ++i) t.wq[i] = (double)t.nq * mesh->w[i];
  } else {
    t.nq = p.Lq * p.Lq;
    t.qxv.resize(t.nq);
    t.qyv.resize(t.nq);
    for (int q = 0; q < t.nq; ++q) {
      t.qxv[q] = 2.0 * M_PI * (double)(q / p.Lq - p.Lq / 2) / (double)p.Lq;
      t.qyv[q] = 2.0 * M_PI * (double)(q % p.Lq - p.Lq / 2) / (double)p.Lq;
    }
    t.wq.assign(t.nq, 1.0);
  }
  t.lk = p.Lk;
  const int nff = t.nff;

  // bonds, form factors and their real-space coefficients
  auto table = form_factor_table();
  t.bx.clear(); t.by.clear(); t.parity.clear(); t.irrep.clear();
  t.c.assign((size_t)nff * nff, cplx(0, 0));
  std::map<std::pair<int, int>, int> bond_index;
  int idx = 0;
  for (int s = 0; s < t.nshell; ++s) {
    t.shell_start[s] = idx;
    for (int i = 0; i < kShellCount[s]; ++i) {
      bond_index[{kShellBonds[s][i][0], kShellBonds[s][i][1]}] = idx + i;
      t.bx.push_back(kShellBonds[s][i][0]);
      t.by.push_back(kShellBonds[s][i][1]);
    }
    for (size_t i = 0; i < table[s].size(); ++i) {
      const FF& f = table[s][i];
      int m = idx + (int)i;
      t.parity.push_back(f.parity);
      t.irrep.push_back(f.irrep);
      // cos(k.R) = (e^{-ik.R} + e^{ik.R})/2 ; sin(k.R) = (e^{ik.R} - e^{-ik.R})/(2i)
      for (const Term& tm : f.terms) {
        int bp = bond_index.at({tm.rx, tm.ry});
        int bm = bond_index.at({-tm.rx, -tm.ry});
        if (!tm.is_sin) {
          t.c[(size_t)m * nff + bp] += cplx(0.5 * tm.coef, 0.0);
          t.c[(size_t)m * nff + bm] += cplx(0.5 * tm.coef, 0.0);
        } else {
          t.c[(size_t)m * nff + bp] += cplx(0.0, 0.5 * tm.coef);
          t.c[(size_t)m * nff + bm] += cplx(0.0, -0.5 * tm.coef);
        }
      }
    }
    idx += kShellCount[s];
  }
  t.shell_start[t.nshell] = idx;

  // harmonic set bonds + bonds and its half set (Hh[0] = 0)
  std::map<std::pair<int, int>, int> half_index;
  t.hx.assign(1, 0);
  t.hy.assign(1, 0);
  half_index[{0, 0}] = 0;
  for (int a = 0; a < nff; ++a)
    for (int b = 0; b < nff; ++b) {
      int sx = t.bx[a] + t.bx[b], sy = t.by[a] + t.by[b];
      if (sx < 0 || (sx == 0 && sy < 0)) { sx = -sx; sy = -sy; }
      if (!half_index.count({sx, sy})) {
        half_index[{sx, sy}] = (int)t.hx.size();
        t.hx.push_back(sx);
        t.hy.push_back(sy);
      }
    }
  t.nsh = (int)t.hx.size();
  t.ncol = 2 * t.nsh - 1;
  // canonical bond pair of each half-set harmonic: the first (a, b) in bond
  // order with R_a + R_b = S (the surrogate's encoding of S)
  t.pairs.assign((size_t)4 * t.nsh, 0);
  for (int j = 0; j < t.nsh; ++j) {
    bool found = false;
    for (int a = 0; a < nff && !found; ++a)
      for (int b = 0; b < nff && !found; ++b)
        if (t.bx[a] + t.bx[b] == t.hx[j] && t.by[a] + t.by[b] == t.hy[j]) {
          t.pairs[4 * j + 0] = t.bx[a];
          t.pairs[4 * j + 1] = t.by[a];
          t.pairs[4 * j + 2] = t.bx[b];
          t.pairs[4 * j + 3] = t.by[b];
          found = true;
        }
    if (!found) return "internal error: harmonic without a bond pair";
  }
  auto half_of = [&](int sx, int sy, int* conj) {
    bool neg = sx < 0 || (sx == 0 && sy < 0);
    *conj = neg ? 1 : 0;
    if (neg) { sx = -sx; sy = -sy; }
    return half_index.at({sx, sy});
  };

  // Point-group reduction of the transfer grid.  The dispersion and the
  // unshifted fine grid are invariant under the 8 operations g of C4v, so the
  // loop harmonics obey ghat(g q, g S) = ghat(q, S); shifting q by 2 pi e_x
  // moves the fine grid by half a period and gives ghat(q + 2 pi e_x, S) =
  // (-1)^{S_x} ghat(q, S) (Lk even).  Each q maps to the representative r of
  // its orbit (smallest flat index) through an operation h with h q = r + G,
  // G in {0, 2 pi}^2, so that ghat(q, S_j) = (-1)^{G.hS_j / 2 pi} ghat(r, +-h S_j)
  // (ghat is even in S).  Without `symmetric` every q is its own representative.
  if (t.mesh) {
    // no point-group reduction on a mesh: every momentum represents itself,
    // each orbit is the momentum alone with the identity permutation
    t.nirr = t.nq;
    t.irr.resize(t.nq);
    t.symmap.assign((size_t)t.nq * t.nsh, 0);
    for (int q = 0; q < t.nq; ++q) {
      t.irr[q] = q;
      for (int j = 0; j < t.nsh; ++j) t.symmap[(size_t)q * t.nsh + j] = pack_sym(q, j, 0);
    }
    t.tperm.resize(nff);
    for (int m = 0; m < nff; ++m) t.tperm[m] = pack_perm(m, 0);
    t.ntr = 1;
    t.orb_start.resize((size_t)t.nq + 1);
    t.orb_q.resize(t.nq);
    t.orb_tr.assign(t.nq, 0);
    for (int q = 0; q <= t.nq; ++q) t.orb_start[q] = q;
    for (int q = 0; q < t.nq; ++q) t.orb_q[q] = q;
  } else {
    static const int ops[8][4] = {{1, 0, 0, 1},  {-1, 0, 0, 1}, {1, 0, 0, -1}, {-1, 0, 0, -1},
                                  {0, 1, 1, 0},  {0, -1, 1, 0}, {0, 1, -1, 0}, {0, -1, -1, 0}};
    const int lq = p.Lq, half = lq / 2;
    std::vector<int> rep(t.nq), op(t.nq), gx(t.nq), gy(t.nq);
    for (int q = 0; q < t.nq; ++q) {
      const int a = q / lq - half, b = q % lq - half;
      int best = t.nq, bo = 0, bgx = 0, bgy = 0;
      for (int o = 0; o < (symmetric ? 8 : 1); ++o) {
        int a2 = ops[o][0] * a + ops[o][1] * b, b2 = ops[o][2] * a + ops[o][3] * b;
        int sx = 0, sy = 0;
        if (a2 >= half) { a2 -= lq; sx = 1; }     // components lie in [-half, half]
        if (b2 >= half) { b2 -= lq; sy = 1; }
        const int f = (a2 + half) * lq + (b2 + half);
        if (f < best) { best = f; bo = o; bgx = sx; bgy = sy; }
      }
      rep[q] = best; op[q] = bo; gx[q] = bgx; gy[q] = bgy;
    }
    std::vector<int> slot_of(t.nq, -1);
    t.irr.clear();
    for (int q = 0; q < t.nq; ++q)
      if (rep[q] == q) {
        slot_of[q] = (int)t.irr.size();
        t.irr.push_back(q);
      }
    t.nirr = (int)t.irr.size();
    t.symmap.assign((size_t)t.nq * t.nsh, 0);
    for (int q = 0; q < t.nq; ++q) {
      const int* m = ops[op[q]];
      const int slot = slot_of[rep[q]];
      if (slot < 0) return "internal error: orbit representative";
      for (int j = 0; j < t.nsh; ++j) {
        const int s2x = m[0] * t.hx[j] + m[1] * t.hy[j], s2y = m[2] * t.hx[j] + m[3] * t.hy[j];
        int conj;
        const int j2 = half_of(s2x, s2y, &conj);
        const int neg = (gx[q] * s2x + gy[q] * s2y) & 1;
        t.symmap[(size_t)q * t.nsh + j] = pack_sym(slot, j2, neg);
      }
    }
    // Orbits for symmetric states.  In the grid sum of the loops (form
    // factors at p, energies at p +- q/2) the substitution p = h^-1 (p' - G/2)
    // with h q = r + G gives X(q) = T X(r) T^T, T_mn from
    // f_m(h^-1 (k - G/2)) = sum_n T_mn f_n(k).  Expanded in bonds,
    // f_m(h^-1 (k - G/2)) = sum_b c_mb (-1)^{G.(h R_b)/2pi} exp(-i k.(h R_b)),
    // so row m of T is found by matching these coefficients against +-c_n.
    // For this basis every T is a signed permutation (checked here).
    std::map<std::pair<int, int>, int> bond_of;
    for (int b = 0; b < nff; ++b) bond_of[{t.bx[b], t.by[b]}] = b;
    std::map<int, int> tr_index;    // key o * 4 + 2 gx + gy
    t.tperm.clear();
    auto transform_of = [&](int o, int sx, int sy) -> int {
      const int key = o * 4 + 2 * sx + sy;
      auto it = tr_index.find(key);
      if (it != tr_index.end()) return it->second;
      const int* m = ops[o];
      std::vector<cplx> cp((size_t)nff);
      std::vector<int32_t> row((size_t)nff);
      for (int a = 0; a < nff; ++a) {
        std::fill(cp.begin(), cp.end(), cplx(0, 0));
        for (int b = 0; b < nff; ++b) {
          const int rx = m[0] * t.bx[b] + m[1] * t.by[b], ry = m[2] * t.bx[b] + m[3] * t.by[b];
          auto f = bond_of.find({rx, ry});
          if (f == bond_of.end()) return -1;
          const double sg = ((sx * rx + sy * ry) & 1) ? -1.0 : 1.0;
          cp[(size_t)f->second] = sg * t.c[(size_t)a * nff + b];
        }
        int found = -1, neg = 0;
        for (int n = 0; n < nff && found < 0; ++n) {
          double dp = 0.0, dm = 0.0;
          for (int b = 0; b < nff; ++b) {
            dp = std::max(dp, std::abs(cp[(size_t)b] - t.c[(size_t)n * nff + b]));
            dm = std::max(dm, std::abs(cp[(size_t)b] + t.c[(size_t)n * nff + b]));
          }
          if (dp < 1e-9) found = n;
          else if (dm < 1e-9) { found = n; neg = 1; }
        }
        if (found < 0) return -1;
        row[(size_t)a] = pack_perm(found, neg);
      }
      const int idx = (int)(t.tperm.size() / (size_t)nff);
      t.tperm.insert(t.tperm.end(), row.begin(), row.end());
      tr_index[key] = idx;
      return idx;
    };
    t.orb_start.assign((size_t)t.nirr + 1, 0);
    for (int q = 0; q < t.nq; ++q) ++t.orb_start[(size_t)slot_of[rep[q]] + 1];
    for (int s2 = 0; s2 < t.nirr; ++s2) {
      if (t.orb_start[(size_t)s2 + 1] > 8)   // an orbit of C4v has at most 8 members
        return "internal error: orbit larger than the point group";
      t.orb_start[(size_t)s2 + 1] += t.orb_start[(size_t)s2];
    }
    t.orb_q.assign((size_t)t.nq, 0);
    t.orb_tr.assign((size_t)t.nq, 0);
    std::vector<int32_t> fill(t.orb_start.begin(), t.orb_start.end() - 1);
    for (int q = 0; q < t.nq; ++q) {
      const int tr = transform_of(op[q], gx[q], gy[q]);
      if (tr < 0) return "internal error: form factors not closed under the point group";
      const int32_t e = fill[(size_t)slot_of[rep[q]]]++;
      t.orb_q[(size_t)e] = q;
      t.orb_tr[(size_t)e] = tr;
    }
    t.ntr = (int)(t.tperm.size() / (size_t)nff);
  }

  // loop epilogue: chi_mn = sum_{A,B} c_mA c_nB ghat(A+B), ghat even in S
  t.ebub.assign((size_t)nff * nff * t.nsh, 0.0);
  for (int m = 0; m < nff; ++m)
    for (int n = 0; n < nff; ++n)
      for (int a = 0; a < nff; ++a)
        for (int b = 0; b < nff; ++b) {
          cplx w = t.c[(size_t)m * nff + a] * t.c[(size_t)n * nff + b];
          if (w == cplx(0, 0)) continue;
          int conj;
          int j = half_of(t.bx[a] + t.bx[b], t.by[a] + t.by[b], &conj);
          t.ebub[((size_t)m * nff + n) * t.nsh + j] += w.real();
        }

  // loop harmonic tables on the fine grid; w(py) = 1 on the self-paired rows
  // py = 0 and py = Lk/2, 2 on the others (the loop weight is even in p)
  const int nh = 2 * t.smax + 1;
  const int lk = t.lk;
  t.pxtab.assign((size_t)lk * nh, 0.0);
  t.pytab.assign((size_t)(lk / 2 + 1) * nh, 0.0);
  const double two_pi = 2.0 * M_PI;
  for (int j = 0; j < lk; ++j) {
    for (int n = 0; n <= t.smax; ++n) {
      // exact integer reduction of the phase n*j/lk
      double ang = two_pi * (double)((int64_t)n * j % lk) / lk;
      t.pxtab[(size_t)j * nh + n] = std::cos(ang);
      if (n > 0) t.pxtab[(size_t)j * nh + t.smax + n] = std::sin(ang);
    }
  }
  for (int j = 0; j <= lk / 2; ++j) {
    double w = (j == 0 || j == lk / 2) ? 1.0 : 2.0;
    for (int n = 0; n <= t.smax; ++n) {
      double ang = two_pi * (double)((int64_t)n * j % lk) / lk;
      t.pytab[(size_t)j * nh + n] = w * std::cos(ang);
      if (n > 0) t.pytab[(size_t)j * nh + t.smax + n] = w * std::sin(ang);
    }
  }

  // shifted cosines of the loop energies per axis value: p_j = 2 pi j/Lk,
  // cos(p_j + q/2), cos(p_j - q/2)
  auto shift_table = [&](const std::vector<double>& vals, std::vector<double>& tab) {
    tab.assign(vals.size() * lk * 2, 0.0);
    for (size_t i = 0; i < vals.size(); ++i) {
      const double qh = 0.5 * vals[i];
      for (int j = 0; j < lk; ++j) {
        const double pj = two_pi * (double)j / (double)lk;
        tab[(i * lk + j) * 2] = std::cos(pj + qh);
        tab[(i * lk + j) * 2 + 1] = std::cos(pj - qh);
      }
    }
  };
  t.qax.resize(t.nq);
  if (!t.mesh) {
    // one table for both axes: q_i = 2 pi (i - Lq/2)/Lq, halved exactly
    std::vector<double> vals(p.Lq);
    for (int i = 0; i < p.Lq; ++i) vals[i] = 2.0 * M_PI * (double)(i - p.Lq / 2) / (double)p.Lq;
    shift_table(vals, t.cshift);
    t.cshift_y.clear();
    for (int q = 0; q < t.nq; ++q) t.qax[q] = ((q / p.Lq) << 16) | (q % p.Lq);
  } else {
    // the distinct x and y components of the mesh, each axis its own table
    std::vector<double> xs(t.qxv), ys(t.qyv);
    std::sort(xs.begin(), xs.end());
    xs.erase(std::unique(xs.begin(), xs.end()), xs.end());
    std::sort(ys.begin(), ys.end());
    ys.erase(std::unique(ys.begin(), ys.end()), ys.end());
    shift_table(xs, t.cshift);
    shift_table(ys, t.cshift_y);
    for (int q = 0; q < t.nq; ++q) {
      const int ix = (int)(std::lower_bound(xs.begin(), xs.end(), t.qxv[q]) - xs.begin());
      const int iy = (int)(std::lower_bound(ys.begin(), ys.end(), t.qyv[q]) - ys.begin());
      t.qax[q] = (ix << 16) | iy;
    }
  }

  // projection phase table E[u][k] over the transfer momenta, u.S/2: on the
  // uniform grid u_i = 2 pi (i - Lq/2)/Lq, reduced exactly modulo 2 pi in
  // units of pi/Lq; on a mesh from the coordinates
  const int lq = p.Lq;
  t.eph.assign((size_t)t.nq * t.ncol, 0.0);
  if (t.mesh)
    for (int u = 0; u < t.nq; ++u)
      for (int j = 0; j < t.nsh; ++j) {
        const double ang = 0.5 * (t.qxv[u] * t.hx[j] + t.qyv[u] * t.hy[j]);
        t.eph[(size_t)u * t.ncol + j] = std::cos(ang);
        if (j > 0) t.eph[(size_t)u * t.ncol + t.nsh - 1 + j] = std::sin(ang);
      }
  for (int ix = 0; ix < (t.mesh ? 0 : lq); ++ix)
    for (int iy = 0; iy < lq; ++iy) {
      int u = ix * lq + iy;
      for (int j = 0; j < t.nsh; ++j) {
        // u.S/2 = pi * ((ix - lq/2) Sx + (iy - lq/2) Sy) / lq
        int64_t num = (int64_t)(ix - lq / 2) * t.hx[j] + (int64_t)(iy - lq / 2) * t.hy[j];
        int64_t r = ((num % (2 * lq)) + 2 * lq) % (2 * lq);
        double ang = M_PI * (double)r / lq;
        t.eph[(size_t)u * t.ncol + j] = std::cos(ang);
        if (j > 0) t.eph[(size_t)u * t.ncol + t.nsh - 1 + j] = std::sin(ang);
      }
    }

  // projection entry lists. For output channel X and phase vector V, the
  // coefficient matrix M^X_AB(V) collects the bond-space Fourier coefficients
  //   Yhat^{in}_{R1R2}(W) = sum_{m'n'} c_{m'R1} c_{n'R2} Xt^{in}_{m'n'}(W - (R1+R2)/2)
  // of eqn. proj_pos (R3 on the half-shifted lattice):
  //   P: +K1[C] + K1[D] diag(pi)    C: -K1[P] + K2[D]    D: -K2[P] diag(pi) + K2[C]
  //   K1: R1 = B+W, R2 = A+W, V = R1+R2      (Z_AB, A <-> m, B <-> n)
  //   K2: W = -A, R2 = -A-B-R1, V = R1-R2
  // and diag(pi) on the right maps Z_AB -> Z_{A,-B}.
  const int nv = 2 * t.nsh - 1;
  const size_t rows = (size_t)3 * nv * nff * nff;
  std::vector<std::vector<int32_t>> lists(rows);
  auto vfull = [&](int vx, int vy) {
    int conj;
    int j = half_of(vx, vy, &conj);
    return (conj && j > 0) ? (t.nsh - 1 + j) : j;
  };
  auto bond = [&](int x, int y) {
    auto it = bond_index.find({x, y});
    return it == bond_index.end() ? -1 : it->second;
  };
  auto add = [&](int X, int a, int b, int vx, int vy, int in, int b1, int b2, int sox, int soy,
                 int neg) {
    size_t row = (((size_t)X * nv + vfull(vx, vy)) * nff + a) * nff + b;
    lists[row].push_back(pack_entry(in, b1, b2, vfull(sox, soy), neg));
  };
  const int rW = t.smax;
  for (int a = 0; a < nff; ++a)
    for (int b = 0; b < nff; ++b) {
      const int Ax = t.bx[a], Ay = t.by[a], Bx = t.bx[b], By = t.by[b];
      const int mb = bond(-Bx, -By);
      for (int flip = 0; flip < 2; ++flip) {
        // K1 with n-side bond B (flip 0) or -B (flip 1, the diag(pi) term)
        const int Ex = flip ? -Bx : Bx, Ey = flip ? -By : By;
        for (int wx = -rW; wx <= rW; ++wx)
          for (int wy = -rW; wy <= rW; ++wy) {
            int b1 = bond(Ex + wx, Ey + wy), b2 = bond(Ax + wx, Ay + wy);
            if (b1 < 0 || b2 < 0) continue;
            int R1x = Ex + wx, R1y = Ey + wy, R2x = Ax + wx, R2y = Ay + wy;
            int vx = R1x + R2x, vy = R1y + R2y;
            int sox = 2 * wx - R1x - R2x, soy = 2 * wy - R1y - R2y;
            if (flip == 0) {
              add(0, a, b, vx, vy, 1, b1, b2, sox, soy, 0);   // P <- +K1[C]
              add(1, a, b, vx, vy, 0, b1, b2, sox, soy, 1);   // C <- -K1[P]
            } else {
              add(0, a, b, vx, vy, 2, b1, b2, sox, soy, 0);   // P <- +K1[D] diag(pi)
            }
          }
        // K2 with n-side bond B (flip 0) or -B (flip 1)
        for (int b1 = 0; b1 < nff; ++b1) {
          int R1x = t.bx[b1], R1y = t.by[b1];
          int R2x = -Ax - Ex - R1x, R2y = -Ay - Ey - R1y;
          int b2 = bond(R2x, R2y);
          if (b2 < 0) continue;
          int wx = -Ax, wy = -Ay;
          int vx = R1x - R2x, vy = R1y - R2y;
          int sox = 2 * wx - R1x - R2x, soy = 2 * wy - R1y - R2y;
          if (flip == 0) {
            add(1, a, b, vx, vy, 2, b1, b2, sox, soy, 0);     // C <- +K2[D]
            add(2, a, b, vx, vy, 1, b1, b2, sox, soy, 0);     // D <- +K2[C]
          } else {
            add(2, a, b, vx, vy, 0, b1, b2, sox, soy, 1);     // D <- -K2[P] diag(pi)
          }
        }
      }
      (void)mb;
    }
  t.mrow.assign(rows + 1, 0);
  t.ment.clear();
  for (size_t r = 0; r < rows; ++r) {
    t.mrow[r] = (int32_t)t.ment.size();
    t.ment.insert(t.ment.end(), lists[r].begin(), lists[r].end());
  }
  t.mrow[rows] = (int32_t)t.ment.size();

  // algorithmic flop counts of one right-hand side (FP64 flops, FMA = 2).
  // Loops: per (q, p) pair of the half fine grid, 157 flops for the two loop
  // derivatives (the executed FP64 flops of the temperature-flow loop kernel
  // per pair, from its VALU counters at t'=-0.25, 24x24 / 96x96, after the
  // harmonic and contraction terms below: two exponentials, two refined
  // reciprocals, the divided differences; with the Omega cutoff 58, counted
  // from the code: the two arguments, three reciprocals with two Newton steps
  // each, the one-sign and opposite-sign forms) plus 2 channels x (2 smax + 1)
  // harmonic multiply-adds; per transfer momentum the contraction over px
  // (2 N_S' outputs x Lk columns x 2 multiply-adds) and the form-factor
  // epilogue (2 nff^2 N_S' multiply-adds).
  // With the point-group reduction only the representatives of the transfer
  // momenta are integrated; the epilogue runs for every momentum.
  const double nq = t.nq, f2 = (double)nff * nff, f3 = f2 * nff;
  const double pairs = (double)t.nirr * (double)lk * (lk / 2 + 1);
  const double c_pair = omega ? 58.0 : 157.0;
  const double c_acc = 2.0 * 2.0 * (2 * t.smax + 1);
  t.flops_loop_kernel = (int64_t)(pairs * (c_pair + c_acc) + (double)t.nirr * 2.0 * t.nsh * lk * 4.0);
  t.flops_loops = t.flops_loop_kernel + (int64_t)(nq * 2.0 * 2.0 * f2 * t.nsh);
  // forward and inverse transforms (2 flops per real multiply-add), the bond
  // basis change of the transformed propagators and the gathered sums
  double bb = 0.0;
  for (int s = 0; s < t.nshell; ++s) {
    const double ns = t.shell_start[s + 1] - t.shell_start[s];
    bb += ns * ns;
  }
  const double basis = 3.0 * nv * 8.0 * bb * f2 * 2.0;   // two sides, complex, both stages
  t.flops_fwd = (int64_t)(3.0 * f2 * t.ncol * nq * 2.0);
  t.flops_inv = t.flops_fwd;
  t.flops_basis = (int64_t)basis;
  t.flops_gather = (int64_t)(2.0 * t.ment.size());
  t.flops_proj = t.flops_fwd + t.flops_basis + t.flops_gather + t.flops_inv;
  t.flops_prod = (int64_t)(nq * 6.0 * 2.0 * f3);
  return "";
}

}  // namespace tufrg

extern "C" tufrg_status tufrg_mu_from_filling(double t, double tp, double n, double T, int32_t L,
                                              double* mu) {
  if (!mu || !(n > 0.0 && n < 2.0) || !(T > 0.0) || L < 2 || !(t > 0.0)) return TUFRG_EINVAL;
  // n(mu) = (2/L^2) sum_k n_F(eps_k - mu) increases with mu; bisection
  std::vector<double> e0((size_t)L * L);
  double emin = 1e300, emax = -1e300;
  for (int i = 0; i < L; ++i) {
    double cx = std::cos(2.0 * M_PI * i / L);
    for (int j = 0; j < L; ++j) {
      double cy = std::cos(2.0 * M_PI * j / L);
      double e = -2.0 * t * (cx + cy) - 4.0 * tp * cx * cy;
      e0[(size_t)i * L + j] = e;
      emin = std::min(emin, e);
      emax = std::max(emax, e);
    }
  }
  double lo = emin - 1.0, hi = emax + 1.0;
  while (hi - lo > 1e-13) {
    double mid = 0.5 * (lo + hi);
    double acc = 0.0;
    for (double e : e0) acc += 0.5 * (1.0 - std::tanh((e - mid) / (2.0 * T)));
    double nm = 2.0 * acc / ((double)L * L);
    if (nm < n) lo = mid; else hi = mid;
  }
  *mu = 0.5 * (lo + hi);
  return TUFRG_OK;
}
