// Host-side FP64 construction of the multilevel operators of a uniform 3:1 spacetree.
//
//  * Q1 element operator from the coefficient (Sec. 2.1, element-wise form of Sec. 4.2),
//  * BoxMG prolongation for 3-partitioning (Sec. 2.5) or d-linear interpolation,
//  * Ritz-Galerkin coarse operators A_{l-1} = P^T A_l P (Sec. 2.2),
//  * the smoothed restriction R~ = omega R A M^-1 of the eps = 1 operator, truncated to the
//    support of P (Sec. 3.2).
//
// Levels whose cells each lie inside one coefficient block (l >= k for eps given on the
// cells of level k) keep the Q1 operator with that block's eps: the Galerkin product of a Q1
// operator with d-linear transfers is the Q1 operator of the coarse cells, and BoxMG reduces
// to d-linear interpolation when eps is constant on every coarse cell and along every coarse
// face.  Only levels below k store explicit 3^d stencils and BoxMG weights.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

#include "adafac_internal.hpp"
#include "adaptive.hpp"

namespace adafac {
namespace {

// 1D element matrices of the unit interval: stiffness and mass of linear shape functions.
constexpr double k1[2][2] = {{1.0, -1.0}, {-1.0, 1.0}};
constexpr double m1[2][2] = {{1.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 1.0 / 3.0}};

// Element stiffness of the unit d-cell as a sum of tensor products: K = sum_a k(a) x m(others).
double ref_element(int d, int i, int j) {
  double s = 0.0;
  for (int a = 0; a < d; ++a) {
    double p = 1.0;
    for (int b = 0; b < d; ++b) {
      int ib = (i >> b) & 1, jb = (j >> b) & 1;
      p *= (a == b) ? k1[ib][jb] : m1[ib][jb];
    }
    s += p;
  }
  return s;
}

struct Grid {
  int d, nv;
  size_t lin(const int* v) const {
    size_t r = 0;
    for (int a = d - 1; a >= 0; --a) r = r * nv + v[a];
    return r;
  }
  bool inside(const int* v) const {
    for (int a = 0; a < d; ++a) if (v[a] < 0 || v[a] >= nv) return false;
    return true;
  }
  bool interior(const int* v) const {
    for (int a = 0; a < d; ++a) if (v[a] <= 0 || v[a] >= nv - 1) return false;
    return true;
  }
  void unlin(size_t i, int* v) const {
    for (int a = 0; a < d; ++a) { v[a] = int(i % nv); i /= nv; }
  }
};

inline int st_index(int d, const int* o) {  // offsets in {-1,0,1}^d
  int r = 0;
  for (int a = d - 1; a >= 0; --a) r = r * 3 + (o[a] + 1);
  return r;
}
inline int st_size(int d) { return d == 2 ? 9 : 27; }
// offset o in {-1,0,1}^d of stencil slot t (x fastest); o[2] = 0 in 2D
inline void st_offset(int t, int d, int* o) {
  o[0] = t % 3 - 1;
  o[1] = (t / 3) % 3 - 1;
  o[2] = d == 3 ? t / 9 - 1 : 0;
}

double cell_eps(const HostOps& ops, int level, const int* c) {
  int bs = ipow3(level - ops.k);
  size_t idx = 0;
  for (int a = ops.dim - 1; a >= 0; --a) idx = idx * ops.nb + c[a] / bs;
  return ops.eps[idx];
}

// Q1 stencil entry: sum over the cells containing both v and v+o of eps h^(d-2) K[i][j].
double fem_entry(const HostOps& ops, int level, const int* v, const int* o) {
  int d = ops.dim, n = ipow3(level);
  double h = 1.0 / n, s = 0.0;
  for (int cm = 0; cm < (1 << d); ++cm) {
    int c[3], i = 0, j = 0;
    bool ok = true;
    for (int a = 0; a < d; ++a) {
      c[a] = v[a] - ((cm >> a) & 1);            // lower corner of an adjacent cell
      if (c[a] < 0 || c[a] >= n) { ok = false; break; }
      int li = v[a] - c[a], lj = v[a] + o[a] - c[a];
      if (lj < 0 || lj > 1) { ok = false; break; }
      i |= li << a; j |= lj << a;
    }
    if (!ok) continue;
    s += cell_eps(ops, level, c) * std::pow(h, d - 2) * ref_element(d, i, j);
  }
  return s;
}

// Stencil (3^d per vertex) of a Q1 level; rows and columns of boundary vertices are zero.
void fill_fem_stencil(const HostOps& ops, HostLevel& hl) {
  int d = ops.dim, ns = st_size(d);
  Grid g{d, hl.nv};
  hl.st.assign(hl.nverts * ns, 0.0);
  for (size_t i = 0; i < hl.nverts; ++i) {
    int v[3] = {0, 0, 0};
    g.unlin(i, v);
    if (!g.interior(v)) continue;
    for (int t = 0; t < ns; ++t) {
      int o[3], w[3] = {0, 0, 0};
      st_offset(t, d, o);
      for (int a = 0; a < d; ++a) w[a] = v[a] + o[a];
      if (!g.interior(w)) continue;
      hl.st[i * ns + st_index(d, o)] = fem_entry(ops, hl.level, v, o);
    }
  }
}

// P(f <- c) of the transfer from level l-1 into level l (masked to dofs).
double pweight(const HostOps& ops, int l, const int* f, const int* c) {
  int d = ops.dim;
  const HostLevel& F = ops.lev[l];
  Grid gf{d, F.nv}, gc{d, ops.lev[l - 1].nv};
  if (!gf.interior(f) || !gc.interior(c)) return 0.0;
  if (F.pw.empty()) {
    double w = 1.0;
    for (int a = 0; a < d; ++a) {
      int dd = std::abs(f[a] - 3 * c[a]);
      if (dd >= 3) return 0.0;
      w *= 1.0 - dd / 3.0;
    }
    return w;
  }
  int nc = ops.lev[l - 1].n, e = 0;
  for (int a = 0; a < d; ++a) {
    int cell = std::min(f[a] / 3, nc - 1);
    int ea = c[a] - cell;
    if (ea < 0 || ea > 1) return 0.0;
    e |= ea << a;
  }
  return F.pw[gf.lin(f) * (1u << d) + e];
}

bool solve_dense(int m, double* M, double* x) {  // Gaussian elimination, partial pivoting; x holds rhs
  for (int c = 0; c < m; ++c) {
    int p = c;
    for (int r = c + 1; r < m; ++r) if (std::fabs(M[r * m + c]) > std::fabs(M[p * m + c])) p = r;
    if (M[p * m + c] == 0.0) return false;
    if (p != c) {
      for (int k = 0; k < m; ++k) std::swap(M[c * m + k], M[p * m + k]);
      std::swap(x[c], x[p]);
    }
    for (int r = c + 1; r < m; ++r) {
      double f = M[r * m + c] / M[c * m + c];
      for (int k = c; k < m; ++k) M[r * m + k] -= f * M[c * m + k];
      x[r] -= f * x[c];
    }
  }
  for (int c = m - 1; c >= 0; --c) {
    double s = x[c];
    for (int k = c + 1; k < m; ++k) s -= M[c * m + k] * x[k];
    x[c] = s / M[c * m + c];
  }
  return true;
}

// BoxMG weights (Sec. 2.5) of the transfer into level l, from the stencil of level l.
// For every coarse cell and each of its corners e: identity at c-points; on every coarse
// edge, then face, the stencil is summed along the normal directions and the collapsed
// homogeneous equations are solved for the points inside it; inside the cell A P e = 0.
bool fill_boxmg(const HostOps& ops, HostLevel& F) {
  int d = ops.dim, ns = st_size(d), nc = F.n / 3, nf = F.n;
  Grid gf{d, F.nv};
  const int nloc = d == 2 ? 16 : 64;           // 4^d points of a closed coarse cell
  auto lidx = [&](const int* p) { int r = 0; for (int a = d - 1; a >= 0; --a) r = r * 4 + p[a]; return r; };
  F.pw.assign(F.nverts * (1u << d), 0.0);
  int ncell = 1;
  for (int a = 0; a < d; ++a) ncell *= nc;
  for (int ci = 0; ci < ncell; ++ci) {
    int cc[3] = {0, 0, 0}, base[3] = {0, 0, 0};
    { int t = ci; for (int a = 0; a < d; ++a) { cc[a] = t % nc; t /= nc; base[a] = 3 * cc[a]; } }
    for (int e = 0; e < (1 << d); ++e) {
      int cv[3] = {0, 0, 0};
      bool cint = true;
      for (int a = 0; a < d; ++a) { cv[a] = cc[a] + ((e >> a) & 1); if (cv[a] <= 0 || cv[a] >= nc) cint = false; }
      if (!cint) continue;                      // no shape function on a boundary coarse vertex
      double val[64];
      for (int t = 0; t < nloc; ++t) val[t] = 0.0;
      { int p[3] = {0, 0, 0}; for (int a = 0; a < d; ++a) p[a] = 3 * ((e >> a) & 1); val[lidx(p)] = 1.0; }
      // sub-faces by increasing dimension m: free axes take local values {1,2}
      for (int m = 1; m <= d; ++m) {
        for (int freem = 0; freem < (1 << d); ++freem) {
          if (__builtin_popcount(freem) != m) continue;
          int nfix = d - m;
          for (int fv = 0; fv < (1 << nfix); ++fv) {
            int fixval[3] = {0, 0, 0};
            { int t = 0; for (int a = 0; a < d; ++a) if (!((freem >> a) & 1)) fixval[a] = 3 * ((fv >> t++) & 1); }
            bool onb = false;
            for (int a = 0; a < d; ++a)
              if (!((freem >> a) & 1) && (base[a] + fixval[a] == 0 || base[a] + fixval[a] == nf)) onb = true;
            int npts = 1 << m;
            int pts[8][3];
            for (int q = 0; q < npts; ++q) {
              int t = 0;
              for (int a = 0; a < d; ++a) pts[q][a] = ((freem >> a) & 1) ? 1 + ((q >> t++) & 1) : fixval[a];
            }
            if (onb) { for (int q = 0; q < npts; ++q) val[lidx(pts[q])] = 0.0; continue; }
            double M[64], x[8];
            for (int q = 0; q < npts * npts; ++q) M[q] = 0.0;
            for (int q = 0; q < npts; ++q) {
              x[q] = 0.0;
              int g[3] = {0, 0, 0};
              for (int a = 0; a < d; ++a) g[a] = base[a] + pts[q][a];
              const double* row = &F.st[gf.lin(g) * ns];
              for (int t = 0; t < ns; ++t) {
                int o[3];
                st_offset(t, d, o);
                double a_ = row[st_index(d, o)];
                if (a_ == 0.0) continue;
                int p[3] = {0, 0, 0};
                for (int a = 0; a < d; ++a) p[a] = pts[q][a] + (((freem >> a) & 1) ? o[a] : 0);
                int col = -1;
                for (int r = 0; r < npts; ++r) {
                  bool same = true;
                  for (int a = 0; a < d; ++a) same = same && pts[r][a] == p[a];
                  if (same) { col = r; break; }
                }
                if (col >= 0) M[q * npts + col] += a_;
                else x[q] -= a_ * val[lidx(p)];
              }
            }
            if (!solve_dense(npts, M, x)) return false;
            for (int q = 0; q < npts; ++q) val[lidx(pts[q])] = x[q];
          }
        }
      }
      // store: fine points whose clamped coarse cell is this one
      int p[3] = {0, 0, 0};
      for (int t = 0; t < nloc; ++t) {
        int tt = t;
        bool mine = true;
        for (int a = 0; a < d; ++a) {
          p[a] = tt % 4; tt /= 4;
          if (p[a] == 3 && cc[a] != nc - 1) mine = false;
        }
        if (!mine) continue;
        int f[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) f[a] = base[a] + p[a];
        if (!gf.interior(f)) continue;
        F.pw[gf.lin(f) * (1u << d) + e] = val[t];
      }
    }
  }
  return true;
}

// Ritz-Galerkin: stencil of level l-1 from the stencil of level l and P_l.
void fill_galerkin(HostOps& ops, int l) {
  int d = ops.dim, ns = st_size(d);
  const HostLevel& F = ops.lev[l];
  HostLevel& C = ops.lev[l - 1];
  Grid gf{d, F.nv}, gc{d, C.nv};
  C.st.assign(C.nverts * ns, 0.0);
  const int r5 = 5, r7 = 7;
  int n5 = d == 2 ? 25 : 125, n7 = d == 2 ? 49 : 343;
  std::vector<double> phi(n5), y(n7);
  for (size_t wi = 0; wi < C.nverts; ++wi) {
    int w[3] = {0, 0, 0};
    gc.unlin(wi, w);
    if (!gc.interior(w)) continue;
    // phi = P e_w on [3w-2, 3w+2]^d
    for (int t = 0; t < n5; ++t) {
      int f[3] = {0, 0, 0}, tt = t;
      for (int a = 0; a < d; ++a) { f[a] = 3 * w[a] - 2 + tt % r5; tt /= r5; }
      phi[t] = pweight(ops, l, f, w);
    }
    // y = A_l phi on [3w-3, 3w+3]^d
    for (int t = 0; t < n7; ++t) {
      int g[3] = {0, 0, 0}, tt = t;
      for (int a = 0; a < d; ++a) { g[a] = 3 * w[a] - 3 + tt % r7; tt /= r7; }
      double s = 0.0;
      if (gf.interior(g)) {
        const double* row = &F.st[gf.lin(g) * ns];
        for (int so = 0; so < ns; ++so) {
          int o[3];
          st_offset(so, d, o);
          int q[3] = {0, 0, 0};
          bool in5 = true;
          int idx = 0, mul = 1;
          for (int a = 0; a < d; ++a) {
            q[a] = g[a] + o[a] - (3 * w[a] - 2);
            if (q[a] < 0 || q[a] >= r5) in5 = false;
            idx += q[a] * mul; mul *= r5;
          }
          if (in5) s += row[st_index(d, o)] * phi[idx];
        }
      }
      y[t] = s;
    }
    // A_{l-1}(v, w) = sum_g P(g, v) y(g), v = w + o
    for (int so = 0; so < ns; ++so) {
      int o[3];
      st_offset(so, d, o);
      int v[3] = {0, 0, 0};
      for (int a = 0; a < d; ++a) v[a] = w[a] + o[a];
      if (!gc.interior(v)) continue;
      double s = 0.0;
      for (int t = 0; t < n7; ++t) {
        if (y[t] == 0.0) continue;
        int g[3] = {0, 0, 0}, tt = t;
        for (int a = 0; a < d; ++a) { g[a] = 3 * w[a] - 3 + tt % r7; tt /= r7; }
        s += pweight(ops, l, g, v) * y[t];
      }
      int mo[3] = {-o[0], -o[1], d == 3 ? -o[2] : 0};
      C.st[gc.lin(v) * ns + st_index(d, mo)] = s;   // row v, column w = v - (-o)
    }
  }
}

// (A_l phi)(f) at an interior vertex f of level l for a function phi of the level's vertices
// (zero on the boundary): the stored stencil row, or the Q1 elements of the cells around f.
template <typename Phi>
double apply_row(const HostOps& ops, int l, const int* f, Phi&& phi) {
  const int d = ops.dim, ns = st_size(d);
  const HostLevel& F = ops.lev[l];
  Grid g{d, F.nv};
  double s = 0.0;
  if (!F.st.empty()) {
    const double* row = &F.st[g.lin(f) * ns];
    for (int t = 0; t < ns; ++t) {
      if (row[t] == 0.0) continue;
      int o[3], w[3] = {0, 0, 0};
      st_offset(t, d, o);
      for (int a = 0; a < d; ++a) w[a] = f[a] + o[a];
      s += row[t] * phi(w);
    }
    return s;
  }
  const int n = F.n;
  const double hd2 = std::pow(F.h, d - 2);
  for (int cm = 0; cm < (1 << d); ++cm) {
    int c[3] = {0, 0, 0}, i = 0;
    bool ok = true;
    for (int a = 0; a < d; ++a) {
      c[a] = f[a] - ((cm >> a) & 1);
      if (c[a] < 0 || c[a] >= n) { ok = false; break; }
      i |= (f[a] - c[a]) << a;
    }
    if (!ok) continue;
    double cs = 0.0;
    for (int j = 0; j < (1 << d); ++j) {
      int w[3] = {0, 0, 0};
      for (int a = 0; a < d; ++a) w[a] = c[a] + ((j >> a) & 1);
      const double k = ref_element(d, i, j);
      if (k != 0.0 && g.interior(w)) cs += k * phi(w);
    }
    s += cell_eps(ops, l, c) * hd2 * cs;
  }
  return s;
}

// The smoothed restriction of Sec. 3.2 built from the operator itself (the second of the two
// choices discussed there; the paper notes that R~ must then be stored): for every interior
// vertex c of level l-1 and fine offset o with |o|_inf <= 2,
//   R~(c, 3c + o) = omega sum_w P(w <- c) A_l(w, 3c + o) / D_l(3c + o),
// i.e. omega P^T A D^-1 truncated to the support of P.  A is symmetric, so the sum is
// (A_l (P e_c))(3c + o).  Stored on level l-1 as 5^d weights per vertex.
void fill_rtilde_operator(HostOps& ops, int l, double omega) {
  const int d = ops.dim, n5 = d == 2 ? 25 : 125;
  const HostLevel& F = ops.lev[l];
  HostLevel& C = ops.lev[l - 1];
  Grid gf{d, F.nv}, gc{d, C.nv};
  C.rtw.assign(C.nverts * n5, 0.0);
  const int zero[3] = {0, 0, 0};
  auto diag = [&](const int* f) { return F.dg.empty() ? fem_entry(ops, l, f, zero) : F.dg[gf.lin(f)]; };
  parallel_ranges(C.nverts, [&](size_t c0, size_t c1) {
    double pe[125];
    for (size_t ci = c0; ci < c1; ++ci) {
      int c[3] = {0, 0, 0};
      gc.unlin(ci, c);
      if (!gc.interior(c)) continue;
      // P e_c on its support [3c - 2, 3c + 2]^d
      for (int t = 0; t < n5; ++t) {
        int w[3] = {0, 0, 0}, tt = t;
        for (int a = 0; a < d; ++a) { w[a] = 3 * c[a] + tt % 5 - 2; tt /= 5; }
        pe[t] = pweight(ops, l, w, c);
      }
      auto phi = [&](const int* w) {
        int t = 0, mul = 1;
        for (int a = 0; a < d; ++a) {
          const int q = w[a] - 3 * c[a] + 2;
          if (q < 0 || q > 4) return 0.0;
          t += q * mul;
          mul *= 5;
        }
        return pe[t];
      };
      for (int t = 0; t < n5; ++t) {
        int f[3] = {0, 0, 0}, tt = t;
        for (int a = 0; a < d; ++a) { f[a] = 3 * c[a] + tt % 5 - 2; tt /= 5; }
        if (!gf.interior(f)) continue;
        C.rtw[ci * n5 + t] = omega * apply_row(ops, l, f, phi) / diag(f);
      }
    }
  });
}

}  // namespace

double fem_stencil_entry(const HostOps& ops, int level, const int* v, const int* o) {
  return fem_entry(ops, level, v, o);
}

std::string build_host_ops(HostOps& ops, int transfer_boxmg, double omega, int rtilde_operator) {
  int d = ops.dim;
  ops.lev.assign(ops.L + 1, HostLevel{});
  for (int l = 0; l <= ops.L; ++l) {
    HostLevel& hl = ops.lev[l];
    hl.level = l; hl.n = ipow3(l); hl.nv = hl.n + 1; hl.h = 1.0 / hl.n;
    hl.nverts = 1;
    for (int a = 0; a < d; ++a) hl.nverts *= hl.nv;
    hl.fem = l >= ops.k;
  }
  // levels that need explicit stencils: k (if used as the fine side of a stored transfer) and below
  int top_stored = std::min(ops.k, ops.L);
  for (int l = ops.lmin; l <= ops.L; ++l) {
    if (l <= top_stored && l >= ops.k) fill_fem_stencil(ops, ops.lev[l]);
  }
  for (int l = top_stored; l > ops.lmin; --l) {
    HostLevel& F = ops.lev[l];
    if (!F.fem && F.st.empty()) return "internal: missing stencil";
    if (transfer_boxmg && l - 1 < ops.k) {
      if (!fill_boxmg(ops, F)) return "BoxMG: singular collapsed system";
    }
    if (l - 1 < ops.k) {
      fill_galerkin(ops, l);   // level l-1 becomes a stored (Galerkin) level
      ops.lev[l - 1].fem = false;
    }
  }
  // diagonals of the stored levels (a Q1 level's diagonal is positive because eps is, and the
  // kernels derive it from eps)
  for (int l = ops.lmin; l <= ops.L; ++l) {
    HostLevel& hl = ops.lev[l];
    if (hl.fem) continue;
    hl.dg.assign(hl.nverts, 0.0);
    Grid g{d, hl.nv};
    int zero[3] = {0, 0, 0}, ns = st_size(d), ctr = st_index(d, zero);
    for (size_t i = 0; i < hl.nverts; ++i) {
      int v[3] = {0, 0, 0};
      g.unlin(i, v);
      if (!g.interior(v)) continue;
      hl.dg[i] = hl.st.empty() ? fem_entry(ops, l, v, zero) : hl.st[i * ns + ctr];
      if (!(hl.dg[i] > 0.0)) return "non-positive diagonal";
    }
  }
  if (rtilde_operator)
    for (int l = ops.lmin + 1; l <= ops.L; ++l) fill_rtilde_operator(ops, l, omega);
  // R~: omega times the eps = 1 smoothed operator M^-1 A P (d-linear hat, unit stencil),
  // truncated to offsets |o| <= 2 (the support of P).
  {
    int n5 = d == 2 ? 25 : 125;
    ops.rtilde.assign(n5, 0.0);
    // unit Q1 stencil (h = 1, eps = 1) at an interior vertex
    double unit[27];
    for (int t = 0; t < 27; ++t) unit[t] = 0.0;
    for (int t = 0; t < st_size(d); ++t) {
      int o[3];
      st_offset(t, d, o);
      double s = 0.0;
      for (int cm = 0; cm < (1 << d); ++cm) {
        int i = 0, j = 0;
        bool ok = true;
        for (int a = 0; a < d; ++a) {
          int li = (cm >> a) & 1, lj = li + o[a];
          if (lj < 0 || lj > 1) { ok = false; break; }
          i |= li << a; j |= lj << a;
        }
        if (ok) s += ref_element(d, i, j);
      }
      unit[t] = s;
    }
    int zero[3] = {0, 0, 0};
    double diag = unit[st_index(d, zero)];
    auto hat = [&](const int* p) {
      double w = 1.0;
      for (int a = 0; a < d; ++a) { int q = std::abs(p[a]); if (q >= 3) return 0.0; w *= 1.0 - q / 3.0; }
      return w;
    };
    for (int t = 0; t < n5; ++t) {
      int p[3] = {0, 0, 0}, tt = t;
      for (int a = 0; a < d; ++a) { p[a] = tt % 5 - 2; tt /= 5; }
      double s = 0.0;
      for (int so = 0; so < st_size(d); ++so) {
        int o[3], q[3] = {0, 0, 0};
        st_offset(so, d, o);
        for (int a = 0; a < d; ++a) q[a] = p[a] + o[a];
        s += unit[so] * hat(q);
      }
      ops.rtilde[t] = omega * s / diag;
    }
    // tensor-product factors: m = (1D mass stencil) * (1D hat), kc = (1D stiffness * hat)(0)
    double mass1[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0}, stiff1[3] = {-1.0, 2.0, -1.0};
    auto hat1 = [](int q) { q = std::abs(q); return q >= 3 ? 0.0 : 1.0 - q / 3.0; };
    for (int o = -2; o <= 2; ++o) {
      double mm = 0.0;
      for (int j = -1; j <= 1; ++j) mm += mass1[j + 1] * hat1(o + j);
      ops.rt_m[o + 2] = mm;
    }
    double kc = 0.0;
    for (int j = -1; j <= 1; ++j) kc += stiff1[j + 1] * hat1(j);
    ops.rt_scale = omega * kc / diag;
    for (int t = 0; t < n5; ++t) {
      int p[3] = {0, 0, 0}, tt = t;
      for (int a = 0; a < d; ++a) { p[a] = tt % 5 - 2; tt /= 5; }
      double sep = 0.0;
      for (int a = 0; a < d; ++a) {
        if (p[a] != 0) continue;
        double w = 1.0;
        for (int b = 0; b < d; ++b) if (b != a) w *= ops.rt_m[p[b] + 2];
        sep += w;
      }
      sep *= ops.rt_scale;
      if (std::fabs(sep - ops.rtilde[t]) > 1e-14 * omega) return "R~ is not the expected tensor-product sum";
    }
  }
  return "";
}

}  // namespace adafac
