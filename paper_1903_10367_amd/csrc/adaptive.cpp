// Host set-up of adaptive spacetrees (Sec. 2.1): the ragged levels, their bounding boxes,
// cell existence and refinement, and the vertex classes (dof, hanging, composite dof).
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "adaptive.hpp"

namespace adafac {

size_t AdaptHostLevel::nverts() const { return size_t(nc[0] + 1) * (nc[1] + 1) * (d == 3 ? nc[2] + 1 : 1); }
size_t AdaptHostLevel::ncells() const { return size_t(nc[0]) * nc[1] * nc[2]; }

namespace {

// does the closed cell [c h, (c + 1) h]^d meet the closed ball?
bool cell_meets_ball(int d, const int* c, double h, const double* centre, double radius) {
  double d2 = 0.0;
  for (int a = 0; a < d; ++a) {
    const double lo = c[a] * h, hi = (c[a] + 1) * h;
    const double g = std::max(0.0, std::max(lo - centre[a], centre[a] - hi));
    d2 += g * g;
  }
  return d2 <= radius * radius;
}

}  // namespace

std::string build_adapt_tree(AdaptHost& t, int d, int lmin, int L, const std::vector<RefineSpec>& specs,
                             const double* centre, double radius, int l_from) {
  t = AdaptHost{};
  t.d = d;
  t.lmin = lmin;
  t.L = L;
  t.lev.assign(L + 1, AdaptHostLevel{});
  const RefineSpec* spec[32] = {nullptr};
  for (const RefineSpec& s : specs) {
    if (s.level < lmin || s.level >= L) return "refinement flags given for a level outside l_min..l_max-1";
    spec[s.level] = &s;
  }
  auto vbox = [&](const AdaptHostLevel& A, int a) { return A.nc[a] + 1; };
  for (int l = lmin; l <= L; ++l) {
    AdaptHostLevel& A = t.lev[l];
    A.d = d;
    const int n = ipow3(l);
    if (l == lmin) {
      for (int a = 0; a < 3; ++a) {
        A.lo[a] = 0;
        A.nc[a] = a < d ? n : 1;
      }
      A.exists.assign(A.ncells(), 1);
    } else {
      // the children of the refined cells of level l-1, inside 3 x their bounding box
      const AdaptHostLevel& P = t.lev[l - 1];
      int plo[3] = {1 << 30, 1 << 30, 1 << 30}, phi[3] = {-1, -1, -1};
      for (int cz = 0; cz < P.nc[2]; ++cz)
        for (int cy = 0; cy < P.nc[1]; ++cy)
          for (int cx = 0; cx < P.nc[0]; ++cx) {
            if (!P.refined[(size_t(cz) * P.nc[1] + cy) * P.nc[0] + cx]) continue;
            const int c[3] = {cx, cy, cz};
            for (int a = 0; a < 3; ++a) {
              plo[a] = std::min(plo[a], c[a]);
              phi[a] = std::max(phi[a], c[a]);
            }
          }
      if (phi[0] < 0) return "level " + std::to_string(l) + " has no cells (nothing refined on level " +
                             std::to_string(l - 1) + ")";
      for (int a = 0; a < 3; ++a) {
        if (a < d) {
          A.lo[a] = 3 * (P.lo[a] + plo[a]);
          A.nc[a] = 3 * (phi[a] - plo[a] + 1);
        } else {
          A.lo[a] = 0;
          A.nc[a] = 1;
        }
      }
      A.exists.assign(A.ncells(), 0);
      for (int cz = 0; cz < A.nc[2]; ++cz)
        for (int cy = 0; cy < A.nc[1]; ++cy)
          for (int cx = 0; cx < A.nc[0]; ++cx) {
            const int g[3] = {A.lo[0] + cx, A.lo[1] + cy, A.lo[2] + cz};
            int pc[3];
            for (int a = 0; a < 3; ++a) pc[a] = a < d ? g[a] / 3 - P.lo[a] : 0;
            A.exists[(size_t(cz) * A.nc[1] + cy) * A.nc[0] + cx] =
                P.refined[(size_t(pc[2]) * P.nc[1] + pc[1]) * P.nc[0] + pc[0]];
          }
    }
    A.refined.assign(A.ncells(), 0);
    if (l < L) {
      const double h = 1.0 / n;
      for (int cz = 0; cz < A.nc[2]; ++cz)
        for (int cy = 0; cy < A.nc[1]; ++cy)
          for (int cx = 0; cx < A.nc[0]; ++cx) {
            const size_t ci = (size_t(cz) * A.nc[1] + cy) * A.nc[0] + cx;
            if (!A.exists[ci]) continue;
            const int g[3] = {A.lo[0] + cx, A.lo[1] + cy, A.lo[2] + cz};
            bool r = true;
            if (spec[l]) {
              size_t gi = size_t(g[0]) + size_t(n) * (size_t(g[1]) + (d == 3 ? size_t(n) * g[2] : 0));
              r = spec[l]->flags[gi] != 0;
            } else if (radius > 0.0 && l >= l_from) {
              r = cell_meets_ball(d, g, h, centre, radius);
            }
            A.refined[ci] = r ? 1 : 0;
          }
    }
  }
  // vertex classes
  for (int l = lmin; l <= L; ++l) {
    AdaptHostLevel& A = t.lev[l];
    const int n = ipow3(l);
    const int mx = vbox(A, 0), my = vbox(A, 1), mz = d == 3 ? vbox(A, 2) : 1;
    A.vcls.assign(size_t(mx) * my * mz, 0);
    for (int z = 0; z < mz; ++z)
      for (int y = 0; y < my; ++y)
        for (int x = 0; x < mx; ++x) {
          const int g[3] = {A.lo[0] + x, A.lo[1] + y, d == 3 ? A.lo[2] + z : 0};
          bool inter = true;
          for (int a = 0; a < d; ++a) inter = inter && g[a] > 0 && g[a] < n;
          int cnt = 0;
          for (int e = 0; e < (1 << d); ++e) {
            const int cx = x - 1 + (e & 1), cy = y - 1 + ((e >> 1) & 1), cz = d == 3 ? z - 1 + ((e >> 2) & 1) : 0;
            if (cx < 0 || cy < 0 || cz < 0 || cx >= A.nc[0] || cy >= A.nc[1] || cz >= A.nc[2]) continue;
            cnt += A.exists[(size_t(cz) * A.nc[1] + cy) * A.nc[0] + cx];
          }
          uint8_t c = 0;
          if (inter && cnt == (1 << d)) c = kDof;
          else if (inter && cnt > 0) c = kHang;
          A.vcls[(size_t(z) * my + y) * mx + x] = c;
        }
  }
  t.composite = 0;
  for (int l = lmin; l <= L; ++l) {
    AdaptHostLevel& A = t.lev[l];
    const int mx = vbox(A, 0), my = vbox(A, 1), mz = d == 3 ? vbox(A, 2) : 1;
    const AdaptHostLevel* F = l < L ? &t.lev[l + 1] : nullptr;
    const int fx = F ? vbox(*F, 0) : 0, fy = F ? vbox(*F, 1) : 0, fz = F ? (d == 3 ? vbox(*F, 2) : 1) : 0;
    for (int z = 0; z < mz; ++z)
      for (int y = 0; y < my; ++y)
        for (int x = 0; x < mx; ++x) {
          uint8_t& c = A.vcls[(size_t(z) * my + y) * mx + x];
          if (!(c & kDof)) continue;
          bool finer = false;
          if (F) {
            const int X = 3 * (A.lo[0] + x) - F->lo[0], Y = 3 * (A.lo[1] + y) - F->lo[1];
            const int Z = d == 3 ? 3 * (A.lo[2] + z) - F->lo[2] : 0;
            if (X >= 0 && Y >= 0 && Z >= 0 && X < fx && Y < fy && Z < fz)
              finer = (F->vcls[(size_t(Z) * fy + Y) * fx + X] & kDof) != 0;
          }
          if (!finer) {
            c |= kComp;
            ++t.composite;
          }
        }
  }
  return "";
}

}  // namespace adafac
