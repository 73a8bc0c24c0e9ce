// Host set-up of adaptive spacetrees (Sec. 2.1): the ragged levels, their bounding boxes,
// cell existence and refinement, and the vertex classes (dof, hanging, composite dof).
// Every pass is linear in the box and split over host threads by z-planes (a regrid of a
// level-6 3D tree touches about 10^7 cells and vertices per level).
#include <algorithm>
#include <cmath>
#include <cstring>
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

// Runs over the vertices whose class has a bit of mask: disjoint windows of at most 64 box
// vertices, each starting at the first such vertex rounded down to a multiple of 16 (not below
// the previous run's end), in box order.  Unselected vertices inside a window are skipped by the
// kernels' own class tests.  Eight class bytes at a time are skipped where none is selected.
static void make_runs(const std::vector<uint8_t>& cls, uint8_t mask, std::vector<uint32_t>& out) {
  out.clear();
  const size_t n = cls.size();
  uint64_t rep = 0;
  for (int b = 0; b < 8; ++b) rep |= uint64_t(mask) << (8 * b);
  size_t i = 0, prev = 0;
  while (i < n) {
    if (i + 8 <= n) {
      uint64_t w;
      std::memcpy(&w, &cls[i], 8);
      if (!(w & rep)) {
        i += 8;
        continue;
      }
    }
    if (!(cls[i] & mask)) {
      ++i;
      continue;
    }
    const size_t s = std::max(i & ~size_t(15), prev);
    const size_t e = std::min(n, s + 64);
    out.push_back(uint32_t(s));
    out.push_back(uint32_t(e - s));
    prev = i = e;
  }
}

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
      // every refined parent writes its 3^d children (parent planes own disjoint child planes)
      const int zlo = d == 3 ? plo[2] : 0, zn = d == 3 ? phi[2] - plo[2] + 1 : 1;
      parallel_ranges(size_t(zn), [&](size_t q0, size_t q1) {
        for (size_t q = q0; q < q1; ++q) {
          const int pz = zlo + int(q);
          for (int py = plo[1]; py <= phi[1]; ++py)
            for (int px = plo[0]; px <= phi[0]; ++px) {
              if (!P.refined[(size_t(pz) * P.nc[1] + py) * P.nc[0] + px]) continue;
              const int x0 = 3 * (P.lo[0] + px) - A.lo[0], y0 = 3 * (P.lo[1] + py) - A.lo[1];
              const int z0 = d == 3 ? 3 * (P.lo[2] + pz) - A.lo[2] : 0;
              for (int dz = 0; dz < (d == 3 ? 3 : 1); ++dz)
                for (int dy = 0; dy < 3; ++dy)
                  std::fill_n(&A.exists[(size_t(z0 + dz) * A.nc[1] + (y0 + dy)) * A.nc[0] + x0], 3, uint8_t(1));
            }
        }
      });
    }
    A.refined.assign(A.ncells(), 0);
    if (l < L) {
      const double h = 1.0 / n;
      parallel_ranges(size_t(A.nc[2]), [&](size_t z0, size_t z1) {
        for (int cz = int(z0); cz < int(z1); ++cz)
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
      });
    }
  }
  // Vertex classes, finest level first: interior vertices with all 2^d cells of their level are
  // dofs, with some of them hang; a dof is composite unless the next finer level has a dof at
  // its position.
  t.composite = 0;
  const uint8_t full = uint8_t(1 << d);
  for (int l = L; l >= lmin; --l) {
    AdaptHostLevel& A = t.lev[l];
    const int n = ipow3(l);
    const int cx = A.nc[0], cy = A.nc[1], cz = A.nc[2];
    const int mx = cx + 1, my = cy + 1, mz = d == 3 ? cz + 1 : 1;
    const AdaptHostLevel* F = l < L ? &t.lev[l + 1] : nullptr;
    const int fx = F ? F->nc[0] + 1 : 0, fy = F ? F->nc[1] + 1 : 0, fz = F ? (d == 3 ? F->nc[2] + 1 : 1) : 0;
    const std::vector<uint8_t> zero(size_t(cx), 0);
    A.vcls.assign(size_t(mx) * my * mz, 0);
    std::vector<size_t> part(size_t(mz), 0);
    parallel_ranges(size_t(mz), [&](size_t z0, size_t z1) {
      for (int z = int(z0); z < int(z1); ++z) {
        const int gz = d == 3 ? A.lo[2] + z : 1;
        if (d == 3 && (gz <= 0 || gz >= n)) continue;
        size_t k = 0;
        for (int y = 0; y < my; ++y) {
          const int gy = A.lo[1] + y;
          if (gy <= 0 || gy >= n) continue;
          // the (up to) 2^(d-1) cell rows around this vertex row; missing rows read as zero
          const uint8_t* r[4];
          int nr = 0;
          for (int dz = (d == 3 ? -1 : 0); dz <= 0; ++dz)
            for (int dy = -1; dy <= 0; ++dy) {
              const int zz = z + dz, yy = y + dy;
              const bool in = zz >= 0 && zz < cz && yy >= 0 && yy < cy;
              r[nr++] = in ? &A.exists[(size_t(zz) * cy + yy) * cx] : zero.data();
            }
          uint8_t* out = &A.vcls[(size_t(z) * my + y) * mx];
          for (int x = 0; x < mx; ++x) {
            const int gx = A.lo[0] + x;
            if (gx <= 0 || gx >= n) continue;
            int cnt = 0;
            for (int q = 0; q < nr; ++q) cnt += (x > 0 ? r[q][x - 1] : 0) + (x < cx ? r[q][x] : 0);
            if (cnt == 0) continue;
            if (cnt < full) {
              out[x] = kHang;
              continue;
            }
            uint8_t c = kDof;
            bool finer = false;
            if (F) {
              const int X = 3 * gx - F->lo[0], Y = 3 * gy - F->lo[1], Z = d == 3 ? 3 * gz - F->lo[2] : 0;
              if (X >= 0 && Y >= 0 && Z >= 0 && X < fx && Y < fy && Z < fz)
                finer = (F->vcls[(size_t(Z) * fy + Y) * fx + X] & kDof) != 0;
            }
            if (!finer) {
              c |= kComp;
              ++k;
            }
            out[x] = c;
          }
        }
        part[z] = k;
      }
    });
    for (size_t k : part) t.composite += k;
  }
  for (int l = lmin; l <= L; ++l) {
    AdaptHostLevel& A = t.lev[l];
    make_runs(A.vcls, uint8_t(kDof | kHang), A.run);
    make_runs(A.vcls, kHang, A.hrun);
  }
  return "";
}

}  // namespace adafac
