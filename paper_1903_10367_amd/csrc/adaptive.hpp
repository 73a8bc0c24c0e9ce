// Adaptive spacetrees (Sec. 2.1): ragged levels stored as bounding-box patches of the level
// lattice, with a class byte per vertex and a leaf byte per cell.  Shared by the host set-up
// (adaptive.cpp) and the gfx950 kernels (kernels_adaptive.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "adafac_internal.hpp"

namespace adafac {

// vertex class bits
constexpr uint8_t kDof = 1;        // all 2^d level cells around it exist, interior
constexpr uint8_t kHang = 2;       // vertex of an existing cell, interior, not a dof
constexpr uint8_t kComp = 4;       // dof whose finest dof level is this one (composite dof)

// Device view of one ragged level: the box [o, o + m) of the level's vertex lattice (m = 1
// along z in 2D); cells of the box are the (m - 1)^d cells between its vertices.
struct AdaptLevel {
  int ox, oy, oz, mx, my, mz;
  int n;                    // cells per axis of the whole level
  double h, hd, hdm2;       // h, h^d, h^(d-2)
  int fem;                  // 1: Q1 operator from eps blocks; 0: stored diagonal (uniform Galerkin level)
  int nb, bs;               // eps blocks per axis, cells per block along an axis
  const double* eps;        // nb^d blocks, nullptr: eps = 1
  const double* dg;         // stored diagonal over the box when !fem
  const uint8_t* vcls;      // per box vertex
  const uint8_t* leaf;      // per box cell: 0 = no cell, 1 = leaf cell, 2 = refined cell
  const double* bleaf;      // lumped load of the level's leaf cells at box vertices
  double* u;                // nodal values: composite dofs, copies of finer dofs, hanging interpolations
  double* bb;               // leaf residual, then the level hats tested against the composite residual
  double* hh;               // hanging-only accumulation (composite residual of coarser dofs)
  double* s;                // own correction c - c~ at dofs
  double* S;                // prolongated sum of corrections
};

// All levels of a tree (the old one of a regrid) and the finest-lattice spacing of each level.
struct AdaptTreeView {
  AdaptLevel lv[kMaxLevel + 1];
  int scale[kMaxLevel + 1];    // 3^(L - l)
  int lmin, L;
};

// Host description of the tree.
struct AdaptHostLevel {
  int d = 2;
  int lo[3] = {0, 0, 0}, nc[3] = {1, 1, 1};   // cell box: cells lo .. lo + nc - 1 per axis (nc[2] = 1 in 2D)
  std::vector<uint8_t> exists, refined;        // over the cell box
  std::vector<uint8_t> vcls;                   // over the vertex box (nc + 1 per axis)
  std::vector<double> dg;                      // stored diagonal (Galerkin levels), vertex box
  size_t nverts() const;
  size_t ncells() const;
};

struct AdaptHost {
  int d = 2, lmin = 1, L = 1;
  std::vector<AdaptHostLevel> lev;             // indexed by level
  size_t composite = 0;                        // number of composite dofs
};

// Refinement flags of one level: over the full (3^l)^d cell lattice, C order (x fastest).
struct RefineSpec {
  int level;
  std::vector<uint8_t> flags;
};

// Builds the ragged levels lmin..L: levels below the first flagged level are fully refined.
// ball (centre, radius, l_from) is used for levels l_from..L-1 without explicit flags when
// radius > 0.  Returns "" or a message.
std::string build_adapt_tree(AdaptHost& t, int d, int lmin, int L, const std::vector<RefineSpec>& flags,
                             const double* centre, double radius, int l_from);

// Device launchers (kernels_adaptive.hip).  Every level l is given with its next coarser
// (C) or finer (F) neighbour level where the step needs it.
hipError_t launch_ad_hang(int d, const AdaptLevel& L, const AdaptLevel& C, hipStream_t s);
hipError_t launch_ad_leaf(int d, const AdaptLevel& L, hipStream_t s);
hipError_t launch_ad_up(int d, const AdaptLevel& L, const AdaptLevel* F, const RtSep<double>& rts, double omega,
                        double omega_t, int damping, double* partials, hipStream_t s);
hipError_t launch_ad_down(int d, const AdaptLevel& L, const AdaptLevel* C, hipStream_t s);
hipError_t launch_ad_update(int d, const AdaptLevel& L, const AdaptLevel* F, hipStream_t s);
hipError_t launch_ad_transfer(int d, const AdaptLevel& A, int scale, const AdaptTreeView& O, hipStream_t s);
constexpr int kAdaptNormBlocks = 256;   // norm partial blocks per level

}  // namespace adafac
