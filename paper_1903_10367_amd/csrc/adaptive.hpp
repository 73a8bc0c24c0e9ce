// Adaptive spacetrees (Sec. 2.1): ragged levels stored as bounding-box patches of the level
// lattice, with a class byte per vertex and a leaf byte per cell.  Shared by the host set-up
// (adaptive.cpp) and the gfx950 kernels (kernels_adaptive.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <algorithm>
#include <string>
#include <thread>
#include <vector>

#include "adafac_internal.hpp"

namespace adafac {

// vertex class bits
constexpr uint8_t kDof = 1;        // all 2^d level cells around it exist, interior
constexpr uint8_t kHang = 2;       // vertex of an existing cell, interior, not a dof
constexpr uint8_t kComp = 4;       // dof whose finest dof level is this one (composite dof)

// Device view of one ragged level in the arithmetic of T: the box [o, o + m) of the level's
// vertex lattice (m = 1 along z in 2D); cells of the box are the (m - 1)^d cells between its
// vertices.
template <typename T>
struct AdaptLevelT {
  int ox, oy, oz, mx, my, mz;
  int n;                    // cells per axis of the whole level
  T h, hd, hdm2;            // h, h^d, h^(d-2)
  int fem;                  // 1: Q1 operator from eps blocks; 0: stored diagonal (uniform Galerkin level)
  int nb, bs;               // eps blocks per axis, cells per block along an axis
  const T* eps;             // nb^d blocks, nullptr: eps = 1
  T* dg;                    // diagonal at the dofs (uploaded on Galerkin levels, set-up kernel otherwise)
  T* wc;                    // per box cell: eps_c h^(d-2) on leaf cells, 0 elsewhere (set-up kernel)
  const uint8_t* vcls;      // per box vertex
  const uint8_t* leaf;      // per box cell: 0 = no cell, 1 = leaf cell, 2 = refined cell
  T* bleaf;                 // lumped load of the level's leaf cells (inner form: the outer defect)
  T* u;                     // nodal values: composite dofs, copies of finer dofs, hanging interpolations
  T* bb;                    // leaf residual, then the level hats tested against the composite residual
  T* hh;                    // hanging-only accumulation (composite residual of coarser dofs)
  T* s;                     // own correction c - c~ at dofs
  T* S;                     // prolongated sum of corrections
  const T* pw;              // BoxMG transfer from the next coarser level into this one (a complete level):
                            // 2^d weights per vertex of the corners of its coarse cell, or nullptr: d-linear
  const uint2* run;         // runs (first box vertex, count <= 64) covering every dof and hanging vertex
  const uint2* hrun;        // the same for the hanging vertices alone
  unsigned nrun, nhrun;
};
using AdaptLevel = AdaptLevelT<double>;

// All levels of a tree (the old one of a regrid) and the finest-lattice spacing of each level.
struct AdaptTreeView {
  AdaptLevel lv[kMaxLevel + 1];
  int scale[kMaxLevel + 1];    // 3^(L - l)
  int lmin, L;
};

// Where the nodal values of a tree's levels live, for the copies of a level's updated dofs into
// the coinciding dofs of the coarser levels (every level-l dof is a dof of level l-1 where the
// position lies on the coarser lattice).
template <typename T>
struct AdaptCopyView {
  struct Lv {
    int ox, oy, oz, mx, my, mz;
    const uint8_t* vcls;
    T* u;
  };
  Lv lv[kMaxLevel + 1];
  int lmin;
};

// Host description of the tree.
struct AdaptHostLevel {
  int d = 2;
  int lo[3] = {0, 0, 0}, nc[3] = {1, 1, 1};   // cell box: cells lo .. lo + nc - 1 per axis (nc[2] = 1 in 2D)
  std::vector<uint8_t> exists, refined;        // over the cell box
  std::vector<uint8_t> vcls;                   // over the vertex box (nc + 1 per axis)
  std::vector<double> dg;                      // stored diagonal (Galerkin levels), vertex box
  // runs of the vertex box, (first index, count) pairs in box order, disjoint, each at most 64
  // vertices from a multiple of 16 on: every dof or hanging vertex (run), every hanging vertex
  // (hrun).  The per-vertex kernels walk these instead of the whole box.
  std::vector<uint32_t> run, hrun;
  size_t nverts() const;
  size_t ncells() const;
};

struct AdaptHost {
  int d = 2, lmin = 1, L = 1;
  std::vector<AdaptHostLevel> lev;             // indexed by level
  size_t composite = 0;                        // number of composite dofs
};

// f(lo, hi) over [0, n) on up to 16 host threads, one contiguous range each (host set-up of
// boxes with 10^7 cells and vertices).
template <class F>
void parallel_ranges(size_t n, F&& f) {
  unsigned nt = std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
  if (n < 2 || nt == 1) {
    f(size_t(0), n);
    return;
  }
  nt = unsigned(std::min<size_t>(nt, n));
  std::vector<std::thread> th;
  th.reserve(nt);
  for (unsigned k = 0; k < nt; ++k) th.emplace_back([&f, n, nt, k] { f(n * k / nt, n * (k + 1) / nt); });
  for (auto& t : th) t.join();
}

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
template <typename T>
hipError_t launch_ad_hang(int d, const AdaptLevelT<T>& L, const AdaptLevelT<T>& C, hipStream_t s, Gate g = Gate{});
// Levels with a finer level F (F must not be null; the finest level runs launch_ad_leaf_up): the
// level's own leaf residual (computed in place) plus the restrictions from F.
// norms_only: only the composite residual: norm partials, hh, and bb replaced by the composite
// residual at composite dofs (zero elsewhere)
// tiled: the 3D tiled kernel (adapt_up_tiled), else the five-wave gathers
template <typename T>
hipError_t launch_ad_up(int d, const AdaptLevelT<T>& L, const AdaptLevelT<T>* F, const RtSep<T>& rts, T omega,
                        T omega_t, int damping, int norms_only, int tiled, double* partials, hipStream_t s,
                        Gate g = Gate{});
// The finest level: leaf residual and up in one pass
template <typename T>
hipError_t launch_ad_leaf_up(int d, const AdaptLevelT<T>& L, T omega, T omega_t, int norms_only, double* partials,
                             hipStream_t s, Gate g = Gate{});
// Down and update of level `level` (L; C the next coarser level, null on the coarsest): the
// prolongated sum S, u += S at the composite dofs, and those values copied into the coinciding
// dofs of every coarser level (V).  Launched coarsest level first.  keep_s: store S (every level
// but the finest, whose S feeds no finer level).
template <typename T>
hipError_t launch_ad_down_update(int d, const AdaptLevelT<T>& L, const AdaptLevelT<T>* C, const AdaptCopyView<T>& V,
                                 int level, int pi, int keep_s, hipStream_t s, Gate g = Gate{});
// once per tree, after the classes, leaf flags and (Galerkin levels) diagonals are uploaded
template <typename T>
hipError_t launch_ad_setup(int d, const AdaptLevelT<T>& L, hipStream_t s);
hipError_t launch_ad_transfer(int d, const AdaptLevel& A, int scale, const AdaptTreeView& O, hipStream_t s);
// Gaussian source amp exp(-|x - c|^2 / (2 sigma^2)) (x first in c)
struct GaussSource {
  double c[3];
  double sigma, amp;
};
// lumped leaf loads of a Gaussian source on level A (classes and cell bytes uploaded)
hipError_t launch_ad_gauss_load(int d, const AdaptLevel& A, const GaussSource& g, hipStream_t s);
// FP32 inner form: bleaf32 = float(bb), the composite residual of the FP64 iterate at its
// composite dofs (the inner loads), inner iterate e = 0
hipError_t launch_ad_to_inner(int d, const AdaptLevel& A, const AdaptLevelT<float>& E, hipStream_t s);
// u += e at every dof (composite dofs and their coarse copies)
hipError_t launch_ad_accumulate(int d, const AdaptLevel& A, const AdaptLevelT<float>& E, hipStream_t s);
#ifndef ADAFAC_AD_UP_MAX_BLOCKS
#define ADAFAC_AD_UP_MAX_BLOCKS 4096
#endif
constexpr int kAdaptNormBlocks = ADAFAC_AD_UP_MAX_BLOCKS;   // most blocks (norm partial slots) of an up launch
// g, rule: a pipelined solve's gate and stopping rule (see run_cycle)
hipError_t launch_ad_norm_finalize(const double* partials, int n, double* out, hipStream_t s, Gate g = Gate{},
                                   StopRule rule = StopRule{});
unsigned adapt_up_blocks(long box_vertices);     // blocks of an up launch without a finer level
unsigned adapt_up_blocks_f(long box_vertices);   // with one (2D)
unsigned adapt_up_blocks_tiled(int mx, int my, int mz);   // with one (3D, large levels)
// does a level with a finer one run tiled (3D, at least min_tiles tiles)?  FP64 only: in FP32 the
// per-vertex gathers move half the bytes and were measured faster than the tile march.
bool adapt_up_tiled(int d, int mx, int my, int mz, int min_tiles);
constexpr int kAdaptTiledMinTiles = 256;   // default: one tile per CU
// norm partial slots of a level's up launch (box of mx x my x mz vertices)
unsigned adapt_up_slots(int d, int mx, int my, int mz, bool has_finer, bool tiled);
constexpr long kAdaptMaxBox = (1L << 31) - 1;   // vertices (and cells) of one level's box

}  // namespace adafac
