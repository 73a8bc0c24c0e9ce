// gfx950 kernels of the adAFAC cycle on adaptive spacetrees (ragged levels with hanging
// vertices; Sec. 2.1, 2.3, 2.4; eq. (adaFACx) / Algorithm 1 over the generating system).
// One thread per vertex of a level's box (grid-stride; box indices fit 31 bits).  Per cycle:
//   hang    hanging vertices take the d-linear interpolation of the next coarser level
//   leaf    residual of the level's leaf cells (element-wise Q1, lumped load)
//   up      finest to coarsest: b_l = r^leaf_l + R b_{l+1} (the level hats tested against the
//           composite residual), the hanging-only part that forms the composite residual at
//           the composite dofs (norm partials), and the corrections c - c~ at the dofs
//   down    coarsest to finest: S_l = (c - c~)_l + P S_{l-1}
//   update  finest to coarsest: composite dofs u += S, other dofs copy the finer dof
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "adafac.h"
#include "adafac_internal.hpp"
#include "adaptive.hpp"
#include "kernels_common.hpp"

namespace adafac {
namespace {

constexpr int NTA = 256;

// Grid-stride over the box: at any time the whole grid works on one contiguous window of it,
// so the rows and planes a stencil reads are shared through the caches.  (One contiguous
// eighth of the box per XCD, for L2 locality, measured slower for every kernel here.)
#define AD_LOOP(i, nb) for (unsigned i = blockIdx.x * NTA + threadIdx.x; i < (nb); i += gridDim.x * NTA)

// One wavefront per run of the level's run list (box vertices run.x .. run.x + run.y - 1, at
// most 64), runs taken in box order by the grid as a whole (the same cache sharing of rows and
// planes as above), empty corners of the box never read.  The body sees box vertex i and may
// `continue` to the next run.
#define AD_RUNS(i, RUNS, NRUN)                                                                  \
  for (unsigned q_ = blockIdx.x * (NTA / 64) + (threadIdx.x >> 6); q_ < (NRUN);                 \
       q_ += gridDim.x * (NTA / 64))                                                            \
    for (unsigned i = (RUNS)[q_].x + (threadIdx.x & 63), e_ = (RUNS)[q_].x + (RUNS)[q_].y; i < e_; i = e_)

template <int D, typename L>
__device__ __forceinline__ long vidx(const L& A, int x, int y, int z) {
  x -= A.ox;
  y -= A.oy;
  z -= A.oz;
  if (x < 0 || x >= A.mx || y < 0 || y >= A.my) return -1;
  if (D == 3 && (z < 0 || z >= A.mz)) return -1;
  return (long(D == 3 ? z : 0) * A.my + y) * A.mx + x;
}

template <int D, typename L>
__device__ __forceinline__ long cidx(const L& A, int cx, int cy, int cz) {
  cx -= A.ox;
  cy -= A.oy;
  cz -= A.oz;
  if (cx < 0 || cx >= A.mx - 1 || cy < 0 || cy >= A.my - 1) return -1;
  if (D == 3 && (cz < 0 || cz >= A.mz - 1)) return -1;
  return (long(D == 3 ? cz : 0) * (A.my - 1) + cy) * (A.mx - 1) + cx;
}

template <int D, typename L>
__device__ __forceinline__ unsigned nbox(const L& A) {
  return unsigned(A.mx) * unsigned(A.my) * unsigned(D == 3 ? A.mz : 1);
}

// box-relative coordinates of box vertex i (32-bit division: the host keeps boxes below 2^31)
template <int D, typename L>
__device__ __forceinline__ void box_coords(const L& A, unsigned i, int& bx, int& by, int& bz) {
  const unsigned mx = unsigned(A.mx), q = i / mx;
  bx = int(i - q * mx);
  if (D == 3) {
    const unsigned my = unsigned(A.my), r = q / my;
    by = int(q - r * my);
    bz = int(r);
  } else {
    by = int(q);
    bz = 0;
  }
}

template <int D, typename L>
__device__ __forceinline__ void coords(const L& A, unsigned i, int& x, int& y, int& z) {
  box_coords<D>(A, i, x, y, z);
  x += A.ox;
  y += A.oy;
  z += D == 3 ? A.oz : 0;
}

template <typename T>
__device__ __forceinline__ T eps_of(const AdaptLevelT<T>& A, int cx, int cy, int cz, int d) {
  if (!A.eps) return T(1);
  const int bx = cx / A.bs, by = cy / A.bs, bz = cz / A.bs;
  return d == 2 ? A.eps[by * A.nb + bx] : A.eps[(bz * A.nb + by) * A.nb + bx];
}

// d-linear interpolation weight of coarse corner e at fine offset s (0..3 along each axis)
template <typename T>
__device__ __forceinline__ T lin3(int s, int e) { return e ? T(s) * T(1.0 / 3.0) : T(3 - s) * T(1.0 / 3.0); }

template <int D, typename T>
__device__ __forceinline__ T interp(const AdaptLevelT<T>& C, const T* v, int x, int y, int z) {
  const int nc = C.n;
  const int cx = min(x / 3, nc - 1), cy = min(y / 3, nc - 1), cz = D == 3 ? min(z / 3, nc - 1) : 0;
  const int sx = x - 3 * cx, sy = y - 3 * cy, sz = z - 3 * cz;
  T acc = T(0);
#pragma unroll
  for (int e = 0; e < (1 << D); ++e) {
    const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
    T w = lin3<T>(sx, ex) * lin3<T>(sy, ey);
    if (D == 3) w *= lin3<T>(sz, ez);
    if (w == T(0)) continue;
    const long k = vidx<D>(C, cx + ex, cy + ey, cz + ez);
    if (k >= 0) acc += w * v[k];
  }
  return acc;
}

// S_C at coarse vertex k = (X, Y, Z) of level C, less (adAFAC-PI) the injected correction of
// level A there: c_A at the coinciding level-A vertex when k is a dof of C (A.s holds c at the
// dofs of A under PI, zero elsewhere).
template <int D, typename T, bool PI>
__device__ __forceinline__ T coarse_sum(const AdaptLevelT<T>& A, const AdaptLevelT<T>& C, long k, int X, int Y,
                                        int Z) {
  T v = C.S[k];
  if (PI && (C.vcls[k] & kDof)) {
    const long kf = vidx<D>(A, 3 * X, 3 * Y, 3 * Z);
    if (kf >= 0) v -= A.s[kf];
  }
  return v;
}

// P (S_C - I c_A) at vertex i = (x, y, z) of level A (PI; else P S_C): stored BoxMG weights on
// complete levels that carry them (the box is the whole lattice there), else d-linear weights.
template <int D, typename T, bool PI>
__device__ __forceinline__ T prolong_at(const AdaptLevelT<T>& A, const AdaptLevelT<T>& C, unsigned i, int x, int y,
                                        int z) {
  const int nc = C.n;
  const int cx = min(x / 3, nc - 1), cy = min(y / 3, nc - 1), cz = D == 3 ? min(z / 3, nc - 1) : 0;
  const int sx = x - 3 * cx, sy = y - 3 * cy, sz = z - 3 * cz;
  T acc = T(0);
#pragma unroll
  for (int e = 0; e < (1 << D); ++e) {
    const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
    T w;
    if (A.pw) {
      w = A.pw[size_t(i) * (1 << D) + e];
    } else {
      w = lin3<T>(sx, ex) * lin3<T>(sy, ey);
      if (D == 3) w *= lin3<T>(sz, ez);
    }
    if (w == T(0)) continue;
    const long k = vidx<D>(C, cx + ex, cy + ey, cz + ez);
    if (k >= 0) acc += w * coarse_sum<D, T, PI>(A, C, k, cx + ex, cy + ey, cz + ez);
  }
  return acc;
}

// R = P^T weight of fine vertex k = (fx, fy, fz) of level F for coarse vertex (x, y, z): the
// stored BoxMG weight of that coarse corner of the fine vertex's coarse cell.
template <int D, typename T>
__device__ __forceinline__ T stored_rweight(const AdaptLevelT<T>& F, long k, int fx, int fy, int fz, int x, int y,
                                            int z, int nc) {
  const int ex = x - min(fx / 3, nc - 1), ey = y - min(fy / 3, nc - 1), ez = D == 3 ? z - min(fz / 3, nc - 1) : 0;
  if (ex < 0 || ex > 1 || ey < 0 || ey > 1 || ez < 0 || ez > 1) return T(0);
  return F.pw[size_t(k) * (1 << D) + (ex | (ey << 1) | (ez << 2))];
}

// Q1 diagonal at a dof (all 2^d cells exist): kref h^(d-2) sum of the cells' eps
template <int D, typename T>
__device__ __forceinline__ T fem_diag(const AdaptLevelT<T>& A, int x, int y, int z) {
  T es = T(0);
#pragma unroll
  for (int e = 0; e < (1 << D); ++e) {
    const int cx = x - 1 + (e & 1), cy = y - 1 + ((e >> 1) & 1), cz = D == 3 ? z - 1 + ((e >> 2) & 1) : 0;
    es += eps_of(A, cx, cy, cz, D);
  }
  return T(D == 2 ? 2.0 / 3.0 : 1.0 / 3.0) * A.hdm2 * es;
}

// Q1 reference element entry between corners i and j (bit a = offset along axis a)
template <int D, typename T>
__device__ __forceinline__ T kref(int i, int j) {
  const int hd = __popc(unsigned(i ^ j));
  if (D == 2) return hd == 0 ? T(2.0 / 3.0) : (hd == 1 ? T(-1.0 / 6.0) : T(-1.0 / 3.0));
  return hd == 0 ? T(1.0 / 3.0) : (hd == 1 ? T(0) : T(-1.0 / 12.0));
}

template <int D, typename T, bool G>
__global__ void __launch_bounds__(NTA) k_ad_hang(AdaptLevelT<T> A, AdaptLevelT<T> C, Gate g) {
  if (G && gated(g)) return;
  AD_RUNS(i, A.hrun, A.nhrun) {
    if (!(A.vcls[i] & kHang)) continue;
    int x, y, z;
    coords<D>(A, i, x, y, z);
    A.u[i] = interp<D>(C, C.u, x, y, z);
  }
}

// Set-up of a level (once per tree): the leaf-cell weights eps_c h^(d-2) (zero on cells that
// are not leaves) and, on levels with the Q1 operator, the diagonal at the dofs.
template <int D, typename T>
__global__ void __launch_bounds__(NTA) k_ad_setup(AdaptLevelT<T> A) {
  const unsigned cmx = unsigned(A.mx - 1), cmy = unsigned(A.my - 1);
  const unsigned nc = cmx * cmy * unsigned(D == 3 ? A.mz - 1 : 1);
  AD_LOOP(c, nc) {
    const unsigned q = c / cmx;
    const int cx = A.ox + int(c - q * cmx);
    const int cy = A.oy + int(D == 3 ? q % cmy : q);
    const int cz = D == 3 ? A.oz + int(q / cmy) : 0;
    A.wc[c] = A.leaf[c] == 1 ? eps_of(A, cx, cy, cz, D) * A.hdm2 : T(0);
  }
  if (!A.fem) return;
  const unsigned nb = nbox<D>(A);
  AD_LOOP(i, nb) {
    int x, y, z;
    coords<D>(A, i, x, y, z);
    A.dg[i] = (A.vcls[i] & kDof) ? fem_diag<D>(A, x, y, z) : T(0);
  }
}

// Leaf residual at a vertex whose 3^d neighbours lie in the box: the 2^d cell weights folded
// into the coefficients of the 3^d neighbours (the zero entries of the reference element drop
// out at compile time).
template <int D, typename T>
__device__ __forceinline__ T leaf_inner(const AdaptLevelT<T>& A, unsigned i, int bx, int by, int bz, T r) {
  const long cmx = A.mx - 1, cmy = A.my - 1;
  const long c0 = (long(D == 3 ? bz - 1 : 0) * cmy + (by - 1)) * cmx + (bx - 1);
  T w[1 << D];
#pragma unroll
  for (int e = 0; e < (1 << D); ++e)
    w[e] = A.wc[c0 + (e & 1) + ((e >> 1) & 1) * cmx + (D == 3 ? ((e >> 2) & 1) * cmx * cmy : 0)];
  const long sy = A.mx, sz = long(A.mx) * A.my;
  constexpr int NO = D == 2 ? 9 : 27;
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = D == 3 ? o / 9 - 1 : 0;
    T cf = T(0);
    bool any = false;
#pragma unroll
    for (int e = 0; e < (1 << D); ++e) {
      // cell e has lower corner v - 1 + e; its corner j sits at offset e + j - 1 from v
      const int jx = ox + 1 - (e & 1), jy = oy + 1 - ((e >> 1) & 1), jz = D == 3 ? oz + 1 - ((e >> 2) & 1) : 0;
      if (jx < 0 || jx > 1 || jy < 0 || jy > 1 || jz < 0 || jz > 1) continue;
      const T k = kref<D, T>(e ^ ((1 << D) - 1), jx | (jy << 1) | (jz << 2));
      if (k == T(0)) continue;
      cf += k * w[e];
      any = true;
    }
    if (any) r -= cf * A.u[long(i) + ox + oy * sy + oz * sz];
  }
  return r;
}

// Leaf residual at box vertex i of class dof or hanging (such vertices are interior).
template <int D, typename T>
__device__ __forceinline__ T leaf_residual(const AdaptLevelT<T>& A, unsigned i) {
  const int cmx = A.mx - 1, cmy = A.my - 1, cmz = D == 3 ? A.mz - 1 : 1;
  int bx, by, bz;
  box_coords<D>(A, i, bx, by, bz);
  T r = A.bleaf[i];
  if (bx >= 1 && bx < cmx && by >= 1 && by < cmy && (D == 2 || (bz >= 1 && bz < cmz))) return leaf_inner<D>(A, i, bx, by, bz, r);
#pragma unroll
  for (int e = 0; e < (1 << D); ++e) {
    // cell with lower corner v - 1 + e (box-relative); this vertex is its corner iw
    const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
    const int cx = bx - 1 + ex, cy = by - 1 + ey, cz = D == 3 ? bz - 1 + ez : 0;
    if (cx < 0 || cx >= cmx || cy < 0 || cy >= cmy || cz < 0 || cz >= cmz) continue;
    const T wv = A.wc[(long(cz) * cmy + cy) * cmx + cx];
    if (wv == T(0)) continue;
    const int iw = e ^ ((1 << D) - 1);
    T sum = T(0);
#pragma unroll
    for (int j = 0; j < (1 << D); ++j) {
      const long k = (long(cz + ((j >> 2) & 1)) * A.my + (cy + ((j >> 1) & 1))) * A.mx + (cx + (j & 1));
      sum += kref<D, T>(iw, j) * A.u[k];
    }
    r -= wv * sum;
  }
  return r;
}

// Vertices of class 0 (no existing cell, or the domain boundary) are never written: their
// arrays hold the zeros of the workspace set-up, which is what every reader expects there.

// d-linear restriction weight of fine offset o (|o| <= 2)
template <typename T>
__device__ __forceinline__ T wl(int o) { return o == 0 ? T(1) : (o == 1 || o == -1) ? T(2.0 / 3.0) : T(1.0 / 3.0); }

template <typename T>
__device__ __forceinline__ T sel5(const RtSep<T>& r, int o) {
  return o == -2 ? r.m[0] : o == -1 ? r.m[1] : o == 0 ? r.m[2] : o == 1 ? r.m[3] : r.m[4];
}

// R~ weight of fine offset o: scale sum_a delta(o_a) prod_{b != a} m(o_b) (selects, not an
// indexed load: the factors stay in registers)
template <int D, typename T>
__device__ __forceinline__ T rt_weight(const RtSep<T>& rts, int ox, int oy, int oz) {
  const T mx = sel5(rts, ox), my = sel5(rts, oy);
  T wt;
  if (D == 2) {
    wt = (ox == 0 ? my : T(0)) + (oy == 0 ? mx : T(0));
  } else {
    const T mz = sel5(rts, oz);
    wt = (ox == 0 ? my * mz : T(0)) + (oy == 0 ? mx * mz : T(0)) + (oz == 0 ? mx * my : T(0));
  }
  return rts.scale * wt;
}

// One plane (fixed oz) of the 5^d fine neighbourhood at fixed offsets from k: the d-linear
// restriction weights wl(ox) wl(oy) of hh and bb, and the R~ terms.  pa collects the terms
// with ox = 0 or oy = 0 (factor m(oz) applied by the caller), pc those with oz = 0 (CENTRE).
// Per vertex, after the restrictions from the finer level: the hanging-only accumulation, the
// composite residual (norms), b_l and the correction c - c~ at the dofs.
template <typename T, int MODE>
__device__ __forceinline__ void up_finish(const AdaptLevelT<T>& A, unsigned i, uint8_t cls, T rl, T Rh, T Rb, T Rt,
                                          int has_f, T omega, T omega_t, double& ssum, double& smax) {
  const T acch = rl + Rh;
  A.hh[i] = (cls & kHang) ? acch : T(0);
  if (cls & kComp) {
    const double a = double(acch);
    ssum += double(A.hd) * a * a;
    smax = fmax(smax, fabs(a));
  }
  if (MODE == 0) {
    // the composite residual in place of the leaf residual (same index, read before)
    A.bb[i] = (cls & kComp) ? acch : T(0);
    return;
  }
  const T acc = rl + Rb;
  A.bb[i] = acc;
  T sv = T(0);
  if (cls & kDof) {
    const T dg = A.dg[i];
    sv = omega * acc / dg;
    if (MODE == 2 && has_f) sv -= omega_t * Rt / dg;
  }
  A.s[i] = sv;
}

// MODE: 0 composite residual only (norms_only), 1 plain additive, 2 adAFAC-Jac.
// The finest level (no finer level to restrict from): its leaf residual and the per-vertex tail
// in one pass, one thread per vertex.
template <int D, typename T, int MODE, bool G>
__global__ void __launch_bounds__(NTA) k_ad_leaf_up(AdaptLevelT<T> A, T omega, T omega_t, double* partials, Gate g) {
  if (G && gated(g)) return;
  double ssum = 0.0, smax = 0.0;
  AD_RUNS(i, A.run, A.nrun) {
    const uint8_t cls = A.vcls[i];
    if (!(cls & (kDof | kHang))) continue;
    up_finish<T, MODE>(A, i, cls, leaf_residual<D>(A, i), T(0), T(0), T(0), 0, omega, omega_t, ssum, smax);
  }
  block_norm_partials(ssum, smax, partials);
}

// Levels with a finer level: five waves per group of 64 coarse vertices, wave w gathering the
// fine plane oz = w - 2 (3D) or row oy = w - 2 (2D) of every vertex's 5^d neighbourhood; wave
// 0 adds the other waves' partial sums in a fixed order and finishes the vertices.  Five times
// the lanes of one thread per vertex, for the small levels whose gathers are latency bound.
constexpr int NTU = 320;

template <int D, typename T, int MODE, bool G>
__global__ void __launch_bounds__(NTU) k_ad_up_f(AdaptLevelT<T> A, AdaptLevelT<T> F, RtSep<T> rts, T omega,
                                                 T omega_t, double* partials, Gate g) {
  if (G && gated(g)) return;
  __shared__ T sh[3][4][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int o2 = wave - 2;                 // oz in 3D, oy in 2D
  double ssum = 0.0, smax = 0.0;
  // one group of (at most) 64 vertices per run of the level's run list
  for (unsigned g = blockIdx.x; g < A.nrun; g += gridDim.x) {
    const uint2 run = A.run[g];
    const unsigned i = run.x + lane;
    const uint8_t cls = unsigned(lane) < run.y ? A.vcls[i] : uint8_t(0);
    T Rh = T(0), Rb = T(0), Rt = T(0);
    if (cls & (kDof | kHang)) {
      int x, y, z;
      coords<D>(A, i, x, y, z);
      const int fx = 3 * x - F.ox, fy = 3 * y - F.oy, fz = D == 3 ? 3 * z - F.oz : 0;
      const bool tdof = MODE == 2 && (cls & kDof);
      const int oz = D == 3 ? o2 : 0;
      const T wz = D == 3 ? wl<T>(oz) : T(1);
      const T mz = D == 3 ? sel5(rts, oz) : T(1);
      if (!F.pw && fx >= 2 && fx + 2 < F.mx && fy >= 2 && fy + 2 < F.my && (D == 2 || (fz >= 2 && fz + 2 < F.mz))) {
        const long k0 = (long(fz) * F.my + fy) * F.mx + fx, sy = F.mx, sz = long(F.mx) * F.my;
        const int ylo = D == 3 ? -2 : o2, yhi = D == 3 ? 2 : o2;
#pragma unroll 1
        for (int oy = ylo; oy <= yhi; ++oy) {
          const long kr = k0 + oz * sz + oy * sy;
          const T* hh = F.hh + kr;
          T hr = T(0);
#pragma unroll
          for (int ox = -2; ox <= 2; ++ox) hr += wl<T>(ox) * hh[ox];
          const T wyz = wl<T>(oy) * wz;
          Rh += wyz * hr;
          if (MODE == 0) continue;
          const T* bb = F.bb + kr;
          T fb[5], br = T(0);
#pragma unroll
          for (int ox = -2; ox <= 2; ++ox) {
            fb[ox + 2] = bb[ox];
            br += wl<T>(ox) * fb[ox + 2];
          }
          Rb += wyz * br;
          if (MODE != 2 || !tdof) continue;
          // R~ over fine dofs: rows through the centre line use the whole row, others one tap
          const uint8_t* vc = F.vcls + kr;
          const T my = sel5(rts, oy);
          T rt = ((vc[0] & kDof) ? fb[2] : T(0)) * my * mz;
          if (oy == 0 || (D == 3 && oz == 0)) {
            T fm = T(0);
#pragma unroll
            for (int ox = -2; ox <= 2; ++ox) fm += rts.m[ox + 2] * ((vc[ox] & kDof) ? fb[ox + 2] : T(0));
            if (oy == 0) rt += fm * mz;
            if (D == 3 && oz == 0) rt += fm * my;
          }
          Rt += rts.scale * rt;
        }
      } else {
        const int ylo = D == 3 ? -2 : o2, yhi = D == 3 ? 2 : o2;
        for (int oy = ylo; oy <= yhi; ++oy)
          for (int ox = -2; ox <= 2; ++ox) {
            const long k = vidx<D>(F, 3 * x + ox, 3 * y + oy, 3 * z + oz);
            if (k < 0) continue;
            const T w = F.pw ? stored_rweight<D>(F, k, 3 * x + ox, 3 * y + oy, 3 * z + oz, x, y, z, A.n)
                             : wl<T>(ox) * wl<T>(oy) * wz;
            Rh += w * F.hh[k];
            if (MODE == 0) continue;
            const T fb = F.bb[k];
            Rb += w * fb;
            if (MODE == 2) Rt += rt_weight<D>(rts, ox, oy, oz) * ((tdof && (F.vcls[k] & kDof)) ? fb : T(0));
          }
      }
    }
    if (wave > 0) {
      sh[0][wave - 1][lane] = Rh;
      sh[1][wave - 1][lane] = Rb;
      sh[2][wave - 1][lane] = Rt;
    }
    __syncthreads();
    if (wave == 0 && (cls & (kDof | kHang))) {
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        Rh += sh[0][w][lane];
        Rb += sh[1][w][lane];
        Rt += sh[2][w][lane];
      }
      up_finish<T, MODE>(A, i, cls, leaf_residual<D>(A, i), Rh, Rb, Rt, 1, omega, omega_t, ssum, smax);
    }
    __syncthreads();
  }
  block_norm_partials(ssum, smax, partials);
}

// 3D levels with a finer level, tiled: a workgroup owns TCX x TCY coarse columns and TZC coarse
// planes of the box and marches the finer box through z once.  Per fine plane: the plane's part
// of the tile's 5^3 neighbourhoods is staged in LDS (hh, bb, and bb at fine dofs for R~), an x
// pass forms per fine row the d-linear and R~ sums of every coarse column, a y pass per coarse
// column the planar sums, which are added with their z weights into the (at most two) coarse
// planes the fine plane reaches (R = P^T and R~ are tensor-product sums).  Each fine value is
// read about 1.3 times instead of (5/3)^3 times by per-vertex gathers.
#ifndef ADAFAC_AD_TILE_ZC
#define ADAFAC_AD_TILE_ZC 6
#endif
constexpr int TCX = 16, TCY = 8, TZC = ADAFAC_AD_TILE_ZC, NTT = 256;
constexpr int FXW = 3 * TCX + 2, FYW = 3 * TCY + 2, NFT = FXW * FYW;

template <typename T, int MODE, bool G>
__global__ void __launch_bounds__(NTT) k_ad_up_tiled(AdaptLevelT<T> A, AdaptLevelT<T> F, RtSep<T> rts, T omega,
                                                     T omega_t, double* partials, Gate g) {
  if (G && gated(g)) return;
  __shared__ T Lh[NFT];
  __shared__ T Lb[MODE ? NFT : 1];
  __shared__ T Ld[MODE == 2 ? NFT : 1];
  __shared__ T Xh[FYW * TCX];
  __shared__ T Xb[MODE ? FYW * TCX : 1];
  __shared__ T Xd[MODE == 2 ? FYW * TCX : 1];
  __shared__ T Xm[MODE == 2 ? FYW * TCX : 1];
  const int tid = threadIdx.x;
  const int ntx = (A.mx + TCX - 1) / TCX, nty = (A.my + TCY - 1) / TCY;
  const int tx = blockIdx.x % ntx, ty = (blockIdx.x / ntx) % nty, tzc = blockIdx.x / (ntx * nty);
  const int bx0 = tx * TCX, by0 = ty * TCY, bz0 = tzc * TZC, bz1 = min(bz0 + TZC, A.mz);
  // finer-box coordinates of the tile's fine region (3 c - 2 .. 3 c + 2 around its columns)
  const int fx0 = 3 * (A.ox + bx0) - 2 - F.ox, fy0 = 3 * (A.oy + by0) - 2 - F.oy;
  // a tile whose coarse block holds no dof or hanging vertex writes nothing: only its (zero) norm
  // partials
  {
    int any = 0;
    for (int k = tid; k < TCX * TCY * TZC; k += NTT) {
      const int cx = bx0 + k % TCX, cy = by0 + (k / TCX) % TCY, cz = bz0 + k / (TCX * TCY);
      if (cx < A.mx && cy < A.my && cz < bz1 &&
          (A.vcls[(unsigned(cz) * unsigned(A.my) + unsigned(cy)) * unsigned(A.mx) + unsigned(cx)] & (kDof | kHang)))
        any = 1;
    }
    if (!__syncthreads_or(any)) {
      block_norm_partials(0.0, 0.0, partials);
      return;
    }
  }
  const bool item = tid < TCX * TCY;
  const int icx = tid % TCX, icy = tid / TCX;
  const int cbx = bx0 + icx, cby = by0 + icy;
  const bool in_xy = item && cbx < A.mx && cby < A.my;
  T aH[2] = {T(0), T(0)}, aB[2] = {T(0), T(0)}, aT[2] = {T(0), T(0)};
  double ssum = 0.0, smax = 0.0;
  const int fzs = 3 * (A.oz + bz0) - 2, fze = 3 * (A.oz + bz1 - 1) + 2;
  // this lane's staging items k = tid + j NTT: their offset inside a finer-box plane (-1: off the box)
  constexpr int NJ = (NFT + NTT - 1) / NTT;
  long off[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int k = tid + j * NTT;
    const int X = fx0 + k % FXW, Y = fy0 + k / FXW;
    off[j] = (k < NFT && X >= 0 && X < F.mx && Y >= 0 && Y < F.my) ? long(Y) * F.mx + X : -1;
  }
  const long fplane = long(F.mx) * F.my;
  // the next plane's values are loaded into registers while the current one is processed
  T ph[NJ], pb[NJ], pd[NJ];
  auto fetch = [&](int fz) {
    const int fzb = fz - F.oz;
    const bool zin = fzb >= 0 && fzb < F.mz;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      T h = T(0), b = T(0), dm = T(0);
      if (zin && off[j] >= 0) {
        const long f = fzb * fplane + off[j];
        h = F.hh[f];
        if (MODE) b = F.bb[f];
        if (MODE == 2) dm = (F.vcls[f] & kDof) ? b : T(0);
      }
      ph[j] = h;
      pb[j] = b;
      pd[j] = dm;
    }
  };
  fetch(fzs);
  for (int fz = fzs; fz <= fze; ++fz) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int k = tid + j * NTT;
      if (k < NFT) {
        Lh[k] = ph[j];
        if (MODE) Lb[k] = pb[j];
        if (MODE == 2) Ld[k] = pd[j];
      }
    }
    if (fz < fze) fetch(fz + 1);
    __syncthreads();
    for (int k = tid; k < FYW * TCX; k += NTT) {
      const int ly = k / TCX, cx = k % TCX;
      const int c = ly * FXW + 3 * cx + 2;
      T sh = T(0), sb = T(0), sm = T(0);
#pragma unroll
      for (int o = -2; o <= 2; ++o) {
        sh += wl<T>(o) * Lh[c + o];
        if (MODE) sb += wl<T>(o) * Lb[c + o];
        if (MODE == 2) sm += rts.m[o + 2] * Ld[c + o];
      }
      Xh[k] = sh;
      if (MODE) Xb[k] = sb;
      if (MODE == 2) {
        Xd[k] = Ld[c];
        Xm[k] = sm;
      }
    }
    __syncthreads();
    if (item) {
      T H = T(0), B = T(0), Aa = T(0), Cc = T(0);
#pragma unroll
      for (int o = -2; o <= 2; ++o) {
        const int r = (3 * icy + 2 + o) * TCX + icx;
        H += wl<T>(o) * Xh[r];
        if (MODE) B += wl<T>(o) * Xb[r];
        if (MODE == 2) {
          Aa += rts.m[o + 2] * Xd[r];
          Cc += rts.m[o + 2] * Xm[r];
        }
      }
      // R~ planes: [ox = 0] m(oy) m(oz) + [oy = 0] m(ox) m(oz) + [oz = 0] m(ox) m(oy)
      const T Bt = MODE == 2 ? Xm[(3 * icy + 2) * TCX + icx] : T(0);
      const int m = ((fz % 3) + 3) % 3, czlo = (fz - m) / 3;
      aH[0] += wl<T>(m) * H;
      if (MODE) aB[0] += wl<T>(m) * B;
      if (MODE == 2) aT[0] += rts.scale * (sel5(rts, m) * (Aa + Bt) + (m == 0 ? Cc : T(0)));
      if (m >= 1) {
        aH[1] += wl<T>(m - 3) * H;
        if (MODE) aB[1] += wl<T>(m - 3) * B;
        if (MODE == 2) aT[1] += rts.scale * sel5(rts, m - 3) * (Aa + Bt);
      }
      if (m == 2) {
        // coarse plane czlo has all five fine planes
        const int czb = czlo - A.oz;
        if (in_xy && czb >= bz0 && czb < bz1) {
          const unsigned i = (unsigned(czb) * unsigned(A.my) + unsigned(cby)) * unsigned(A.mx) + unsigned(cbx);
          const uint8_t cls = A.vcls[i];
          if (cls & (kDof | kHang))
            up_finish<T, MODE>(A, i, cls, leaf_residual<3>(A, i), aH[0], aB[0], aT[0], 1, omega, omega_t, ssum, smax);
        }
        aH[0] = aH[1];
        aB[0] = aB[1];
        aT[0] = aT[1];
        aH[1] = aB[1] = aT[1] = T(0);
      }
    }
  }
  block_norm_partials(ssum, smax, partials);
}

// The updated value of a composite dof at lattice point (x, y, z) of level l, copied into the dofs
// of the coarser levels that sit at the same position (their nodal values copy the finer one).
template <int D, typename T>
__device__ __forceinline__ void copy_down(const AdaptCopyView<T>& V, int l, int x, int y, int z, T val) {
  for (int m = l - 1; m >= V.lmin; --m) {
    if (x % 3 || y % 3 || (D == 3 && z % 3)) return;
    x /= 3;
    y /= 3;
    z /= 3;
    const typename AdaptCopyView<T>::Lv& C = V.lv[m];
    const int bx = x - C.ox, by = y - C.oy, bz = z - C.oz;
    if (bx < 0 || bx >= C.mx || by < 0 || by >= C.my || (D == 3 && (bz < 0 || bz >= C.mz))) return;
    const long k = (long(D == 3 ? bz : 0) * C.my + by) * C.mx + bx;
    if (!(C.vcls[k] & kDof)) return;
    C.u[k] = val;
  }
}

// S_l = (c - c~)_l + P S_{l-1}; adAFAC-PI: S_l = c_l + P (S_{l-1} - I c_l), which is
// c_l - P I c_l + P S_{l-1} (c~_l = P I c_l, Sec. 3.2).  Then u += S_l at the composite dofs,
// copied into the coinciding coarser dofs.
template <int D, typename T, bool PI, bool G>
__global__ void __launch_bounds__(NTA) k_ad_down_update(AdaptLevelT<T> A, AdaptLevelT<T> C, int has_c,
                                                        AdaptCopyView<T> V, int level, int keep_s, Gate g) {
  if (G && gated(g)) return;
  AD_RUNS(i, A.run, A.nrun) {
    const uint8_t cls = A.vcls[i];
    if (!(cls & (kDof | kHang))) continue;
    int x, y, z;
    coords<D>(A, i, x, y, z);
    T S = A.s[i];
    if (has_c) S += prolong_at<D, T, PI>(A, C, i, x, y, z);
    if (keep_s) A.S[i] = S;   // the finest level's S feeds no finer level
    if (cls & kComp) {
      const T nu = A.u[i] + S;
      A.u[i] = nu;
      copy_down<D>(V, level, x, y, z, nu);
    }
  }
}

// The composite FE function of tree O at finest-lattice point (X, Y, Z): d-linear interpolation
// in the finest existing cell of O that contains the point (Sec. 2.1: continuous Q1 on the
// leaves; refined cells are represented by their children).
template <int D>
__device__ double composite_at(const AdaptTreeView& O, int X, int Y, int Z) {
  int best = -1;
  long bc = -1;
  int cx = 0, cy = 0, cz = 0;
  for (int m = O.lmin; m <= O.L; ++m) {
    const AdaptLevel& A = O.lv[m];
    const int s = O.scale[m];
    const int qx = min(X / s, A.n - 1), qy = min(Y / s, A.n - 1), qz = D == 3 ? min(Z / s, A.n - 1) : 0;
    const long c = cidx<D>(A, qx, qy, qz);
    if (c < 0 || A.leaf[c] == 0) break;
    best = m;
    bc = c;
    cx = qx;
    cy = qy;
    cz = qz;
    if (A.leaf[c] == 1) break;
  }
  if (best < 0 || bc < 0) return 0.0;
  const AdaptLevel& A = O.lv[best];
  const int s = O.scale[best];
  const double fx = double(X - cx * s) / s, fy = double(Y - cy * s) / s, fz = D == 3 ? double(Z - cz * s) / s : 0.0;
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < (1 << D); ++e) {
    const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
    double w = (ex ? fx : 1.0 - fx) * (ey ? fy : 1.0 - fy);
    if (D == 3) w *= ez ? fz : 1.0 - fz;
    if (w == 0.0) continue;
    const long k = vidx<D>(A, cx + ex, cy + ey, cz + ez);
    if (k >= 0) acc += w * A.u[k];
  }
  return acc;
}

// New level A of a regridded tree: every dof takes the old tree's composite function.
template <int D>
__global__ void __launch_bounds__(NTA) k_ad_transfer(AdaptLevel A, int scale, AdaptTreeView O) {
  const unsigned nb = nbox<D>(A);
  AD_LOOP(i, nb) {
    if (!(A.vcls[i] & kDof)) continue;
    int x, y, z;
    coords<D>(A, i, x, y, z);
    A.u[i] = composite_at<D>(O, x * scale, y * scale, z * scale);
  }
}

// Lumped load of a Gaussian source on a level: m_v f(x_v) with m_v = |leaf cells around v| h^d / 2^d
// at dofs and hanging vertices (the set-up of the loads on the device, for the moving source).
template <int D>
__global__ void __launch_bounds__(NTA) k_ad_gauss_load(AdaptLevel A, GaussSource g) {
  const unsigned nb = nbox<D>(A);
  const int cmx = A.mx - 1, cmy = A.my - 1, cmz = D == 3 ? A.mz - 1 : 1;
  const double share = A.hd / double(1 << D);
  AD_LOOP(i, nb) {
    if (!(A.vcls[i] & (kDof | kHang))) continue;
    int bx, by, bz;
    box_coords<D>(A, i, bx, by, bz);
    int nleaf = 0;
#pragma unroll
    for (int e = 0; e < (1 << D); ++e) {
      const int cx = bx - 1 + (e & 1), cy = by - 1 + ((e >> 1) & 1), cz = D == 3 ? bz - 1 + ((e >> 2) & 1) : 0;
      if (cx < 0 || cx >= cmx || cy < 0 || cy >= cmy || cz < 0 || cz >= cmz) continue;
      nleaf += A.leaf[(long(cz) * cmy + cy) * cmx + cx] == 1;
    }
    double r2 = 0.0;
    const double px = (A.ox + bx) * A.h - g.c[0], py = (A.oy + by) * A.h - g.c[1];
    r2 = px * px + py * py;
    if (D == 3) {
      const double pz = (A.oz + bz) * A.h - g.c[2];
      r2 += pz * pz;
    }
    A.bleaf[i] = nleaf ? nleaf * share * g.amp * exp(-r2 / (2.0 * g.sigma * g.sigma)) : 0.0;
  }
}

// FP32 inner form of defect correction: the inner load is the FP64 leaf residual, the inner
// iterate starts at zero.
template <int D>
__global__ void __launch_bounds__(NTA) k_ad_to_inner(AdaptLevel A, AdaptLevelT<float> E) {
  AD_RUNS(i, A.run, A.nrun) {
    if (!(A.vcls[i] & (kDof | kHang))) continue;
    E.bleaf[i] = float(A.bb[i]);
    E.u[i] = 0.f;
  }
}

template <int D>
__global__ void __launch_bounds__(NTA) k_ad_accumulate(AdaptLevel A, AdaptLevelT<float> E) {
  AD_RUNS(i, A.run, A.nrun)
    if (A.vcls[i] & kDof) A.u[i] += double(E.u[i]);
}

unsigned blocks_of(long n, long per_block, long cap) {
  long g = (n + per_block - 1) / per_block;
  return unsigned(g < cap ? (g < 1 ? 1 : g) : cap);
}

unsigned grid_for(long nb) { return blocks_of(nb, NTA, 8192); }
// one wavefront per run
unsigned grid_runs(unsigned nrun) { return blocks_of(long(nrun), NTA / 64, 8192); }

}  // namespace

// Norms from the packed partials of all levels: one workgroup of 1024 lanes, fixed order.
template <bool G>
__global__ void __launch_bounds__(1024) k_ad_norm_finalize(const double* __restrict__ partials, int n,
                                                            double* __restrict__ out, Gate g, StopRule rule) {
  if (G && gated(g)) return;
  __shared__ double ss[16], sm[16];
  double sv = 0.0, mv = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    sv += partials[2 * i];
    mv = fmax(mv, partials[2 * i + 1]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sv += __shfl_xor(sv, off);
    mv = fmax(mv, __shfl_xor(mv, off));
  }
  if ((threadIdx.x & 63) == 0) {
    ss[threadIdx.x >> 6] = sv;
    sm[threadIdx.x >> 6] = mv;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < 16; ++w) {
      a += ss[w];
      b = fmax(b, sm[w]);
    }
    out[0] = sqrt(a);
    out[1] = b;
    if (G) apply_stop_rule(rule, out);
  }
}

hipError_t launch_ad_norm_finalize(const double* partials, int n, double* out, hipStream_t s, Gate g, StopRule rule) {
  if (g.stop || rule.stop)
    k_ad_norm_finalize<true><<<1, 1024, 0, s>>>(partials, n, out, g, rule);
  else
    k_ad_norm_finalize<false><<<1, 1024, 0, s>>>(partials, n, out, g, rule);
  return hipGetLastError();
}

unsigned adapt_up_blocks(long nb) { return blocks_of(nb, NTA, kAdaptNormBlocks); }

// tiles of the 3D up kernel: one workgroup per TCX x TCY x TZC coarse box block
unsigned adapt_up_blocks_tiled(int mx, int my, int mz) {
  return unsigned((mx + TCX - 1) / TCX) * unsigned((my + TCY - 1) / TCY) * unsigned((mz + TZC - 1) / TZC);
}

// The tiled kernel marches each tile's fine planes one after another; with fewer tiles than
// CUs (small levels) the five-wave gathers finish sooner.
bool adapt_up_tiled(int d, int mx, int my, int mz, int min_tiles) {
  return d == 3 && adapt_up_blocks_tiled(mx, my, mz) >= unsigned(min_tiles);
}

unsigned adapt_up_slots(int d, int mx, int my, int mz, bool has_finer, bool tiled) {
  const long nb = long(mx) * my * (d == 3 ? mz : 1);
  if (!has_finer) return adapt_up_blocks(nb);
  // a tiled level still runs the five-wave kernel in FP32 (its inner cycles)
  return tiled ? std::max(adapt_up_blocks_tiled(mx, my, mz), adapt_up_blocks_f(nb)) : adapt_up_blocks_f(nb);
}

// groups of 64 vertices per block of the five-wave up kernel
unsigned adapt_up_blocks_f(long nb) { return blocks_of(nb, 64, kAdaptNormBlocks); }

template <typename T>
hipError_t launch_ad_hang(int d, const AdaptLevelT<T>& A, const AdaptLevelT<T>& C, hipStream_t s, Gate g) {
#define AD_H(DD, GG) k_ad_hang<DD, T, GG><<<grid_runs(A.nhrun), NTA, 0, s>>>(A, C, g)
  if (d == 2) {
    if (g.stop) AD_H(2, true); else AD_H(2, false);
  } else {
    if (g.stop) AD_H(3, true); else AD_H(3, false);
  }
#undef AD_H
  return hipGetLastError();
}


template <typename T>
hipError_t launch_ad_up(int d, const AdaptLevelT<T>& A, const AdaptLevelT<T>* F, const RtSep<T>& rts, T omega,
                        T omega_t, int damping, int norms_only, int tiled, double* partials, hipStream_t s,
                        Gate g) {
  const bool gg = g.stop != nullptr;
  const AdaptLevelT<T> Fv = F ? *F : AdaptLevelT<T>{};
  const int mode = norms_only ? 0 : (damping == ADAFAC_DAMP_JAC ? 2 : 1);
  const long nbv = long(A.mx) * A.my * (d == 3 ? A.mz : 1);
  if (F && tiled) {
    if constexpr (std::is_same<T, double>::value) {
      if (d != 3) return hipErrorInvalidValue;
      const unsigned gt = adapt_up_blocks_tiled(A.mx, A.my, A.mz);
#define AD_UT(M, GG) k_ad_up_tiled<T, M, GG><<<gt, NTT, 0, s>>>(A, Fv, rts, omega, omega_t, partials, g)
      if (mode == 0) { if (gg) AD_UT(0, true); else AD_UT(0, false); }
      else if (mode == 1) { if (gg) AD_UT(1, true); else AD_UT(1, false); }
      else { if (gg) AD_UT(2, true); else AD_UT(2, false); }
#undef AD_UT
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;   // FP64 levels only
    }
  }
  if (F) {
    const unsigned gf = adapt_up_blocks_f(nbv);
#define AD_UPF(DD, M)                                                                          \
  do {                                                                                         \
    if (gg) k_ad_up_f<DD, T, M, true><<<gf, NTU, 0, s>>>(A, Fv, rts, omega, omega_t, partials, g);  \
    else k_ad_up_f<DD, T, M, false><<<gf, NTU, 0, s>>>(A, Fv, rts, omega, omega_t, partials, g);    \
  } while (0)
    if (d == 2) {
      if (mode == 0) AD_UPF(2, 0);
      else if (mode == 1) AD_UPF(2, 1);
      else AD_UPF(2, 2);
    } else {
      if (mode == 0) AD_UPF(3, 0);
      else if (mode == 1) AD_UPF(3, 1);
      else AD_UPF(3, 2);
    }
#undef AD_UPF
    return hipGetLastError();
  }
  return hipErrorInvalidValue;   // the finest level runs launch_ad_leaf_up
}

template <typename T>
hipError_t launch_ad_leaf_up(int d, const AdaptLevelT<T>& A, T omega, T omega_t, int norms_only, double* partials,
                             hipStream_t s, Gate g) {
  const unsigned nbk = adapt_up_blocks(long(A.mx) * A.my * (d == 3 ? A.mz : 1));
#define AD_LF(DD, M)                                                                    \
  do {                                                                                  \
    if (g.stop) k_ad_leaf_up<DD, T, M, true><<<nbk, NTA, 0, s>>>(A, omega, omega_t, partials, g);  \
    else k_ad_leaf_up<DD, T, M, false><<<nbk, NTA, 0, s>>>(A, omega, omega_t, partials, g);        \
  } while (0)
  if (d == 2) {
    if (norms_only) AD_LF(2, 0);
    else AD_LF(2, 1);
  } else {
    if (norms_only) AD_LF(3, 0);
    else AD_LF(3, 1);
  }
#undef AD_LF
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ad_down_update(int d, const AdaptLevelT<T>& A, const AdaptLevelT<T>* C, const AdaptCopyView<T>& V,
                                 int level, int pi, int keep_s, hipStream_t s, Gate g) {
  const AdaptLevelT<T> Cv = C ? *C : AdaptLevelT<T>{};
  const int hc = C ? 1 : 0;
  const int keep = keep_s ? 1 : 0;
#define AD_DU(DD, P)                                                                                          \
  do {                                                                                                        \
    if (g.stop) k_ad_down_update<DD, T, P, true><<<grid_runs(A.nrun), NTA, 0, s>>>(A, Cv, hc, V, level, keep, g); \
    else k_ad_down_update<DD, T, P, false><<<grid_runs(A.nrun), NTA, 0, s>>>(A, Cv, hc, V, level, keep, g);       \
  } while (0)
  if (d == 2) {
    if (pi) AD_DU(2, true);
    else AD_DU(2, false);
  } else {
    if (pi) AD_DU(3, true);
    else AD_DU(3, false);
  }
#undef AD_DU
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ad_setup(int d, const AdaptLevelT<T>& A, hipStream_t s) {
  const long nb = long(A.mx) * A.my * (d == 3 ? A.mz : 1);
  if (d == 2) k_ad_setup<2, T><<<grid_for(nb), NTA, 0, s>>>(A);
  else k_ad_setup<3, T><<<grid_for(nb), NTA, 0, s>>>(A);
  return hipGetLastError();
}

hipError_t launch_ad_transfer(int d, const AdaptLevel& A, int scale, const AdaptTreeView& O, hipStream_t s) {
  const long nb = long(A.mx) * A.my * (d == 3 ? A.mz : 1);
  if (d == 2) k_ad_transfer<2><<<grid_for(nb), NTA, 0, s>>>(A, scale, O);
  else k_ad_transfer<3><<<grid_for(nb), NTA, 0, s>>>(A, scale, O);
  return hipGetLastError();
}

hipError_t launch_ad_gauss_load(int d, const AdaptLevel& A, const GaussSource& g, hipStream_t s) {
  const long nb = long(A.mx) * A.my * (d == 3 ? A.mz : 1);
  if (d == 2) k_ad_gauss_load<2><<<grid_for(nb), NTA, 0, s>>>(A, g);
  else k_ad_gauss_load<3><<<grid_for(nb), NTA, 0, s>>>(A, g);
  return hipGetLastError();
}

hipError_t launch_ad_to_inner(int d, const AdaptLevel& A, const AdaptLevelT<float>& E, hipStream_t s) {
  if (d == 2) k_ad_to_inner<2><<<grid_runs(A.nrun), NTA, 0, s>>>(A, E);
  else k_ad_to_inner<3><<<grid_runs(A.nrun), NTA, 0, s>>>(A, E);
  return hipGetLastError();
}

hipError_t launch_ad_accumulate(int d, const AdaptLevel& A, const AdaptLevelT<float>& E, hipStream_t s) {
  if (d == 2) k_ad_accumulate<2><<<grid_runs(A.nrun), NTA, 0, s>>>(A, E);
  else k_ad_accumulate<3><<<grid_runs(A.nrun), NTA, 0, s>>>(A, E);
  return hipGetLastError();
}

#define ADAFAC_AD_INST(T)                                                                                         \
  template hipError_t launch_ad_hang<T>(int, const AdaptLevelT<T>&, const AdaptLevelT<T>&, hipStream_t, Gate);    \
  template hipError_t launch_ad_up<T>(int, const AdaptLevelT<T>&, const AdaptLevelT<T>*, const RtSep<T>&, T, T,  \
                                      int, int, int, double*, hipStream_t, Gate);                                 \
  template hipError_t launch_ad_setup<T>(int, const AdaptLevelT<T>&, hipStream_t);                              \
  template hipError_t launch_ad_leaf_up<T>(int, const AdaptLevelT<T>&, T, T, int, double*, hipStream_t, Gate);    \
  template hipError_t launch_ad_down_update<T>(int, const AdaptLevelT<T>&, const AdaptLevelT<T>*,                 \
                                               const AdaptCopyView<T>&, int, int, int, hipStream_t, Gate);
ADAFAC_AD_INST(double)
ADAFAC_AD_INST(float)

}  // namespace adafac
