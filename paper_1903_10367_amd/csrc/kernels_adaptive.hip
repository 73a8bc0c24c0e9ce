// gfx950 kernels of the adAFAC cycle on adaptive spacetrees (ragged levels with hanging
// vertices; Sec. 2.1, 2.3, 2.4; eq. (adaFACx) / Algorithm 1 over the generating system).
// One thread per vertex of a level's box.  Per cycle:
//   hang    hanging vertices take the d-linear interpolation of the next coarser level
//   leaf    residual of the level's leaf cells (element-wise Q1, lumped load)
//   up      finest to coarsest: b_l = r^leaf_l + R b_{l+1} (the level hats tested against the
//           composite residual), the hanging-only part that forms the composite residual at
//           the composite dofs (norm partials), and the corrections c - c~ at the dofs
//   down    coarsest to finest: S_l = (c - c~)_l + P S_{l-1}
//   update  finest to coarsest: composite dofs u += S, other dofs copy the finer dof
#include <hip/hip_runtime.h>

#include "adafac.h"
#include "adafac_internal.hpp"
#include "adaptive.hpp"
#include "kernels_common.hpp"

namespace adafac {
namespace {

constexpr int NTA = 256;

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
__device__ __forceinline__ long nbox(const L& A) {
  return long(A.mx) * A.my * (D == 3 ? A.mz : 1);
}

template <int D, typename L>
__device__ __forceinline__ void coords(const L& A, long i, int& x, int& y, int& z) {
  x = A.ox + int(i % A.mx);
  y = A.oy + int((i / A.mx) % A.my);
  z = D == 3 ? A.oz + int(i / (long(A.mx) * A.my)) : 0;
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

// Q1 diagonal at a dof (all 2^d cells exist): kref h^(d-2) sum of the cells' eps
template <int D, typename T>
__device__ __forceinline__ T diag_at(const AdaptLevelT<T>& A, long i, int x, int y, int z) {
  if (!A.fem) return A.dg[i];
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

template <int D, typename T>
__global__ void __launch_bounds__(NTA) k_ad_hang(AdaptLevelT<T> A, AdaptLevelT<T> C) {
  const long nb = nbox<D>(A);
  for (long i = long(blockIdx.x) * NTA + threadIdx.x; i < nb; i += long(gridDim.x) * NTA) {
    if (!(A.vcls[i] & kHang)) continue;
    int x, y, z;
    coords<D>(A, i, x, y, z);
    A.u[i] = interp<D>(C, C.u, x, y, z);
  }
}

template <int D, typename T>
__global__ void __launch_bounds__(NTA) k_ad_leaf(AdaptLevelT<T> A) {
  const long nb = nbox<D>(A);
  const int n = A.n;
  for (long i = long(blockIdx.x) * NTA + threadIdx.x; i < nb; i += long(gridDim.x) * NTA) {
    int x, y, z;
    coords<D>(A, i, x, y, z);
    T r = T(0);
    const bool inter = x > 0 && x < n && y > 0 && y < n && (D == 2 || (z > 0 && z < n));
    if (inter) {
      r = A.bleaf[i];
#pragma unroll
      for (int e = 0; e < (1 << D); ++e) {
        // cell with lower corner (cx, cy, cz); this vertex is its corner iw
        const int ax = e & 1, ay = (e >> 1) & 1, az = (e >> 2) & 1;
        const int cx = x - ax, cy = y - ay, cz = D == 3 ? z - az : 0;
        const long c = cidx<D>(A, cx, cy, cz);
        if (c < 0 || A.leaf[c] != 1) continue;
        const int iw = ax | (ay << 1) | (az << 2);
        T sum = T(0);
#pragma unroll
        for (int j = 0; j < (1 << D); ++j) {
          const long k = vidx<D>(A, cx + (j & 1), cy + ((j >> 1) & 1), cz + ((j >> 2) & 1));
          sum += kref<D, T>(iw, j) * A.u[k];
        }
        r -= eps_of(A, cx, cy, cz, D) * A.hdm2 * sum;
      }
    }
    A.bb[i] = r;
  }
}

template <typename T>
__device__ __forceinline__ T wl(int o) { return o == 0 ? T(1) : (o == 1 || o == -1) ? T(2.0 / 3.0) : T(1.0 / 3.0); }

template <int D, typename T>
__global__ void __launch_bounds__(NTA) k_ad_up(AdaptLevelT<T> A, AdaptLevelT<T> F, int has_f, RtSep<T> rts,
                                               T omega, T omega_t, int jac, int norms_only, double* partials) {
  const long nb = nbox<D>(A);
  double ssum = 0.0, smax = 0.0;
  for (long i = long(blockIdx.x) * NTA + threadIdx.x; i < nb; i += long(gridDim.x) * NTA) {
    const uint8_t cls = A.vcls[i];
    const T rl = A.bb[i];
    T Rb = T(0), Rh = T(0), Rt = T(0);
    int x, y, z;
    coords<D>(A, i, x, y, z);
    if (has_f && (cls & (kDof | kHang))) {
      for (int oz = (D == 3 ? -2 : 0); oz <= (D == 3 ? 2 : 0); ++oz)
        for (int oy = -2; oy <= 2; ++oy)
          for (int ox = -2; ox <= 2; ++ox) {
            const long k = vidx<D>(F, 3 * x + ox, 3 * y + oy, 3 * z + oz);
            if (k < 0) continue;
            const T w = wl<T>(ox) * wl<T>(oy) * (D == 3 ? wl<T>(oz) : T(1));
            Rh += w * F.hh[k];
            if (norms_only) continue;
            const T fb = F.bb[k];
            Rb += w * fb;
            if (jac && (cls & kDof) && (F.vcls[k] & kDof)) {
              // R~ = scale sum_a delta(o_a) prod_{b != a} m(o_b)
              T wt;
              if (D == 2) {
                wt = (ox == 0 ? rts.m[oy + 2] : T(0)) + (oy == 0 ? rts.m[ox + 2] : T(0));
              } else {
                wt = (ox == 0 ? rts.m[oy + 2] * rts.m[oz + 2] : T(0)) + (oy == 0 ? rts.m[ox + 2] * rts.m[oz + 2] : T(0)) +
                     (oz == 0 ? rts.m[ox + 2] * rts.m[oy + 2] : T(0));
              }
              Rt += rts.scale * wt * fb;
            }
          }
    }
    const T acch = rl + Rh;
    A.hh[i] = (cls & kHang) ? acch : T(0);
    if (cls & kComp) {
      const double a = double(acch);
      ssum += double(A.hd) * a * a;
      smax = fmax(smax, fabs(a));
    }
    if (norms_only) {
      // the composite residual in place of the leaf residual (same index, read above)
      A.bb[i] = (cls & kComp) ? acch : T(0);
      continue;
    }
    const T acc = rl + Rb;
    A.bb[i] = acc;
    T sv = T(0);
    if (cls & kDof) {
      const T dg = diag_at<D>(A, i, x, y, z);
      sv = omega * acc / dg;
      if (jac && has_f) sv -= omega_t * Rt / dg;
    }
    A.s[i] = sv;
  }
  block_norm_partials(ssum, smax, partials);
}

template <int D, typename T>
__global__ void __launch_bounds__(NTA) k_ad_down(AdaptLevelT<T> A, AdaptLevelT<T> C, int has_c) {
  const long nb = nbox<D>(A);
  for (long i = long(blockIdx.x) * NTA + threadIdx.x; i < nb; i += long(gridDim.x) * NTA) {
    const uint8_t cls = A.vcls[i];
    T S = T(0);
    if (cls & (kDof | kHang)) {
      S = A.s[i];
      if (has_c) {
        int x, y, z;
        coords<D>(A, i, x, y, z);
        S += interp<D>(C, C.S, x, y, z);
      }
    }
    A.S[i] = S;
  }
}

template <int D, typename T>
__global__ void __launch_bounds__(NTA) k_ad_update(AdaptLevelT<T> A, AdaptLevelT<T> F, int has_f) {
  const long nb = nbox<D>(A);
  for (long i = long(blockIdx.x) * NTA + threadIdx.x; i < nb; i += long(gridDim.x) * NTA) {
    const uint8_t cls = A.vcls[i];
    if (cls & kComp) {
      A.u[i] += A.S[i];
    } else if ((cls & kDof) && has_f) {
      int x, y, z;
      coords<D>(A, i, x, y, z);
      const long k = vidx<D>(F, 3 * x, 3 * y, 3 * z);
      if (k >= 0) A.u[i] = F.u[k];
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
  const long nb = nbox<D>(A);
  for (long i = long(blockIdx.x) * NTA + threadIdx.x; i < nb; i += long(gridDim.x) * NTA) {
    if (!(A.vcls[i] & kDof)) continue;
    int x, y, z;
    coords<D>(A, i, x, y, z);
    A.u[i] = composite_at<D>(O, x * scale, y * scale, z * scale);
  }
}

// FP32 inner form of defect correction: the inner load is the FP64 leaf residual, the inner
// iterate starts at zero.
template <int D>
__global__ void __launch_bounds__(NTA) k_ad_to_inner(AdaptLevel A, AdaptLevelT<float> E) {
  const long nb = nbox<D>(A);
  for (long i = long(blockIdx.x) * NTA + threadIdx.x; i < nb; i += long(gridDim.x) * NTA) {
    E.bleaf[i] = float(A.bb[i]);
    E.u[i] = 0.f;
  }
}

template <int D>
__global__ void __launch_bounds__(NTA) k_ad_accumulate(AdaptLevel A, AdaptLevelT<float> E) {
  const long nb = nbox<D>(A);
  for (long i = long(blockIdx.x) * NTA + threadIdx.x; i < nb; i += long(gridDim.x) * NTA)
    if (A.vcls[i] & kDof) A.u[i] += double(E.u[i]);
}

unsigned grid_for(long nb) {
  long g = (nb + NTA - 1) / NTA;
  return unsigned(g < 8192 ? (g < 1 ? 1 : g) : 8192);
}

}  // namespace

template <typename T>
hipError_t launch_ad_hang(int d, const AdaptLevelT<T>& A, const AdaptLevelT<T>& C, hipStream_t s) {
  const long nb = long(A.mx) * A.my * (d == 3 ? A.mz : 1);
  if (d == 2) k_ad_hang<2, T><<<grid_for(nb), NTA, 0, s>>>(A, C);
  else k_ad_hang<3, T><<<grid_for(nb), NTA, 0, s>>>(A, C);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ad_leaf(int d, const AdaptLevelT<T>& A, hipStream_t s) {
  const long nb = long(A.mx) * A.my * (d == 3 ? A.mz : 1);
  if (d == 2) k_ad_leaf<2, T><<<grid_for(nb), NTA, 0, s>>>(A);
  else k_ad_leaf<3, T><<<grid_for(nb), NTA, 0, s>>>(A);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ad_up(int d, const AdaptLevelT<T>& A, const AdaptLevelT<T>* F, const RtSep<T>& rts, T omega,
                        T omega_t, int damping, int norms_only, double* partials, hipStream_t s) {
  const AdaptLevelT<T> Fv = F ? *F : AdaptLevelT<T>{};
  const int jac = damping == ADAFAC_DAMP_JAC;
  if (d == 2)
    k_ad_up<2, T><<<kAdaptNormBlocks, NTA, 0, s>>>(A, Fv, F ? 1 : 0, rts, omega, omega_t, jac, norms_only, partials);
  else
    k_ad_up<3, T><<<kAdaptNormBlocks, NTA, 0, s>>>(A, Fv, F ? 1 : 0, rts, omega, omega_t, jac, norms_only, partials);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ad_down(int d, const AdaptLevelT<T>& A, const AdaptLevelT<T>* C, hipStream_t s) {
  const long nb = long(A.mx) * A.my * (d == 3 ? A.mz : 1);
  const AdaptLevelT<T> Cv = C ? *C : AdaptLevelT<T>{};
  if (d == 2) k_ad_down<2, T><<<grid_for(nb), NTA, 0, s>>>(A, Cv, C ? 1 : 0);
  else k_ad_down<3, T><<<grid_for(nb), NTA, 0, s>>>(A, Cv, C ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ad_update(int d, const AdaptLevelT<T>& A, const AdaptLevelT<T>* F, hipStream_t s) {
  const long nb = long(A.mx) * A.my * (d == 3 ? A.mz : 1);
  const AdaptLevelT<T> Fv = F ? *F : AdaptLevelT<T>{};
  if (d == 2) k_ad_update<2, T><<<grid_for(nb), NTA, 0, s>>>(A, Fv, F ? 1 : 0);
  else k_ad_update<3, T><<<grid_for(nb), NTA, 0, s>>>(A, Fv, F ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_ad_transfer(int d, const AdaptLevel& A, int scale, const AdaptTreeView& O, hipStream_t s) {
  const long nb = long(A.mx) * A.my * (d == 3 ? A.mz : 1);
  if (d == 2) k_ad_transfer<2><<<grid_for(nb), NTA, 0, s>>>(A, scale, O);
  else k_ad_transfer<3><<<grid_for(nb), NTA, 0, s>>>(A, scale, O);
  return hipGetLastError();
}

hipError_t launch_ad_to_inner(int d, const AdaptLevel& A, const AdaptLevelT<float>& E, hipStream_t s) {
  const long nb = long(A.mx) * A.my * (d == 3 ? A.mz : 1);
  if (d == 2) k_ad_to_inner<2><<<grid_for(nb), NTA, 0, s>>>(A, E);
  else k_ad_to_inner<3><<<grid_for(nb), NTA, 0, s>>>(A, E);
  return hipGetLastError();
}

hipError_t launch_ad_accumulate(int d, const AdaptLevel& A, const AdaptLevelT<float>& E, hipStream_t s) {
  const long nb = long(A.mx) * A.my * (d == 3 ? A.mz : 1);
  if (d == 2) k_ad_accumulate<2><<<grid_for(nb), NTA, 0, s>>>(A, E);
  else k_ad_accumulate<3><<<grid_for(nb), NTA, 0, s>>>(A, E);
  return hipGetLastError();
}

#define ADAFAC_AD_INST(T)                                                                                         \
  template hipError_t launch_ad_hang<T>(int, const AdaptLevelT<T>&, const AdaptLevelT<T>&, hipStream_t);          \
  template hipError_t launch_ad_leaf<T>(int, const AdaptLevelT<T>&, hipStream_t);                                 \
  template hipError_t launch_ad_up<T>(int, const AdaptLevelT<T>&, const AdaptLevelT<T>*, const RtSep<T>&, T, T,  \
                                      int, int, double*, hipStream_t);                                            \
  template hipError_t launch_ad_down<T>(int, const AdaptLevelT<T>&, const AdaptLevelT<T>*, hipStream_t);          \
  template hipError_t launch_ad_update<T>(int, const AdaptLevelT<T>&, const AdaptLevelT<T>*, hipStream_t);
ADAFAC_AD_INST(double)
ADAFAC_AD_INST(float)

}  // namespace adafac
