// Single-pass finest-level sweep of the adAFAC cycle for gfx950.
//
// One launch touches every finest-level vertex once per cycle and does, per vertex:
//   (a) u <- u + P S_{L-1}: the coarse corrections of the previous cycle, applied one sweep
//       late (the iterate shift of Sec. 5.3; the iterates equal those of the unshifted cycle),
//   (b) r = b - A u with the Q1 operator of -div(eps grad u) (element-wise, Sec. 5.2),
//   (c) u <- u + omega D^-1 r (damped Jacobi, Algorithm 1),
//   (d) the FAS injection u_{L-1} = I u, the restriction R r (the coarse level adds the tau
//       correction, Sec. 2.3) and the auxiliary right-hand side R~ r (Sec. 3.2) for every
//       coarse vertex the tile owns,
//   (e) per-block partial sums of h^d r^2 and max |r| (Sec. 6 residual norms).
//
// Tiling.  A workgroup (256 lanes, four wave64) owns a 27 x 27 x tz block of fine vertices
// (tz a multiple of 3), i.e. whole coarse cells, and every coarse vertex at a multiple of 3
// inside it.  The 5^d-point restriction of an owned coarse vertex reaches two fine vertices
// into the lower neighbour, so the tile recomputes the residual on a 29-wide ring and reads
// u on a 31-wide ring: every coarse value is written by exactly one workgroup, without atomics,
// and the result does not depend on scheduling.  3D tiles march through z with the current
// u plane and the current residual plane in LDS; the 27-point stencil is split into the two
// cell layers below and above a vertex, whose partial sums are carried in registers.
// Workgroup ids are remapped so that consecutive tiles (which share halo planes) run on the
// same XCD and hit the same L2.
#include <hip/hip_runtime.h>

#include "adafac.h"
#include "adafac_internal.hpp"
#include "kernels_common.hpp"

namespace adafac {
namespace {

constexpr int TX = 27;            // owned fine vertices per tile along x and y
constexpr int UW = TX + 4;        // u ring: x0-3 .. x0+27
constexpr int RW = TX + 2;        // residual ring: x0-2 .. x0+26
constexpr int CW = TX / 3 + 3;    // coarse S block: x0/3-1 .. x0/3+10
constexpr int NCO = TX / 3;       // owned coarse vertices per axis
constexpr int MAXTZ = 27;
constexpr int NSLOT = (RW * RW + 255) / 256;

__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  // blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous range of tiles
  const int q = nblk / 8, rem = nblk % 8;
  const int x = bid % 8, k = bid / 8;
  return x * q + min(x, rem) + k;
}

template <typename T>
__device__ __forceinline__ T wlin(int o) {  // 1D d-linear restriction weight, |o| <= 2
  return o == 0 ? T(1) : (o == 1 || o == -1) ? T(2.0 / 3.0) : T(1.0 / 3.0);
}

// eps of fine cell (cx, cy, cz), clamped into the lattice (values at non-dof vertices unused)
template <typename T, int D>
__device__ __forceinline__ T eps_fine(const LevelView<T>& F, int cx, int cy, int cz) {
  const int n = F.n;
  cx = min(max(cx, 0), n - 1);
  cy = min(max(cy, 0), n - 1);
  cz = D == 3 ? min(max(cz, 0), n - 1) : 0;
  return eps_cell<T, D>(F, cx, cy, cz);
}

}  // namespace

template <typename T, bool VAREPS>
__global__ void __launch_bounds__(256) k_fine_sweep3d(LevelView<T> F, LevelView<T> C,
                                                      const T* __restrict__ uin, T* __restrict__ uout,
                                                      const T* __restrict__ b, const T* __restrict__ rt,
                                                      T omega, int damping, int apply_pending, int tz,
                                                      int ntx, int ntz, double* __restrict__ partials) {
  __shared__ T Ub[UW * UW];
  __shared__ T Rb[RW * RW];
  __shared__ T Sb[(MAXTZ / 3 + 3) * CW * CW];

  const int nv = F.nv, n = F.n, nvc = C.nv, nc = C.n;
  const int nblk = ntx * ntx * ntz;
  const int t = xcd_remap(blockIdx.x, nblk);
  const int tzi = t % ntz, tyi = (t / ntz) % ntx, txi = t / (ntz * ntx);
  const int x0 = TX * txi, y0 = TX * tyi, z0 = tz * tzi;
  const int cbx = x0 / 3 - 1, cby = y0 / 3 - 1, cbz = z0 / 3 - 1;
  const int nsz = tz / 3 + 3;
  const int tid = threadIdx.x;
  const int pi = damping == ADAFAC_DAMP_PI;
  const T h = F.h;

  // (a) coarse correction block S (minus the injected fine correction for adAFAC-PI)
  if (apply_pending) {
    for (int i = tid; i < nsz * CW * CW; i += 256) {
      const int lx = i % CW, ly = (i / CW) % CW, lz = i / (CW * CW);
      const int cx = cbx + lx, cy = cby + ly, cz = cbz + lz;
      T v = T(0);
      if (cx >= 0 && cx <= nc && cy >= 0 && cy <= nc && cz >= 0 && cz <= nc) {
        const size_t ci = lin<3>(cx, cy, cz, nvc);
        v = C.S[ci];
        if (pi) v -= C.ic[ci];
      }
      Sb[i] = v;
    }
  }

  // per residual column: running sums of the two cell layers (see header)
  T own[NSLOT], dsum[NSLOT], esum[NSLOT], tprev[NSLOT], dq[NSLOT][4], eq[NSLOT][4], epsprev[NSLOT];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    own[s] = dsum[s] = esum[s] = tprev[s] = epsprev[s] = T(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) dq[s][q] = eq[s][q] = T(0);
  }
  T accR[2] = {T(0), T(0)}, accT[2] = {T(0), T(0)};
  double ssum = 0.0, smax = 0.0;

  const int zs = z0 - 3, ze = z0 + tz;
  for (int p = zs; p <= ze; ++p) {
    __syncthreads();  // previous plane fully consumed (Ub) and restricted (Rb), Sb ready
    // load u plane p on the 31 x 31 ring, adding the pending prolongated correction
    for (int i = tid; i < UW * UW; i += 256) {
      const int ux = i % UW, uy = i / UW;
      const int x = x0 - 3 + ux, y = y0 - 3 + uy;
      T v = T(0);
      if (x >= 0 && x <= n && y >= 0 && y <= n && p >= 0 && p <= n) {
        v = uin[lin<3>(x, y, p, nv)];
        if (apply_pending) {
          const int cx = x / 3, cy = y / 3, cz = p / 3;
          const int sx = x - 3 * cx, sy = y - 3 * cy, sz = p - 3 * cz;
          const T wx[2] = {T(3 - sx) * T(1.0 / 3.0), T(sx) * T(1.0 / 3.0)};
          const T wy[2] = {T(3 - sy) * T(1.0 / 3.0), T(sy) * T(1.0 / 3.0)};
          const T wz[2] = {T(3 - sz) * T(1.0 / 3.0), T(sz) * T(1.0 / 3.0)};
          const int lx = cx - cbx, ly = cy - cby, lz = cz - cbz;
          T acc = T(0);
#pragma unroll
          for (int ez = 0; ez < 2; ++ez)
#pragma unroll
            for (int ey = 0; ey < 2; ++ey)
#pragma unroll
              for (int ex = 0; ex < 2; ++ex)
                acc += wz[ez] * wy[ey] * wx[ex] * Sb[((lz + ez) * CW + ly + ey) * CW + lx + ex];
          v += acc;
        }
      }
      Ub[i] = v;
    }
    __syncthreads();
    // residual of plane z = p - 1 on the 29 x 29 ring
    const int z = p - 1;
    const bool zres = p >= zs + 2;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      const int j = tid + 256 * s;
      if (j >= RW * RW) continue;
      const int rx = j % RW, ry = j / RW;
      const int x = x0 - 2 + rx, y = y0 - 2 + ry;
      const T* up = &Ub[(ry + 1) * UW + rx + 1];
      const T o_n = up[0];
      // quadrants q = (sx, sy): 0 = (-,-), 1 = (+,-), 2 = (-,+), 3 = (+,+)
      const T ax_m = up[-1], ax_p = up[1], ay_m = up[-UW], ay_p = up[UW];
      const T d_n[4] = {up[-UW - 1], up[-UW + 1], up[UW - 1], up[UW + 1]};
      const T e_n[4] = {ax_m + ay_m + d_n[0], ax_p + ay_m + d_n[1], ax_m + ay_p + d_n[2], ax_p + ay_p + d_n[3]};
      T bc, tn, esl;
      if (!VAREPS) {
        const T ds_n = (d_n[0] + d_n[1]) + (d_n[2] + d_n[3]);
        const T es_n = (e_n[0] + e_n[1]) + (e_n[2] + e_n[3]);
        bc = T(4.0 / 3.0) * own[s] - T(1.0 / 12.0) * (dsum[s] + es_n);
        tn = T(4.0 / 3.0) * o_n - T(1.0 / 12.0) * (ds_n + esum[s]);
        esl = T(4);
        dsum[s] = ds_n;
        esum[s] = es_n;
      } else {
        // eps of the four cells of layer z (between planes z and z+1) around column (x, y)
        const T e4[4] = {eps_fine<T, 3>(F, x - 1, y - 1, z), eps_fine<T, 3>(F, x, y - 1, z),
                         eps_fine<T, 3>(F, x - 1, y, z), eps_fine<T, 3>(F, x, y, z)};
        bc = T(0);
        tn = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          bc += e4[q] * (T(1.0 / 3.0) * own[s] - T(1.0 / 12.0) * (dq[s][q] + e_n[q]));
          tn += e4[q] * (T(1.0 / 3.0) * o_n - T(1.0 / 12.0) * (d_n[q] + eq[s][q]));
        }
        esl = (e4[0] + e4[1]) + (e4[2] + e4[3]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          dq[s][q] = d_n[q];
          eq[s][q] = e_n[q];
        }
      }
      T res = T(0);
      if (zres && x > 0 && x < n && y > 0 && y < n && z > 0 && z < n) {
        const T au = h * (bc + tprev[s]);
        const T dg = h * T(1.0 / 3.0) * (esl + epsprev[s]);
        const T uz = own[s];
        res = b[lin<3>(x, y, z, nv)] - au;
        const bool owned = rx >= 2 && ry >= 2 && x < x0 + TX && y < y0 + TX && z >= z0 && z < z0 + tz;
        if (owned) {
          const T c = omega * res / dg;
          uout[lin<3>(x, y, z, nv)] = uz + c;
          const double rd = double(res);
          ssum += double(F.hd) * rd * rd;
          smax = fmax(smax, fabs(rd));
          if (x % 3 == 0 && y % 3 == 0 && z % 3 == 0) {
            const size_t ci = lin<3>(x / 3, y / 3, z / 3, nvc);
            C.u[ci] = uz;                    // FAS injection of iterate n
            if (pi) C.ic[ci] = c;            // adAFAC-PI: injected fine correction
          }
        }
      }
      Rb[j] = res;
      tprev[s] = tn;
      epsprev[s] = esl;
      own[s] = o_n;
    }
    __syncthreads();
    if (!zres) continue;
    // restriction of plane z to the owned coarse columns: R r and R~ r (5 x 5 in-plane gathers)
    if (tid < NCO * NCO) {
      const int ccx = tid % NCO, ccy = tid / NCO;
      const T* rc = &Rb[(3 * ccy + 2) * RW + 3 * ccx + 2];
      const int lo = z >= 0 ? z / 3 : -1;   // z >= z0 - 2 >= -2; only z < 0 at the lower boundary
      const int m = z - 3 * lo;             // 0, 1, 2 (offset from coarse plane lo)
      T sR = T(0), sT0 = T(0), sT1 = T(0);
      // R~ in-plane pattern for |oz| = m (coarse plane lo) and |oz| = 3 - m (plane lo + 1)
      const int pa = 2 + m, pb = 2 + (3 - m);   // index into rt's z offset (+|oz| side)
#pragma unroll
      for (int oy = -2; oy <= 2; ++oy)
#pragma unroll
        for (int ox = -2; ox <= 2; ++ox) {
          const T rv = rc[oy * RW + ox];
          sR += wlin<T>(ox) * wlin<T>(oy) * rv;
          if (damping == ADAFAC_DAMP_JAC) {
            sT0 += rt[(ox + 2) + 5 * (oy + 2) + 25 * pa] * rv;
            if (m) sT1 += rt[(ox + 2) + 5 * (oy + 2) + 25 * (pb < 5 ? pb : 0)] * rv;
          }
        }
      accR[0] += wlin<T>(m) * sR;
      accT[0] += sT0;
      if (m) {
        accR[1] += wlin<T>(3 - m) * sR;
        accT[1] += sT1;
      }
      if (m == 2) {
        const int cz = lo;
        const int cx = x0 / 3 + ccx, cy = y0 / 3 + ccy;
        if (cz >= z0 / 3 && cz < (z0 + tz) / 3 && cx > 0 && cx < nc && cy > 0 && cy < nc && cz > 0 &&
            cz < nc) {
          const size_t ci = lin<3>(cx, cy, cz, nvc);
          C.rr[ci] = accR[0];
          C.bt[ci] = accT[0];
        }
        accR[0] = accR[1];
        accT[0] = accT[1];
        accR[1] = accT[1] = T(0);
      }
    }
  }
  block_norm_partials(ssum, smax, partials);
}

template <typename T, bool VAREPS>
__global__ void __launch_bounds__(256) k_fine_sweep2d(LevelView<T> F, LevelView<T> C,
                                                      const T* __restrict__ uin, T* __restrict__ uout,
                                                      const T* __restrict__ b, const T* __restrict__ rt,
                                                      T omega, int damping, int apply_pending, int ntx,
                                                      double* __restrict__ partials) {
  __shared__ T Ub[UW * UW];
  __shared__ T Rb[RW * RW];
  __shared__ T Sb[CW * CW];
  const int nv = F.nv, n = F.n, nvc = C.nv, nc = C.n;
  const int t = xcd_remap(blockIdx.x, ntx * ntx);
  const int txi = t % ntx, tyi = t / ntx;
  const int x0 = TX * txi, y0 = TX * tyi;
  const int cbx = x0 / 3 - 1, cby = y0 / 3 - 1;
  const int tid = threadIdx.x;
  const int pi = damping == ADAFAC_DAMP_PI;
  if (apply_pending) {
    for (int i = tid; i < CW * CW; i += 256) {
      const int cx = cbx + i % CW, cy = cby + i / CW;
      T v = T(0);
      if (cx >= 0 && cx <= nc && cy >= 0 && cy <= nc) {
        const size_t ci = lin<2>(cx, cy, 0, nvc);
        v = C.S[ci];
        if (pi) v -= C.ic[ci];
      }
      Sb[i] = v;
    }
    __syncthreads();
  }
  for (int i = tid; i < UW * UW; i += 256) {
    const int x = x0 - 3 + i % UW, y = y0 - 3 + i / UW;
    T v = T(0);
    if (x >= 0 && x <= n && y >= 0 && y <= n) {
      v = uin[lin<2>(x, y, 0, nv)];
      if (apply_pending) {
        const int cx = x / 3, cy = y / 3, sx = x - 3 * cx, sy = y - 3 * cy;
        const int lx = cx - cbx, ly = cy - cby;
        const T wx0 = T(3 - sx) * T(1.0 / 3.0), wx1 = T(sx) * T(1.0 / 3.0);
        const T wy0 = T(3 - sy) * T(1.0 / 3.0), wy1 = T(sy) * T(1.0 / 3.0);
        v += wy0 * (wx0 * Sb[ly * CW + lx] + wx1 * Sb[ly * CW + lx + 1]) +
             wy1 * (wx0 * Sb[(ly + 1) * CW + lx] + wx1 * Sb[(ly + 1) * CW + lx + 1]);
      }
    }
    Ub[i] = v;
  }
  __syncthreads();
  double ssum = 0.0, smax = 0.0;
  for (int j = tid; j < RW * RW; j += 256) {
    const int rx = j % RW, ry = j / RW;
    const int x = x0 - 2 + rx, y = y0 - 2 + ry;
    T res = T(0);
    if (x > 0 && x < n && y > 0 && y < n) {
      const T* up = &Ub[(ry + 1) * UW + rx + 1];
      const T u0 = up[0];
      const T ax_m = up[-1], ax_p = up[1], ay_m = up[-UW], ay_p = up[UW];
      const T d4[4] = {up[-UW - 1], up[-UW + 1], up[UW - 1], up[UW + 1]};
      T au, dg;
      if (!VAREPS) {
        au = T(8.0 / 3.0) * u0 - T(1.0 / 3.0) * ((ax_m + ax_p) + (ay_m + ay_p)) -
             T(1.0 / 3.0) * ((d4[0] + d4[1]) + (d4[2] + d4[3]));
        dg = T(8.0 / 3.0);
      } else {
        const T e4[4] = {eps_fine<T, 2>(F, x - 1, y - 1, 0), eps_fine<T, 2>(F, x, y - 1, 0),
                         eps_fine<T, 2>(F, x - 1, y, 0), eps_fine<T, 2>(F, x, y, 0)};
        const T axq[4] = {ax_m, ax_p, ax_m, ax_p}, ayq[4] = {ay_m, ay_m, ay_p, ay_p};
        au = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          au += e4[q] * (T(2.0 / 3.0) * u0 - T(1.0 / 6.0) * (axq[q] + ayq[q]) - T(1.0 / 3.0) * d4[q]);
        dg = T(2.0 / 3.0) * ((e4[0] + e4[1]) + (e4[2] + e4[3]));
      }
      res = b[lin<2>(x, y, 0, nv)] - au;
      if (rx >= 2 && ry >= 2 && x < x0 + TX && y < y0 + TX) {
        const T c = omega * res / dg;
        uout[lin<2>(x, y, 0, nv)] = u0 + c;
        const double rd = double(res);
        ssum += double(F.hd) * rd * rd;
        smax = fmax(smax, fabs(rd));
        if (x % 3 == 0 && y % 3 == 0) {
          const size_t ci = lin<2>(x / 3, y / 3, 0, nvc);
          C.u[ci] = u0;
          if (pi) C.ic[ci] = c;
        }
      }
    }
    Rb[j] = res;
  }
  __syncthreads();
  if (tid < NCO * NCO) {
    const int ccx = tid % NCO, ccy = tid / NCO;
    const int cx = x0 / 3 + ccx, cy = y0 / 3 + ccy;
    if (cx > 0 && cx < nc && cy > 0 && cy < nc) {
      const T* rc = &Rb[(3 * ccy + 2) * RW + 3 * ccx + 2];
      T sR = T(0), sT = T(0);
#pragma unroll
      for (int oy = -2; oy <= 2; ++oy)
#pragma unroll
        for (int ox = -2; ox <= 2; ++ox) {
          const T rv = rc[oy * RW + ox];
          sR += wlin<T>(ox) * wlin<T>(oy) * rv;
          if (damping == ADAFAC_DAMP_JAC) sT += rt[(ox + 2) + 5 * (oy + 2)] * rv;
        }
      const size_t ci = lin<2>(cx, cy, 0, nvc);
      C.rr[ci] = sR;
      C.bt[ci] = sT;
    }
  }
  block_norm_partials(ssum, smax, partials);
}

// ---------------------------------------------------------------------------
size_t fine_sweep_partials(int d, int n) {
  if (n % TX) return 0;
  const int ntx = n / TX;
  if (d == 2) return size_t(ntx) * ntx;
  return size_t(ntx) * ntx * (n / 3);   // upper bound over the z-chunk choices
}

static int pick_tz(int n) {
  // longest z chunk (multiple of 3, <= 27, dividing n) that still gives >= 512 workgroups
  const int ntx = n / TX;
  int best = 3;
  for (int tz = 3; tz <= MAXTZ; tz *= 3)
    if (n % tz == 0 && size_t(ntx) * ntx * (n / tz) >= 512) best = tz;
  return best;
}

template <typename T>
hipError_t launch_fine_sweep(int d, const LevelView<T>& F, const LevelView<T>& C, const T* uin, T* uout,
                             const T* b, const T* rt, T omega, int damping, int apply_pending,
                             double* partials, int* nparts, hipStream_t s) {
  const int n = F.n;
  if (n % TX || F.pw) return hipErrorInvalidValue;   // needs 27 | n and d-linear transfer into L
  const int ntx = n / TX;
  const bool var = F.eps != nullptr;
  if (d == 2) {
    const unsigned nb = unsigned(ntx * ntx);
    if (var)
      k_fine_sweep2d<T, true><<<nb, 256, 0, s>>>(F, C, uin, uout, b, rt, omega, damping, apply_pending, ntx, partials);
    else
      k_fine_sweep2d<T, false><<<nb, 256, 0, s>>>(F, C, uin, uout, b, rt, omega, damping, apply_pending, ntx, partials);
    *nparts = int(nb);
  } else {
    const int tz = pick_tz(n), ntz = n / tz;
    const unsigned nb = unsigned(ntx * ntx * ntz);
    if (var)
      k_fine_sweep3d<T, true><<<nb, 256, 0, s>>>(F, C, uin, uout, b, rt, omega, damping, apply_pending, tz, ntx, ntz, partials);
    else
      k_fine_sweep3d<T, false><<<nb, 256, 0, s>>>(F, C, uin, uout, b, rt, omega, damping, apply_pending, tz, ntx, ntz, partials);
    *nparts = int(nb);
  }
  return hipGetLastError();
}

template hipError_t launch_fine_sweep<double>(int, const LevelView<double>&, const LevelView<double>&,
                                              const double*, double*, const double*, const double*, double,
                                              int, int, double*, int*, hipStream_t);
template hipError_t launch_fine_sweep<float>(int, const LevelView<float>&, const LevelView<float>&,
                                             const float*, float*, const float*, const float*, float, int,
                                             int, double*, int*, hipStream_t);

}  // namespace adafac
