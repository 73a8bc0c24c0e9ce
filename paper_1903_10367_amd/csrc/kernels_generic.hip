// gfx950 kernels of the adAFAC cycle, one kernel per step (Sec. 3.1, Algorithm 1).
//
// These kernels are the building blocks that every path uses for the coarse levels and,
// with `fused = 0`, for the finest level too:
//   fine_residual   r_L = b - A_L u, u <- u + omega D^-1 r_L, per-block norm partials
//   level_update    FAS step of one coarse level l (Sec. 2.4): inject u_l = I u_{l+1},
//                   restrict R r_{l+1} and R~ r_{l+1}, form the FAS right-hand side with the
//                   tau correction b_l = R r_{l+1} + A_l I u_{l+1}, the level residual
//                   r_l = b_l - A_l u_l, the Jacobi correction c_l = omega D^-1 r_l and the
//                   auxiliary correction c~_l = omega~ D^-1 b~_l (Sec. 3.2)
//   prolong_add     S_l += P S_{l-1} (accumulation of the prolonged corrections)
//   norm_finalize   fixed-order reduction of the norm partials
// One thread per vertex; arrays cover the full vertex lattice (boundary entries zero).
#include <hip/hip_runtime.h>

#include "adafac.h"
#include "adafac_internal.hpp"
#include "kernels_common.hpp"

namespace adafac {

template <typename T, int D, bool G>
__global__ void __launch_bounds__(256) k_fine_residual(LevelView<T> F, const T* __restrict__ uin,
                                                       T* __restrict__ uout, const T* __restrict__ b,
                                                       T* __restrict__ r, T* __restrict__ ic_coarse,
                                                       int nvc, T omega, int pi,
                                                       double* __restrict__ partials, Gate g) {
  if (G && gated(g)) return;
  const int nv = F.nv;
  const size_t nverts = D == 2 ? size_t(nv) * nv : size_t(nv) * nv * nv;
  double ssum = 0.0, smax = 0.0;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nverts;
       i += size_t(gridDim.x) * blockDim.x) {
    int x = int(i % nv), y = int((i / nv) % nv), z = D == 3 ? int(i / (size_t(nv) * nv)) : 0;
    if (!is_interior<D>(x, y, z, nv)) continue;
    T dg;
    T au = apply_level_op<T, D>(F, x, y, z, dg, [&](int dx, int dy, int dz) {
      return uin[lin<D>(x + dx, y + dy, z + dz, nv)];
    });
    T res = b[i] - au;
    T c = omega * res / dg;
    r[i] = res;
    uout[i] = uin[i] + c;
    if (pi && x % 3 == 0 && y % 3 == 0 && (D == 2 || z % 3 == 0))
      ic_coarse[lin<D>(x / 3, y / 3, z / 3, nvc)] = c;
    double rd = double(res);
    ssum += double(F.hd) * rd * rd;
    smax = fmax(smax, fabs(rd));
  }
  block_norm_partials(ssum, smax, partials);
}

template <typename T, int D, bool G>
__global__ void __launch_bounds__(256) k_level_update(LevelView<T> C, LevelView<T> F, LevelView<T> Cm,
                                                      RtSep<T> rts, T omega, T omega_t, T cscale,
                                                      int damping, int gather, Gate g) {
  if (G && gated(g)) return;
  const size_t nverts = D == 2 ? size_t(C.nv) * C.nv : size_t(C.nv) * C.nv * C.nv;
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nverts) return;
  level_update_vertex<T, D>(C, F, Cm, rts, omega, omega_t, cscale, damping, gather, i);
}

// The smallest levels in one workgroup: the residual norms of the cycle (fixed-order reduction
// of the finest-level partials), the FAS updates of levels hi .. lo (finest first), then the
// prolongation S_l += P S_{l-1} for l = lo+1 .. hi, with a workgroup barrier between levels.
// Lanes of the small-level workgroup: few enough that the 5^d gathers stay in registers.
#ifndef ADAFAC_SMALL_THREADS
#define ADAFAC_SMALL_THREADS 256
#endif
constexpr int kSmallThreads = ADAFAC_SMALL_THREADS;
static_assert(kSmallThreads % 64 == 0 && kSmallThreads <= 1024, "whole wavefronts, at most 16");

template <typename T, int D, bool G>
__global__ void __launch_bounds__(kSmallThreads) k_small_levels(SmallLevelsArgs<T> a) {
  if (G && gated(a.gate)) return;
  const int tid = threadIdx.x;
  const int lo = a.lo, hi = a.hi;
  auto nverts_of = [](const LevelView<T>& v) {
    return D == 2 ? size_t(v.nv) * v.nv : size_t(v.nv) * v.nv * v.nv;
  };
  if (a.norm_out) {
    // fixed order: each lane sums a strided subset, then a fixed butterfly and wave order
    __shared__ double ws[16], wm[16];
    double s = 0.0, m = 0.0;
    for (int i = tid; i < a.nparts; i += kSmallThreads) {
      s += a.partials[2 * i];
      m = fmax(m, a.partials[2 * i + 1]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s += __shfl_xor(s, off);
      m = fmax(m, __shfl_xor(m, off));
    }
    if ((tid & 63) == 0) {
      ws[tid >> 6] = s;
      wm[tid >> 6] = m;
    }
    __syncthreads();
    if (tid == 0) {
      double st = 0.0, mt = 0.0;
      for (int w = 0; w < kSmallThreads / 64; ++w) {
        st += ws[w];
        mt = fmax(mt, wm[w]);
      }
      a.norm_out[0] = sqrt(st);
      a.norm_out[1] = mt;
      if (G) apply_stop_rule(a.rule, a.norm_out);
    }
  }
  for (int l = hi; l >= lo; --l) {
    const LevelView<T>& C = a.lv[l - lo + 1];
    const size_t nverts = nverts_of(C);
    for (size_t i = tid; i < nverts; i += kSmallThreads)
      level_update_vertex<T, D>(C, a.lv[l - lo + 2], a.lv[l - lo], a.rts, a.omega, a.omega_t,
                                a.cscale[l - lo], a.damping, a.gather[l - lo], i);
    __syncthreads();
  }
  const bool pi = a.damping == ADAFAC_DAMP_PI;
  for (int l = lo + 1; l <= hi; ++l) {
    const LevelView<T>& F = a.lv[l - lo + 1];
    const LevelView<T>& C = a.lv[l - lo];
    const int nv = F.nv;
    const size_t nverts = nverts_of(F);
    for (size_t i = tid; i < nverts; i += kSmallThreads) {
      int x = int(i % nv), y = int((i / nv) % nv), z = D == 3 ? int(i / (size_t(nv) * nv)) : 0;
      if (!is_interior<D>(x, y, z, nv)) continue;
      F.S[i] += prolong_value<T, D>(F, C, x, y, z, C.S, pi ? C.ic : nullptr);
    }
    __syncthreads();
  }
}

// dst(f) += sum_c P(f <- c) (src(c) - sub(c)) - self(f) on the interior vertices of level F
// (sub, self may be null).
template <typename T, int D, bool G>
__global__ void __launch_bounds__(256) k_prolong_add(LevelView<T> F, LevelView<T> C, T* __restrict__ dst,
                                                     const T* __restrict__ src, const T* __restrict__ sub,
                                                     const T* __restrict__ self, Gate g) {
  if (G && gated(g)) return;
  // lattices here stay below 2^32 vertices (the launcher checks): 32-bit index arithmetic
  const unsigned nv = unsigned(F.nv);
  const unsigned nverts = D == 2 ? nv * nv : nv * nv * nv;
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nverts) return;
  const unsigned q = i / nv;
  const int x = int(i - q * nv), y = D == 3 ? int(q % nv) : int(q), z = D == 3 ? int(q / nv) : 0;
  if (!is_interior<D>(x, y, z, int(nv))) return;
  T v = prolong_value<T, D>(F, C, x, y, z, src, sub);
  if (self) v -= self[i];
  dst[i] += v;
}

// The prolongations of one cycle, S_k += P (S_{k-1} - sub_{k-1}) for k = 1 .. NT (Sec. 3.1: the
// corrections of all levels summed down to the finest), in one launch instead of NT dependent
// ones.  A workgroup owns a tile of the top target and first gathers, for every level below,
// the region its tile's prolongations read (a level's region: the coarse vertices under the
// finer region, plus one); all global loads of the chain are issued before the first barrier.
// It then forms the levels' new S bottom-up in LDS (recomputing the few vertices its regions
// share with the neighbouring tiles) and writes, to out[k], the intermediate levels' interior
// vertices whose top-level image 3^(NT-k) x lies in its tile, so that each is written once.  The arithmetic per
// vertex is prolong_add's, so the result is bitwise that of the NT single launches.
#ifndef ADAFAC_CHAIN_TZ
#define ADAFAC_CHAIN_TZ 3
#endif
#ifndef ADAFAC_CHAIN_THREADS
#define ADAFAC_CHAIN_THREADS 512
#endif
constexpr int kChainThreads = ADAFAC_CHAIN_THREADS;
template <int D>
struct ChainTile {
  static constexpr int X = D == 3 ? 27 : 81, Y = 9, Z = D == 3 ? ADAFAC_CHAIN_TZ : 1;
};
// width of the coarse region under a finer region of width w (any offset, clamps included)
constexpr int chain_grow(int w) { return (w - 1) / 3 + 3; }

// What the chain reads of each level, packed small: every wave loads it at entry in one batch
// of scalar loads (a kernel-argument block of full level views costs several dependent
// scalar-cache round trips before the first vector load).
template <typename T>
struct ChainLevel {
  T* S;
  const T* sub;
  T* out;
  const T* pw;
  int nv, pad;
};
template <typename T, int NT>
struct ChainDev {
  ChainLevel<T> lv[NT + 1];
  const T* self;
  int tiles0, tiles1;
  Gate gate;
};

template <typename T, int D, int NT, bool G>
__global__ void __launch_bounds__(kChainThreads) k_prolong_chain(ChainDev<T, NT> a) {
  if (G && gated(a.gate)) return;
  constexpr int NTH = kChainThreads;
  constexpr int TX = ChainTile<D>::X, TY = ChainTile<D>::Y, TZ = ChainTile<D>::Z;
  constexpr int TILE = TX * TY * TZ;
  constexpr int TOP = (TILE + NTH - 1) / NTH;
  // the widest region below the top: level NT-1 (regions shrink further down, 3 stays 3)
  constexpr int CAP = chain_grow(TX) * chain_grow(TY) * (D == 3 ? chain_grow(TZ) : 1);
  static_assert(CAP <= NTH, "one region vertex per lane");
  __shared__ T reg[NT][CAP];
  const int tid = threadIdx.x;
  int nv[NT + 1];
  const T *sub[NT + 1], *pw[NT + 1];
  T *S[NT + 1], *out[NT + 1];
#pragma unroll
  for (int k = 0; k <= NT; ++k) {
    nv[k] = a.lv[k].nv;
    S[k] = a.lv[k].S;
    sub[k] = a.lv[k].sub;
    pw[k] = a.lv[k].pw;
    out[k] = a.lv[k].out;
  }
  const T* self = a.self;
  int lo[NT + 1][3], w[NT + 1][3];
  {
    const int b = blockIdx.x, t0 = a.tiles0, t1 = a.tiles1;
    lo[NT][0] = (b % t0) * TX;
    lo[NT][1] = ((b / t0) % t1) * TY;
    lo[NT][2] = D == 3 ? (b / (t0 * t1)) * TZ : 0;
    w[NT][0] = min(TX, nv[NT] - lo[NT][0]);
    w[NT][1] = min(TY, nv[NT] - lo[NT][1]);
    w[NT][2] = D == 3 ? min(TZ, nv[NT] - lo[NT][2]) : 1;
  }
#pragma unroll
  for (int k = NT - 1; k >= 0; --k) {
    const int nc = nv[k] - 1;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      if (ax < D) {
        const int c0 = min(lo[k + 1][ax] / 3, nc - 1);
        const int c1 = min((lo[k + 1][ax] + w[k + 1][ax] - 1) / 3, nc - 1) + 1;
        lo[k][ax] = c0;
        w[k][ax] = c1 - c0 + 1;
      } else {
        lo[k][ax] = 0;
        w[k][ax] = 1;
      }
    }
  }
  // this lane's vertex of each region below the top (global coordinates), if any
  int rx[NT], ry[NT], rz[NT];
  bool rin[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const int e = tid, w0 = w[k][0], w01 = w[k][0] * w[k][1];
    rin[k] = e < w01 * w[k][2];
    const int q = e / w0;
    rx[k] = lo[k][0] + (e - q * w0);
    ry[k] = lo[k][1] + q % w[k][1];
    rz[k] = lo[k][2] + e / w01;
  }
  // all global loads first: the source values, the targets' S and sub, the top's S and self
  T src0 = T(0), srcSub0 = T(0), rawS[NT], rawSub[NT], topS[TOP], topSelf[TOP];
  if (rin[0]) {
    const size_t gi = lin<D>(rx[0], ry[0], rz[0], nv[0]);
    src0 = S[0][gi];
    if (sub[0]) srcSub0 = sub[0][gi];
  }
#pragma unroll
  for (int k = 1; k < NT; ++k) {
    rawS[k] = T(0);
    rawSub[k] = T(0);
    if (rin[k]) {
      const size_t gi = lin<D>(rx[k], ry[k], rz[k], nv[k]);
      rawS[k] = S[k][gi];
      if (sub[k]) rawSub[k] = sub[k][gi];
    }
  }
  const int nvt = nv[NT];
#pragma unroll
  for (int j = 0; j < TOP; ++j) {
    const int e = tid + NTH * j;
    topS[j] = T(0);
    topSelf[j] = T(0);
    if (e < TILE) {
      const int x = lo[NT][0] + e % TX, y = lo[NT][1] + (e / TX) % TY, z = lo[NT][2] + e / (TX * TY);
      if (x < nvt && y < nvt && (D == 2 || z < nvt) && is_interior<D>(x, y, z, nvt)) {
        const size_t gi = lin<D>(x, y, z, nvt);
        topS[j] = S[NT][gi];
        if (self) topSelf[j] = self[gi];
      }
    }
  }
  if (rin[0]) {
    T v = src0;
    if (sub[0]) v -= srcSub0;
    reg[0][tid] = v;
  }
  __syncthreads();
  // the intermediate targets, bottom-up; their global stores wait until after the last barrier
  // (the memory counter that a later load waits on also counts stores)
  T outv[NT];
  size_t outi[NT];
#pragma unroll
  for (int k = 1; k < NT; ++k) {
    outi[k] = ~size_t(0);
    outv[k] = T(0);
    if (rin[k]) {
      const int x = rx[k], y = ry[k], z = rz[k];
      T v = rawS[k];
      if (is_interior<D>(x, y, z, nv[k])) {
        v += prolong_gather<T, D>(pw[k], nv[k], nv[k - 1], x, y, z, [&](int X, int Y, int Z) {
          return reg[k - 1][(X - lo[k - 1][0]) + w[k - 1][0] * ((Y - lo[k - 1][1]) + w[k - 1][1] * (Z - lo[k - 1][2]))];
        });
        // written by the tile that holds this vertex's image on the top level
        int s = 1;
#pragma unroll
        for (int j = k; j < NT; ++j) s *= 3;
        const bool own = s * x >= lo[NT][0] && s * x < lo[NT][0] + TX && s * y >= lo[NT][1] &&
                         s * y < lo[NT][1] + TY && (D == 2 || (s * z >= lo[NT][2] && s * z < lo[NT][2] + TZ));
        if (own) {
          outi[k] = lin<D>(x, y, z, nv[k]);
          outv[k] = v;
        }
      }
      if (sub[k]) v -= rawSub[k];
      reg[k][tid] = v;
    }
    __syncthreads();
  }
  // the top target
#pragma unroll
  for (int j = 0; j < TOP; ++j) {
    const int e = tid + NTH * j;
    if (e < TILE) {
      const int x = lo[NT][0] + e % TX, y = lo[NT][1] + (e / TX) % TY, z = lo[NT][2] + e / (TX * TY);
      if (x < nvt && y < nvt && (D == 2 || z < nvt) && is_interior<D>(x, y, z, nvt)) {
        T v = prolong_gather<T, D>(pw[NT], nvt, nv[NT - 1], x, y, z, [&](int X, int Y, int Z) {
          return reg[NT - 1][(X - lo[NT - 1][0]) +
                             w[NT - 1][0] * ((Y - lo[NT - 1][1]) + w[NT - 1][1] * (Z - lo[NT - 1][2]))];
        });
        if (self) v -= topSelf[j];
        S[NT][lin<D>(x, y, z, nvt)] = topS[j] + v;
      }
    }
  }
#pragma unroll
  for (int k = 1; k < NT; ++k)
    if (outi[k] != ~size_t(0)) out[k][outi[k]] = outv[k];
}

// FP32 cycles inside FP64 defect correction: the two FP64 steps of an outer iteration.
//   accumulate  u <- u + (e + P S_{L-1}): the FP32 correction of the inner cycles (with the
//               prolongation the fused sweep leaves pending) added to the FP64 solution
//   defect      r = b - A_L u in FP64, stored rounded to FP32 as the inner right-hand side,
//               with the FP64 norm partials of r
template <int D>
__global__ void __launch_bounds__(256) k_accumulate(LevelView<float> F, LevelView<float> C, double* __restrict__ u,
                                                    const float* __restrict__ e, const float* __restrict__ S) {
  const int nv = F.nv;
  const size_t nverts = D == 2 ? size_t(nv) * nv : size_t(nv) * nv * nv;
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nverts) return;
  int x = int(i % nv), y = int((i / nv) % nv), z = D == 3 ? int(i / (size_t(nv) * nv)) : 0;
  if (!is_interior<D>(x, y, z, nv)) return;
  float c = e[i];
  if (S) c += prolong_value<float, D>(F, C, x, y, z, S, nullptr);
  u[i] += double(c);
}

template <int D>
__global__ void __launch_bounds__(256) k_defect(LevelView<double> F, const double* __restrict__ u,
                                                const double* __restrict__ b, float* __restrict__ r32,
                                                double* __restrict__ partials) {
  const int nv = F.nv;
  const size_t nverts = D == 2 ? size_t(nv) * nv : size_t(nv) * nv * nv;
  double ssum = 0.0, smax = 0.0;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nverts;
       i += size_t(gridDim.x) * blockDim.x) {
    int x = int(i % nv), y = int((i / nv) % nv), z = D == 3 ? int(i / (size_t(nv) * nv)) : 0;
    if (!is_interior<D>(x, y, z, nv)) continue;
    double dg;
    const double au = apply_level_op<double, D>(F, x, y, z, dg, [&](int dx, int dy, int dz) {
      return u[lin<D>(x + dx, y + dy, z + dz, nv)];
    });
    const double res = b[i] - au;
    r32[i] = float(res);
    ssum += F.hd * res * res;
    smax = fmax(smax, fabs(res));
  }
  block_norm_partials(ssum, smax, partials);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_accumulate(int d, const LevelView<float>& F, const LevelView<float>& C, double* u,
                             const float* e, const float* S, hipStream_t s) {
  size_t nverts = d == 2 ? size_t(F.nv) * F.nv : size_t(F.nv) * F.nv * F.nv;
  unsigned nb = unsigned((nverts + 255) / 256);
  if (d == 2)
    k_accumulate<2><<<nb, 256, 0, s>>>(F, C, u, e, S);
  else
    k_accumulate<3><<<nb, 256, 0, s>>>(F, C, u, e, S);
  return hipGetLastError();
}

hipError_t launch_defect(int d, const LevelView<double>& F, const double* u, const double* b, float* r32,
                         double* partials, int nblocks, hipStream_t s) {
  if (d == 2)
    k_defect<2><<<nblocks, 256, 0, s>>>(F, u, b, r32, partials);
  else
    k_defect<3><<<nblocks, 256, 0, s>>>(F, u, b, r32, partials);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_fine_residual(int d, const LevelView<T>& F, const T* uin, T* uout, const T* b, T* r,
                                T* ic_coarse, int nvc, T omega, int pi, double* partials, int nblocks,
                                hipStream_t s, Gate g) {
#define AD_FR(DD, GG) k_fine_residual<T, DD, GG><<<nblocks, 256, 0, s>>>(F, uin, uout, b, r, ic_coarse, nvc, omega, pi, partials, g)
  if (d == 2) {
    if (g.stop) AD_FR(2, true); else AD_FR(2, false);
  } else {
    if (g.stop) AD_FR(3, true); else AD_FR(3, false);
  }
#undef AD_FR
  return hipGetLastError();
}

template <typename T>
hipError_t launch_level_update(int d, const LevelView<T>& C, const LevelView<T>& F, const LevelView<T>& Cm,
                               const RtSep<T>& rt, T omega, T omega_t, T cscale, int damping, int gather,
                               hipStream_t s, Gate g) {
  size_t nverts = d == 2 ? size_t(C.nv) * C.nv : size_t(C.nv) * C.nv * C.nv;
  if (nverts >= (size_t(1) << 32)) return hipErrorInvalidValue;
  unsigned nb = unsigned((nverts + 255) / 256);
#define AD_LU(DD, GG) k_level_update<T, DD, GG><<<nb, 256, 0, s>>>(C, F, Cm, rt, omega, omega_t, cscale, damping, gather, g)
  if (d == 2) {
    if (g.stop) AD_LU(2, true); else AD_LU(2, false);
  } else {
    if (g.stop) AD_LU(3, true); else AD_LU(3, false);
  }
#undef AD_LU
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(int d, const LevelView<T>& F, const LevelView<T>& C, T* dst, const T* src,
                              const T* sub, hipStream_t s, const T* self, Gate g) {
  size_t nverts = d == 2 ? size_t(F.nv) * F.nv : size_t(F.nv) * F.nv * F.nv;
  if (nverts >= (size_t(1) << 32)) return hipErrorInvalidValue;
  unsigned nb = unsigned((nverts + 255) / 256);
#define AD_PA(DD, GG) k_prolong_add<T, DD, GG><<<nb, 256, 0, s>>>(F, C, dst, src, sub, self, g)
  if (d == 2) {
    if (g.stop) AD_PA(2, true); else AD_PA(2, false);
  } else {
    if (g.stop) AD_PA(3, true); else AD_PA(3, false);
  }
#undef AD_PA
  return hipGetLastError();
}

template <typename T, int D, int NT>
static hipError_t launch_chain_nt(const ProlongChainArgs<T>& a, hipStream_t s) {
  ChainDev<T, NT> dv{};
  for (int k = 0; k <= NT; ++k) {
    dv.lv[k].S = a.lv[k].S;
    dv.lv[k].sub = k < NT ? a.sub[k] : nullptr;
    dv.lv[k].out = (k > 0 && k < NT) ? a.out[k] : nullptr;
    dv.lv[k].pw = a.lv[k].pw;
    dv.lv[k].nv = a.lv[k].nv;
  }
  dv.self = a.self;
  dv.gate = a.gate;
  const int n = a.lv[NT].nv - 1;   // cells of the top target: tiles cover vertices 0 .. n-1
  dv.tiles0 = (n + ChainTile<D>::X - 1) / ChainTile<D>::X;
  dv.tiles1 = (n + ChainTile<D>::Y - 1) / ChainTile<D>::Y;
  const size_t nb = size_t(dv.tiles0) * dv.tiles1 * (D == 3 ? (n + ChainTile<D>::Z - 1) / ChainTile<D>::Z : 1);
  if (nb >= (size_t(1) << 31)) return hipErrorInvalidValue;
  if (a.gate.stop)
    k_prolong_chain<T, D, NT, true><<<unsigned(nb), kChainThreads, 0, s>>>(dv);
  else
    k_prolong_chain<T, D, NT, false><<<unsigned(nb), kChainThreads, 0, s>>>(dv);
  return hipGetLastError();
}

template <typename T, int D>
static hipError_t launch_chain_d(const ProlongChainArgs<T>& a, hipStream_t s) {
  switch (a.nt) {
    case 2: return launch_chain_nt<T, D, 2>(a, s);
    case 3: return launch_chain_nt<T, D, 3>(a, s);
    case 4: return launch_chain_nt<T, D, 4>(a, s);
    case 5: return launch_chain_nt<T, D, 5>(a, s);
    case 6: return launch_chain_nt<T, D, 6>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_prolong_chain(int d, const ProlongChainArgs<T>& a, hipStream_t s) {
  if (a.nt < 2 || a.nt > kMaxChain) return hipErrorInvalidValue;
  for (int k = 0; k < a.nt; ++k)
    if (a.lv[k + 1].nv - 1 != 3 * (a.lv[k].nv - 1) || !a.lv[k].S || (k > 0 && !a.out[k]))
      return hipErrorInvalidValue;
  if (!a.lv[a.nt].S) return hipErrorInvalidValue;
  return d == 2 ? launch_chain_d<T, 2>(a, s) : launch_chain_d<T, 3>(a, s);
}
template hipError_t launch_prolong_chain<double>(int, const ProlongChainArgs<double>&, hipStream_t);
template hipError_t launch_prolong_chain<float>(int, const ProlongChainArgs<float>&, hipStream_t);

template <typename T>
hipError_t launch_small_levels(int d, const SmallLevelsArgs<T>& a, size_t lds_bytes, hipStream_t s) {
  const bool g = a.gate.stop || a.rule.stop;
  if (d == 2) {
    if (g) k_small_levels<T, 2, true><<<1, kSmallThreads, lds_bytes, s>>>(a);
    else k_small_levels<T, 2, false><<<1, kSmallThreads, lds_bytes, s>>>(a);
  } else {
    if (g) k_small_levels<T, 3, true><<<1, kSmallThreads, lds_bytes, s>>>(a);
    else k_small_levels<T, 3, false><<<1, kSmallThreads, lds_bytes, s>>>(a);
  }
  return hipGetLastError();
}
template hipError_t launch_small_levels<double>(int, const SmallLevelsArgs<double>&, size_t, hipStream_t);
template hipError_t launch_small_levels<float>(int, const SmallLevelsArgs<float>&, size_t, hipStream_t);

template <bool G>
__global__ void __launch_bounds__(256) k_norm_finalize(const double* __restrict__ partials, int n,
                                                       double* __restrict__ out, Gate g, StopRule rule) {
  if (G && gated(g)) return;
  __shared__ double ss[256], sm[256];
  double s = 0.0, m = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    s += partials[2 * i];
    m = fmax(m, partials[2 * i + 1]);
  }
  ss[threadIdx.x] = s;
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      ss[threadIdx.x] += ss[threadIdx.x + w];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sqrt(ss[0]);
    out[1] = sm[0];
    if (G) apply_stop_rule(rule, out);
  }
}

// Reference streaming copy (roofline context): 16-byte non-temporal vectors, grid-stride.
typedef double dvec2 __attribute__((ext_vector_type(2)));
__global__ void __launch_bounds__(256) k_stream_copy(const dvec2* __restrict__ a, dvec2* __restrict__ b, size_t n) {
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += size_t(gridDim.x) * 256)
    __builtin_nontemporal_store(__builtin_nontemporal_load(&a[i]), &b[i]);
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t n16, hipStream_t s) {
  k_stream_copy<<<1024, 256, 0, s>>>(static_cast<const dvec2*>(src), static_cast<dvec2*>(dst), n16);
  return hipGetLastError();
}

hipError_t launch_norm_finalize(const double* partials, int n, double* out, hipStream_t s, Gate g, StopRule rule) {
  if (g.stop || rule.stop)
    k_norm_finalize<true><<<1, 256, 0, s>>>(partials, n, out, g, rule);
  else
    k_norm_finalize<false><<<1, 256, 0, s>>>(partials, n, out, g, rule);
  return hipGetLastError();
}

template hipError_t launch_fine_residual<double>(int, const LevelView<double>&, const double*, double*,
                                                 const double*, double*, double*, int, double, int, double*,
                                                 int, hipStream_t, Gate);
template hipError_t launch_fine_residual<float>(int, const LevelView<float>&, const float*, float*,
                                                const float*, float*, float*, int, float, int, double*, int,
                                                hipStream_t, Gate);
template hipError_t launch_level_update<double>(int, const LevelView<double>&, const LevelView<double>&,
                                                const LevelView<double>&, const RtSep<double>&, double, double,
                                                double, int, int, hipStream_t, Gate);
template hipError_t launch_level_update<float>(int, const LevelView<float>&, const LevelView<float>&,
                                               const LevelView<float>&, const RtSep<float>&, float, float, float,
                                               int, int, hipStream_t, Gate);
template hipError_t launch_prolong_add<double>(int, const LevelView<double>&, const LevelView<double>&,
                                               double*, const double*, const double*, hipStream_t, const double*,
                                               Gate);
template hipError_t launch_prolong_add<float>(int, const LevelView<float>&, const LevelView<float>&, float*,
                                              const float*, const float*, hipStream_t, const float*, Gate);

}  // namespace adafac
