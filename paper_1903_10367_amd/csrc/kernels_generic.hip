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

template <typename T, int D>
__global__ void __launch_bounds__(256) k_fine_residual(LevelView<T> F, const T* __restrict__ uin,
                                                       T* __restrict__ uout, const T* __restrict__ b,
                                                       T* __restrict__ r, T* __restrict__ ic_coarse,
                                                       int nvc, T omega, int pi,
                                                       double* __restrict__ partials) {
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

template <typename T, int D>
__global__ void __launch_bounds__(256) k_level_update(LevelView<T> C, LevelView<T> F, LevelView<T> Cm,
                                                      RtSep<T> rts, T omega, T omega_t, T cscale,
                                                      int damping, int gather) {
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

template <typename T, int D>
__global__ void __launch_bounds__(kSmallThreads) k_small_levels(SmallLevelsArgs<T> a) {
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
template <typename T, int D>
__global__ void __launch_bounds__(256) k_prolong_add(LevelView<T> F, LevelView<T> C, T* __restrict__ dst,
                                                     const T* __restrict__ src, const T* __restrict__ sub,
                                                     const T* __restrict__ self) {
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
                                hipStream_t s) {
  if (d == 2)
    k_fine_residual<T, 2><<<nblocks, 256, 0, s>>>(F, uin, uout, b, r, ic_coarse, nvc, omega, pi, partials);
  else
    k_fine_residual<T, 3><<<nblocks, 256, 0, s>>>(F, uin, uout, b, r, ic_coarse, nvc, omega, pi, partials);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_level_update(int d, const LevelView<T>& C, const LevelView<T>& F, const LevelView<T>& Cm,
                               const RtSep<T>& rt, T omega, T omega_t, T cscale, int damping, int gather,
                               hipStream_t s) {
  size_t nverts = d == 2 ? size_t(C.nv) * C.nv : size_t(C.nv) * C.nv * C.nv;
  if (nverts >= (size_t(1) << 32)) return hipErrorInvalidValue;
  unsigned nb = unsigned((nverts + 255) / 256);
  if (d == 2)
    k_level_update<T, 2><<<nb, 256, 0, s>>>(C, F, Cm, rt, omega, omega_t, cscale, damping, gather);
  else
    k_level_update<T, 3><<<nb, 256, 0, s>>>(C, F, Cm, rt, omega, omega_t, cscale, damping, gather);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(int d, const LevelView<T>& F, const LevelView<T>& C, T* dst, const T* src,
                              const T* sub, hipStream_t s, const T* self) {
  size_t nverts = d == 2 ? size_t(F.nv) * F.nv : size_t(F.nv) * F.nv * F.nv;
  if (nverts >= (size_t(1) << 32)) return hipErrorInvalidValue;
  unsigned nb = unsigned((nverts + 255) / 256);
  if (d == 2)
    k_prolong_add<T, 2><<<nb, 256, 0, s>>>(F, C, dst, src, sub, self);
  else
    k_prolong_add<T, 3><<<nb, 256, 0, s>>>(F, C, dst, src, sub, self);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_small_levels(int d, const SmallLevelsArgs<T>& a, size_t lds_bytes, hipStream_t s) {
  if (d == 2)
    k_small_levels<T, 2><<<1, kSmallThreads, lds_bytes, s>>>(a);
  else
    k_small_levels<T, 3><<<1, kSmallThreads, lds_bytes, s>>>(a);
  return hipGetLastError();
}
template hipError_t launch_small_levels<double>(int, const SmallLevelsArgs<double>&, size_t, hipStream_t);
template hipError_t launch_small_levels<float>(int, const SmallLevelsArgs<float>&, size_t, hipStream_t);

__global__ void __launch_bounds__(256) k_norm_finalize(const double* __restrict__ partials, int n,
                                                       double* __restrict__ out) {
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

hipError_t launch_norm_finalize(const double* partials, int n, double* out, hipStream_t s) {
  k_norm_finalize<<<1, 256, 0, s>>>(partials, n, out);
  return hipGetLastError();
}

template hipError_t launch_fine_residual<double>(int, const LevelView<double>&, const double*, double*,
                                                 const double*, double*, double*, int, double, int, double*,
                                                 int, hipStream_t);
template hipError_t launch_fine_residual<float>(int, const LevelView<float>&, const float*, float*,
                                                const float*, float*, float*, int, float, int, double*, int,
                                                hipStream_t);
template hipError_t launch_level_update<double>(int, const LevelView<double>&, const LevelView<double>&,
                                                const LevelView<double>&, const RtSep<double>&, double, double,
                                                double, int, int, hipStream_t);
template hipError_t launch_level_update<float>(int, const LevelView<float>&, const LevelView<float>&,
                                               const LevelView<float>&, const RtSep<float>&, float, float, float,
                                               int, int, hipStream_t);
template hipError_t launch_prolong_add<double>(int, const LevelView<double>&, const LevelView<double>&,
                                               double*, const double*, const double*, hipStream_t, const double*);
template hipError_t launch_prolong_add<float>(int, const LevelView<float>&, const LevelView<float>&, float*,
                                              const float*, const float*, hipStream_t, const float*);

}  // namespace adafac
