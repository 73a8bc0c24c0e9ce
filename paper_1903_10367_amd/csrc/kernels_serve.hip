// Batched phase kernel of the request server: every active request, of any depth and
// dimension, advances by `steps` steps per round (an FP64 cycle, or an outer step of FP32
// cycles inside FP64 defect correction).
//
// A request's step is a chain of phases: the finest level's residual and Jacobi step, the norm
// evaluation with the stopping rule (Sec. 5), the FAS update of each coarser level (finest
// first), the prolongation of the summed corrections back up (coarsest first).  Each phase is
// cut into work items of a fixed number of vertices.  One launch runs one phase slot of one step
// for ALL requests (the slot-th phase of each request's chain), one workgroup per item, so the
// kernel boundary orders a request's phases and publishes their results across the chip's L2
// caches, and the number of launches per round is steps x the longest chain, whatever the
// number of requests.
//
// The per-vertex arithmetic is the one-kernel-per-step path's (fine residual and Jacobi step,
// level_update_vertex, prolong_value) and each request's norm partials are summed in a fixed
// order, so a request's iterates do not depend on the requests it is served with.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "adafac.h"
#include "adafac_internal.hpp"
#include "kernels_common.hpp"

namespace adafac {
namespace {

constexpr int NTS = 256;   // lanes per workgroup

template <int D>
__device__ __forceinline__ size_t nverts_of(int nv) {
  return D == 2 ? size_t(nv) * nv : size_t(nv) * nv * nv;
}

// Rows of a level's vertex lattice: row q holds the nv vertices (x, y, z) with y + nv z = q (2D:
// y = q).  Row-based items give every lane a fixed x and no per-vertex index division.
template <int D>
__device__ __forceinline__ size_t nrows_of(int nv) {
  return D == 2 ? size_t(nv) : size_t(nv) * nv;
}

// Lanes per lattice row: the smallest power of two covering the row's nv - 2 interior vertices
// (at most NTS); NTS / tpr rows are worked on at once, so small levels keep every lane busy.
__device__ __forceinline__ int row_lanes(int nv) {
  int t = 1;
  while (t < nv - 2 && t < NTS) t <<= 1;
  return t;
}

template <int D>
__device__ __forceinline__ void row_yz(unsigned q, int nv, int& y, int& z) {
  if (D == 2) {
    y = int(q);
    z = 0;
  } else {
    z = int(q / unsigned(nv));
    y = int(q - unsigned(z) * unsigned(nv));
  }
}

// (sum, max) over the workgroup into out[0], out[1] (thread 0), fixed order.
__device__ void wg_partials(double s, double m, double* out, double* ws, double* wm) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off);
    m = fmax(m, __shfl_xor(m, off));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    ws[w] = s;
    wm[w] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double st = 0.0, mt = 0.0;
    for (int k = 0; k < NTS / 64; ++k) {
      st += ws[k];
      mt = fmax(mt, wm[k]);
    }
    out[0] = st;
    out[1] = mt;
  }
}

// Residual r = b - A u of iterate uin on rows [q0, q1) of the finest level, its Jacobi step into
// uout, the injected correction (adAFAC-PI), norm partials.
template <typename T, int D>
__device__ void fine_items(const BatchReq& R, const BatchHier<T>& H, const T* uin, T* uout, unsigned q0, unsigned q1,
                           double& s, double& m) {
  const int L = R.L;
  const bool pi = R.damping == ADAFAC_DAMP_PI && L > R.lmin;
  const LevelView<T>& F = H.v[L];
  const LevelView<T>& Lm1 = H.v[L > R.lmin ? L - 1 : L];
  const T omega = T(R.omega);
  const int nv = F.nv;
  const int tpr = row_lanes(nv);
  for (unsigned q = q0 + threadIdx.x / unsigned(tpr); q < q1; q += unsigned(NTS / tpr)) {
    int y, z;
    row_yz<D>(q, nv, y, z);
    if (y == 0 || y == nv - 1 || (D == 3 && (z == 0 || z == nv - 1))) continue;
    for (int x = 1 + int(threadIdx.x % unsigned(tpr)); x < nv - 1; x += tpr) {
      const size_t i = lin<D>(x, y, z, nv);
      T dg;
      const T au = apply_level_op<T, D>(F, x, y, z, dg, [&](int dx, int dy, int dz) {
        return uin[lin<D>(x + dx, y + dy, z + dz, nv)];
      });
      const T res = H.bfine[i] - au;
      const T c = omega * res / dg;
      H.rfine[i] = res;
      uout[i] = uin[i] + c;
      if (pi && x % 3 == 0 && y % 3 == 0 && (D == 2 || z % 3 == 0))
        Lm1.ic[lin<D>(x / 3, y / 3, z / 3, Lm1.nv)] = c;
      const double rd = double(res);
      s += double(F.hd) * rd * rd;
      m = fmax(m, fabs(rd));
    }
  }
}

// FAS update of level l on vertices [v0, v1) (gathering R r, R~ r and I u from level l + 1, or
// with them already written by the finest-level sweep).
template <typename T, int D>
__device__ __forceinline__ void level_items(const BatchReq& R, const BatchHier<T>& H, const T* uin, int l, int gather, size_t v0,
                            size_t v1) {
  const int L = R.L;
  LevelView<T> Fv = H.v[l + 1];
  if (l + 1 == L) {
    Fv.u = const_cast<T*>(uin);
    Fv.r = H.rfine;
  }
  const LevelView<T> Cm = l > R.lmin ? H.v[l - 1] : LevelView<T>{};
  const T cscale = T(R.damping == ADAFAC_DAMP_EXP ? pow(R.omega_hat, double(L - l)) : 1.0);
  for (size_t i = v0 + threadIdx.x; i < v1; i += NTS)
    level_update_vertex<T, D>(H.v[l], Fv, Cm, H.rts, T(R.omega), T(R.omega_t), cscale, R.damping, gather, i);
}

// S_l += P (S_{l-1} - I c_l) on rows [q0, q1) of level l (the finest level: u_out).  self: under
// adAFAC-PI with the finest level swept, level L-1 also subtracts I c_L, which the sweep stored
// there, so that the pending P S_{L-1} is P (S_{L-1} - I c_L).
template <typename T, int D>
__device__ __forceinline__ void prolong_items(const BatchReq& R, const BatchHier<T>& H, T* uout, int l, int self, unsigned q0,
                              unsigned q1) {
  const bool pi = R.damping == ADAFAC_DAMP_PI;
  const LevelView<T>& F = H.v[l];
  const LevelView<T>& C = H.v[l - 1];
  T* dst = l == R.L ? uout : F.S;
  const int nv = F.nv;
  const int tpr = row_lanes(nv);
  for (unsigned q = q0 + threadIdx.x / unsigned(tpr); q < q1; q += unsigned(NTS / tpr)) {
    int y, z;
    row_yz<D>(q, nv, y, z);
    if (y == 0 || y == nv - 1 || (D == 3 && (z == 0 || z == nv - 1))) continue;
    for (int x = 1 + int(threadIdx.x % unsigned(tpr)); x < nv - 1; x += tpr) {
      const size_t i = lin<D>(x, y, z, nv);
      T v = prolong_value<T, D>(F, C, x, y, z, C.S, pi ? C.ic : nullptr);
      if (self) v -= F.ic[i];
      dst[i] += v;
    }
  }
}

// The FAS updates of levels hi .. l_min and the prolongations into levels l_min + 1 .. hi, in
// that order, by one workgroup (a barrier after each level): the per-vertex arithmetic of
// level_items and prolong_items.  gather_hi: level hi gathers from level hi + 1; self: the
// prolongation into level L-1 subtracts I c_L.
template <typename T, int D>
__device__ void small_items(const BatchReq& R, const BatchHier<T>& H, const T* uin, T* uout, int hi, int gather_hi,
                            int self) {
  for (int l = hi; l >= R.lmin; --l) {
    level_items<T, D>(R, H, uin, l, l == hi ? gather_hi : 1, 0, nverts_of<D>(H.v[l].nv));
    __syncthreads();
  }
  for (int l = R.lmin + 1; l <= hi; ++l) {
    prolong_items<T, D>(R, H, uout, l, (self && l == R.L - 1) ? 1 : 0, 0u, unsigned(nrows_of<D>(H.v[l].nv)));
    __syncthreads();
  }
}

// FP32_REFINED: u += e (pend: u += e + P S_{L-1}, the prolongation the last inner sweep left
// pending, summed in FP32 as by the one-kernel-per-step path) on rows [q0, q1) of the finest level.
template <int D>
__device__ void adde_items(const BatchReq& R, const float* e, int pend, unsigned q0, unsigned q1) {
  double* u = R.h64.ufine[0];
  const LevelView<float>& F = R.h32.v[R.L];
  const LevelView<float>& C = R.h32.v[R.L - 1];
  const int nv = R.h64.v[R.L].nv;
  const int tpr = row_lanes(nv);
  for (unsigned q = q0 + threadIdx.x / unsigned(tpr); q < q1; q += unsigned(NTS / tpr)) {
    int y, z;
    row_yz<D>(q, nv, y, z);
    if (y == 0 || y == nv - 1 || (D == 3 && (z == 0 || z == nv - 1))) continue;
    for (int x = 1 + int(threadIdx.x % unsigned(tpr)); x < nv - 1; x += tpr) {
      const size_t i = lin<D>(x, y, z, nv);
      float c = e[i];
      if (pend) c += prolong_value<float, D>(F, C, x, y, z, C.S, nullptr);
      u[i] += double(c);
    }
  }
}

// FP32_REFINED: r32 = float(b - A u) in FP64 on rows [q0, q1), norm partials.
template <int D>
__device__ void defect_items(const BatchReq& R, unsigned q0, unsigned q1, double& s, double& m) {
  const BatchHier<double>& H = R.h64;
  const LevelView<double>& F = H.v[R.L];
  const double* u = H.ufine[0];
  const int nv = F.nv;
  const int tpr = row_lanes(nv);
  for (unsigned q = q0 + threadIdx.x / unsigned(tpr); q < q1; q += unsigned(NTS / tpr)) {
    int y, z;
    row_yz<D>(q, nv, y, z);
    if (y == 0 || y == nv - 1 || (D == 3 && (z == 0 || z == nv - 1))) continue;
    for (int x = 1 + int(threadIdx.x % unsigned(tpr)); x < nv - 1; x += tpr) {
      const size_t i = lin<D>(x, y, z, nv);
      double dg;
      const double au = apply_level_op<double, D>(F, x, y, z, dg, [&](int dx, int dy, int dz) {
        return u[lin<D>(x + dx, y + dy, z + dz, nv)];
      });
      const double res = H.bfine[i] - au;
      R.h32.bfine[i] = float(res);
      s += F.hd * res * res;
      m = fmax(m, fabs(res));
    }
  }
}

// The norms of the measured iterate from its phase's partials (fixed order), the stopping rule,
// and the item count after which the request's later items do no work.  need: this item's own
// position in the request's item sequence.
__device__ void final_item(const BatchReq& R, BatchState& S, const ServeSeg& g, int j, unsigned long long need,
                           double* ws, double* wm, double* out) {
  double s = 0.0, m = 0.0;
  for (int t = threadIdx.x; t < g.nparts; t += NTS) {
    s += R.partials[2 * t];
    m = fmax(m, R.partials[2 * t + 1]);
  }
  wg_partials(s, m, out, ws, wm);
  if (threadIdx.x != 0) return;
  const double l2 = sqrt(out[0]);
  if (S.cycles == 0) S.r0 = l2;
  S.l2h = l2;
  S.linf = out[1];
  int st = 0;
  if (!(l2 == l2) || l2 > 1e300 || l2 > 1e3 * S.r0) st = 2;
  else if (S.r0 == 0.0 || l2 / S.r0 <= R.tol) st = 1;
  S.cycles += 1;
  if (!st && S.cycles >= R.max_cycles) st = 3;
  S.status = st;
  // the iterate it produces (FP64), or the one it measured (after the one-pass 3D defect)
  if (R.precision == ADAFAC_PREC_FP64 || g.pend) S.cur = g.cur0 ^ ((j * g.cps + g.sub + 1) & 1);
  // FP64: the rest of this cycle still runs (it produces the result); FP32_REFINED: the outer
  // iterate just measured is the result
  if (st) S.stop_need = need + 1 + (unsigned long long)g.run_after;
}

// CLS: the kernel class (serve_class) whose phase kinds this instance compiles; each class has
// its own register budget, so that the light phases are not held to the heaviest one's occupancy.
template <int D, int CLS>
__device__ void run_item(const BatchReq& R, BatchState& S, const ServeSeg& g, int j, unsigned long long need, int t,
                         double* ws, double* wm, double* red) {
  const int L = R.L;
  const bool fp64 = R.precision == ADAFAC_PREC_FP64;
  // FP64 iterates ping-pong (cycle g.sub of the step's g.cps cycles); FP32 inner cycle i reads
  // e_i (e_0 = 0) and writes e_{i+1}
  const int cur = g.cur0 ^ ((j * g.cps + g.sub) & 1);
  const double* u64in = R.h64.ufine[cur];
  double* u64out = R.h64.ufine[1 - cur];
  const float* u32in = g.sub == 0 ? R.ezero : R.h32.ufine[g.sub & 1];
  float* u32out = R.h32.ufine[(g.sub + 1) & 1];
  const int nvl = fp64 ? R.h64.v[g.level].nv : R.h32.v[g.level].nv;
  // row-based phases: item t covers rows [q0, q1); the coarse FAS updates: vertices [v0, v1)
  const unsigned q0 = unsigned(t) * unsigned(g.tile);
  const unsigned q1 = unsigned(min(size_t(q0) + size_t(g.tile), nrows_of<D>(nvl)));
  double s = 0.0, m = 0.0;
  if (serve_class(g.kind) != CLS) return;
  switch (g.kind) {
    case SERVE_FINE:
      if constexpr (CLS != SERVE_CLS_HEAVY) break;
      if (fp64) {
        fine_items<double, D>(R, R.h64, u64in, u64out, q0, q1, s, m);
        wg_partials(s, m, R.partials + 2 * t, ws, wm);
      } else {
        fine_items<float, D>(R, R.h32, u32in, u32out, q0, q1, s, m);
      }
      break;
    case SERVE_LEVEL: {
      if constexpr (CLS != SERVE_CLS_HEAVY) break;
      const size_t v0 = size_t(t) * size_t(g.tile);
      const size_t v1 = min(v0 + size_t(g.tile), nverts_of<D>(nvl));
      if (fp64) level_items<double, D>(R, R.h64, u64in, g.level, g.gather, v0, v1);
      else level_items<float, D>(R, R.h32, u32in, g.level, g.gather, v0, v1);
      break;
    }
    case SERVE_SMALL:
      if constexpr (CLS != SERVE_CLS_SMALL) break;
      if (fp64) small_items<double, D>(R, R.h64, u64in, u64out, g.level, g.gather, g.pend);
      else small_items<float, D>(R, R.h32, u32in, u32out, g.level, g.gather, g.pend);
      break;
    case SERVE_PROLONG:
      if constexpr (CLS != SERVE_CLS_LIGHT) break;
      if (fp64) prolong_items<double, D>(R, R.h64, u64out, g.level, g.pend, q0, q1);
      else prolong_items<float, D>(R, R.h32, u32out, g.level, g.pend, q0, q1);
      break;
    case SERVE_ADDE:
      if constexpr (CLS != SERVE_CLS_LIGHT) break;
      // the correction of the previous outer step (none before the first)
      if (S.cycles > 0) adde_items<D>(R, R.h32.ufine[R.inner_k & 1], g.pend, q0, q1);
      break;
    case SERVE_DEFECT:
      if constexpr (CLS != SERVE_CLS_HEAVY) break;
      defect_items<D>(R, q0, q1, s, m);
      wg_partials(s, m, R.partials + 2 * t, ws, wm);
      break;
    case SERVE_FINAL:
      if constexpr (CLS != SERVE_CLS_HEAVY) break;
      final_item(R, S, g, j, need, ws, wm, red);
      break;
    default:
      break;
  }
  (void)L;
}

// One phase slot of one step of every batched request, the phases of one kernel class:
// workgroup b runs item b of the class's work list (segments ordered by request, items numbered
// within the list).
template <int CLS>
__global__ void __launch_bounds__(NTS) k_serve_phase(const BatchReq* __restrict__ reqs, BatchState* states,
                                                     const ServeSeg* __restrict__ segs, int nseg, int j) {
  __shared__ double ws[NTS / 64], wm[NTS / 64], red[2];
  const int q = int(blockIdx.x);
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].item0 <= q) lo = mid;
    else hi = mid - 1;
  }
  const ServeSeg& g = segs[lo];
  const int t = q - g.item0;
  if (t >= g.ntile) return;
  const BatchReq& R = reqs[g.req];
  BatchState& S = states[g.req];
  // the item's position in its request's sequence; at or beyond the stopping point it does no
  // work (the request's earlier FINAL item set it, in an earlier launch)
  const unsigned long long need = g.base + (unsigned long long)j * (unsigned long long)g.per_step +
                                  (unsigned long long)g.need_off + (unsigned long long)t;
  if (need >= S.stop_need) return;
  if (R.dim == 2) run_item<2, CLS>(R, S, g, j, need, t, ws, wm, red);
  else run_item<3, CLS>(R, S, g, j, need, t, ws, wm, red);
}

}  // namespace

// Phase slot launch of kernel class cls: nitems workgroups over its nseg segments, step j of the
// round.
hipError_t launch_serve_phase(int cls, const BatchReq* reqs, BatchState* states, const ServeSeg* segs, int nseg,
                              int nitems, int j, hipStream_t s) {
  if (nseg <= 0 || nitems <= 0) return hipSuccess;
  switch (cls) {
    case SERVE_CLS_LIGHT: k_serve_phase<SERVE_CLS_LIGHT><<<nitems, NTS, 0, s>>>(reqs, states, segs, nseg, j); break;
    case SERVE_CLS_HEAVY: k_serve_phase<SERVE_CLS_HEAVY><<<nitems, NTS, 0, s>>>(reqs, states, segs, nseg, j); break;
    case SERVE_CLS_SMALL: k_serve_phase<SERVE_CLS_SMALL><<<nitems, NTS, 0, s>>>(reqs, states, segs, nseg, j); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace adafac
