// Batched work-queue kernel of the request server: every active small request advances in one
// launch.  A workgroup takes the next request from the launch's work list (global counter),
// runs up to `budget` cycles of it (FP64 form) or outer steps (FP32 cycles inside FP64 defect
// correction), all levels in sequence with workgroup barriers between them, and takes the next
// request; the launch ends when the list is exhausted, so every wave reaches the exit.
//
// One cycle is the additive adAFAC cycle of eq. (adaFACx) / Algorithm 1 (Sec. 3.1) with the
// FAS right-hand sides of Sec. 2.4, computed with the same per-vertex device functions as the
// one-kernel-per-step path (fine residual and Jacobi step, FAS update of every coarse level,
// prolongation of the summed corrections), so a request's iterates do not depend on the mix
// of requests it is served with.  Norms (Sec. 5) are reduced inside the workgroup.
#include <hip/hip_runtime.h>

#include "adafac.h"
#include "adafac_internal.hpp"
#include "kernels_common.hpp"

namespace adafac {
namespace {

constexpr int NTB = 512;           // lanes per workgroup (eight wave64)

// (sum, max) over the workgroup, result in every lane
__device__ __forceinline__ void wg_reduce(double& s, double& m, double* ws, double* wm) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off);
    m = fmax(m, __shfl_xor(m, off));
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    ws[w] = s;
    wm[w] = m;
  }
  __syncthreads();
  s = 0.0;
  m = 0.0;
  for (int k = 0; k < NTB / 64; ++k) {
    s += ws[k];
    m = fmax(m, wm[k]);
  }
}

template <int D>
__device__ __forceinline__ size_t nverts_of(int nv) {
  return D == 2 ? size_t(nv) * nv : size_t(nv) * nv * nv;
}

// One cycle of hierarchy H in T: residual r = b - A u of iterate uin (norms into s, m), its
// Jacobi step into uout, the FAS updates of levels L-1 .. lmin, and u_out += P S.
template <typename T, int D>
__device__ __attribute__((noinline)) void wg_cycle(const BatchReq& R, const BatchHier<T>& H, const T* uin, T* uout, double& s,
                         double& m) {
  const int L = R.L, lmin = R.lmin, tid = threadIdx.x;
  const bool pi = R.damping == ADAFAC_DAMP_PI;
  const T omega = T(R.omega), omega_t = T(R.omega_t);
  LevelView<T> F = H.v[L];
  F.u = const_cast<T*>(uin);
  F.r = H.rfine;
  const LevelView<T> Lm1 = L > lmin ? H.v[L - 1] : LevelView<T>{};
  const int nv = F.nv;
  s = 0.0;
  m = 0.0;
  for (size_t i = tid; i < nverts_of<D>(nv); i += NTB) {
    const int x = int(i % nv), y = int((i / nv) % nv), z = D == 3 ? int(i / (size_t(nv) * nv)) : 0;
    if (!is_interior<D>(x, y, z, nv)) continue;
    T dg;
    const T au = apply_level_op<T, D>(F, x, y, z, dg, [&](int dx, int dy, int dz) {
      return uin[lin<D>(x + dx, y + dy, z + dz, nv)];
    });
    const T res = H.bfine[i] - au;
    const T c = omega * res / dg;
    H.rfine[i] = res;
    uout[i] = uin[i] + c;
    if (pi && L > lmin && x % 3 == 0 && y % 3 == 0 && (D == 2 || z % 3 == 0))
      Lm1.ic[lin<D>(x / 3, y / 3, z / 3, Lm1.nv)] = c;
    const double rd = double(res);
    s += double(F.hd) * rd * rd;
    m = fmax(m, fabs(rd));
  }
  __syncthreads();
  for (int l = L - 1; l >= lmin; --l) {
    const LevelView<T>& C = H.v[l];
    const LevelView<T>& Fv = l + 1 == L ? F : H.v[l + 1];
    const LevelView<T> Cm = l > lmin ? H.v[l - 1] : LevelView<T>{};
    const T cscale = T(R.damping == ADAFAC_DAMP_EXP ? pow(R.omega_hat, double(L - l)) : 1.0);
    for (size_t i = tid; i < nverts_of<D>(C.nv); i += NTB)
      level_update_vertex<T, D>(C, Fv, Cm, H.rts, omega, omega_t, cscale, R.damping, 1, i);
    __syncthreads();
  }
  for (int l = lmin + 1; l <= L; ++l) {
    const LevelView<T>& Fv = l == L ? F : H.v[l];
    const LevelView<T>& C = H.v[l - 1];
    T* dst = l == L ? uout : Fv.S;
    const int nvf = Fv.nv;
    for (size_t i = tid; i < nverts_of<D>(nvf); i += NTB) {
      const int x = int(i % nvf), y = int((i / nvf) % nvf), z = D == 3 ? int(i / (size_t(nvf) * nvf)) : 0;
      if (!is_interior<D>(x, y, z, nvf)) continue;
      dst[i] += prolong_value<T, D>(Fv, C, x, y, z, C.S, pi ? C.ic : nullptr);
    }
    __syncthreads();
  }
}

// FP64 defect of the FP32_REFINED form: u += e (when add_e), r32 = float(b - A u), norms.
template <int D>
__device__ __attribute__((noinline)) void wg_defect(const BatchReq& R, const float* e, bool add_e, double& s, double& m) {
  const BatchHier<double>& H = R.h64;
  const LevelView<double>& F = H.v[R.L];
  double* u = H.ufine[0];
  const int nv = F.nv, tid = threadIdx.x;
  if (add_e) {
    for (size_t i = tid; i < nverts_of<D>(nv); i += NTB) {
      const int x = int(i % nv), y = int((i / nv) % nv), z = D == 3 ? int(i / (size_t(nv) * nv)) : 0;
      if (is_interior<D>(x, y, z, nv)) u[i] += double(e[i]);
    }
    __syncthreads();
  }
  s = 0.0;
  m = 0.0;
  for (size_t i = tid; i < nverts_of<D>(nv); i += NTB) {
    const int x = int(i % nv), y = int((i / nv) % nv), z = D == 3 ? int(i / (size_t(nv) * nv)) : 0;
    if (!is_interior<D>(x, y, z, nv)) continue;
    double dg;
    const double au = apply_level_op<double, D>(F, x, y, z, dg, [&](int dx, int dy, int dz) {
      return u[lin<D>(x + dx, y + dy, z + dz, nv)];
    });
    const double res = H.bfine[i] - au;
    R.h32.bfine[i] = float(res);
    s += F.hd * res * res;
    m = fmax(m, fabs(res));
  }
  __syncthreads();
}

// status after measuring iterate n with norms (s = sum h^d r^2, m = max |r|); lane 0 only
__device__ __forceinline__ int assess(BatchState& S, double s, double m, double tol) {
  const double l2 = sqrt(s);
  if (S.cycles == 0) S.r0 = l2;
  S.l2h = l2;
  S.linf = m;
  if (!(l2 == l2) || l2 > 1e300 || l2 > 1e3 * S.r0) return 2;
  if (S.r0 == 0.0 || l2 / S.r0 <= tol) return 1;
  return 0;
}

template <int D>
__device__ void serve(const BatchReq& R, BatchState& S, int budget, double* ws, double* wm, int* flag) {
  const int tid = threadIdx.x;
  for (int k = 0; k < budget; ++k) {
    if (tid == 0) *flag = S.status == 0 && S.cycles < R.max_cycles ? 0 : 1;
    __syncthreads();
    const int stop = *flag;
    __syncthreads();
    if (stop) break;
    double s, m;
    if (R.precision == ADAFAC_PREC_FP64) {
      const int cur = S.cur;
      wg_cycle<double, D>(R, R.h64, R.h64.ufine[cur], R.h64.ufine[1 - cur], s, m);
      wg_reduce(s, m, ws, wm);
      if (tid == 0) {
        // the cycle that measured iterate n produced n+1: it is the result when n met the tolerance
        const int st = assess(S, s, m, R.tol);
        S.cur = 1 - cur;
        S.cycles += 1;
        S.status = st ? st : (S.cycles >= R.max_cycles ? 3 : 0);
      }
    } else {
      wg_defect<D>(R, R.h32.ufine[S.cur], S.cycles > 0, s, m);
      wg_reduce(s, m, ws, wm);
      if (tid == 0) {
        const int st = assess(S, s, m, R.tol);
        S.cycles += 1;
        S.status = st ? st : (S.cycles >= R.max_cycles ? 3 : 0);
        *flag = S.status;
      }
      __syncthreads();
      const int done = *flag;
      __syncthreads();
      if (done) break;      // the outer iterate itself is the result
      // inner_k FP32 cycles on A e = r from e = 0; e ends in ufine[cur] of the inner hierarchy
      int cur = 0;
      for (int j = 0; j < R.inner_k; ++j) {
        const float* uin = j == 0 ? R.ezero : R.h32.ufine[cur];
        float* uout = R.h32.ufine[1 - cur];
        wg_cycle<float, D>(R, R.h32, uin, uout, s, m);
        cur = 1 - cur;
      }
      if (tid == 0) S.cur = cur;
      __syncthreads();
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(NTB) k_batch_serve(const BatchReq* __restrict__ reqs, BatchState* states,
                                                     const int* __restrict__ work, int nwork, int* next, int budget) {
  __shared__ double ws[NTB / 64], wm[NTB / 64];
  __shared__ int item_s, flag_s;
  for (;;) {
    if (threadIdx.x == 0) item_s = atomicAdd(next, 1);
    __syncthreads();
    const int item = item_s;
    __syncthreads();
    if (item >= nwork) return;
    const int ri = work[item];
    const BatchReq& R = reqs[ri];
    if (R.dim == 2)
      serve<2>(R, states[ri], budget, ws, wm, &flag_s);
    else
      serve<3>(R, states[ri], budget, ws, wm, &flag_s);
  }
}

}  // namespace

// work: indices into reqs of the requests to advance; next: a device int the caller has set
// to zero on the stream.  One workgroup per request while there are fewer requests than
// `max_groups`, else max_groups workgroups that share the list.
hipError_t launch_batch_serve(const BatchReq* reqs, BatchState* states, const int* work, int nwork, int* next,
                              int budget, int max_groups, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  const int groups = nwork < max_groups ? nwork : max_groups;
  k_batch_serve<<<groups, NTB, 0, s>>>(reqs, states, work, nwork, next, budget);
  return hipGetLastError();
}

}  // namespace adafac
