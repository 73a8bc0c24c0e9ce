// Device helpers shared by the adAFAC kernels: lattice indexing, the level operator,
// transfer weights and block reductions.
#pragma once
#include <hip/hip_runtime.h>

#include "adafac_internal.hpp"

namespace adafac {

template <int D>
__device__ __forceinline__ size_t lin(int x, int y, int z, int nv) {
  return D == 2 ? size_t(y) * nv + x : (size_t(z) * nv + y) * nv + x;
}

template <int D>
__device__ __forceinline__ bool is_interior(int x, int y, int z, int nv) {
  bool in = x > 0 && x < nv - 1 && y > 0 && y < nv - 1;
  if (D == 3) in = in && z > 0 && z < nv - 1;
  return in;
}

template <int D>
__device__ __forceinline__ int rt_index(int ox, int oy, int oz) {
  return D == 2 ? (ox + 2) + 5 * (oy + 2) : (ox + 2) + 5 * (oy + 2) + 25 * (oz + 2);
}

// cell / bs for a block size bs = 3^m: a multiply-high by ceil(2^32 / bs), exact for cell
// indices below 2^16 (the error term cell * (bsm bs - 2^32) stays below 2^32 / bs)
template <typename T>
__device__ __forceinline__ int block_of(const LevelView<T>& L, int c) {
  return L.bsm ? int(__umulhi(unsigned(c), L.bsm)) : c;
}

template <typename T, int D>
__device__ __forceinline__ T eps_cell(const LevelView<T>& L, int cx, int cy, int cz) {
  if (!L.eps) return T(1);
  const int bx = block_of(L, cx), by = block_of(L, cy);
  if (D == 2) return L.eps[by * L.nb + bx];
  const int bz = block_of(L, cz);
  return L.eps[(bz * L.nb + by) * L.nb + bx];
}

// A_l u at an interior vertex; U(dx, dy, dz) returns u at the neighbour offset.  dg receives
// the diagonal.  Q1 levels: element-wise sum over the 2^d adjacent cells of
// eps_c h^(d-2) K[i][j] u_j with the d-linear element matrix (2D: 2/3 on the diagonal,
// -1/6 along an edge, -1/3 across; 3D: 1/3, 0, -1/12 for face and body diagonals).
// Stored levels: the 3^d Galerkin stencil.
template <typename T, int D, typename F>
__device__ __forceinline__ T apply_level_op(const LevelView<T>& L, int x, int y, int z, T& dg, F&& U) {
  if (L.fem) {
    const T u0 = U(0, 0, 0);
    T s = T(0), es = T(0);
    if (D == 2) {
#pragma unroll
      for (int sy = -1; sy <= 1; sy += 2)
#pragma unroll
        for (int sx = -1; sx <= 1; sx += 2) {
          T e = eps_cell<T, D>(L, x + (sx < 0 ? -1 : 0), y + (sy < 0 ? -1 : 0), 0);
          s += e * (T(2.0 / 3.0) * u0 - T(1.0 / 6.0) * (U(sx, 0, 0) + U(0, sy, 0)) - T(1.0 / 3.0) * U(sx, sy, 0));
          es += e;
        }
      dg = T(2.0 / 3.0) * es;
      return s;
    } else {
#pragma unroll
      for (int sz = -1; sz <= 1; sz += 2)
#pragma unroll
        for (int sy = -1; sy <= 1; sy += 2)
#pragma unroll
          for (int sx = -1; sx <= 1; sx += 2) {
            T e = eps_cell<T, D>(L, x + (sx < 0 ? -1 : 0), y + (sy < 0 ? -1 : 0), z + (sz < 0 ? -1 : 0));
            s += e * (T(1.0 / 3.0) * u0 -
                      T(1.0 / 12.0) * (U(sx, sy, 0) + U(sx, 0, sz) + U(0, sy, sz) + U(sx, sy, sz)));
            es += e;
          }
      dg = L.h * T(1.0 / 3.0) * es;
      return L.h * s;
    }
  }
  const int nv = L.nv;
  const size_t i = lin<D>(x, y, z, nv);
  const T* st = L.st + i * (D == 2 ? 9 : 27);
  T s = T(0);
  const int zlo = D == 3 ? -1 : 0, zhi = D == 3 ? 1 : 0;
  for (int oz = zlo; oz <= zhi; ++oz)
    for (int oy = -1; oy <= 1; ++oy)
      for (int ox = -1; ox <= 1; ++ox)
        s += st[(ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)] * U(ox, oy, oz);
  dg = L.dg[i];
  return s;
}

// A_l u at an interior vertex from its 3^d neighbourhood nb[(ox+1) + 3 (oy+1) + 9 (oz+1)]
// (already in registers); same arithmetic as apply_level_op.
template <typename T, int D>
__device__ __forceinline__ T apply_level_op_nb(const LevelView<T>& L, int x, int y, int z, const T* nb, T& dg) {
  auto U = [&](int dx, int dy, int dz) { return nb[(dx + 1) + 3 * (dy + 1) + (D == 3 ? 9 * (dz + 1) : 0)]; };
  if (L.fem) {
    const T u0 = U(0, 0, 0);
    T s = T(0), es = T(0);
    if (D == 2) {
#pragma unroll
      for (int sy = -1; sy <= 1; sy += 2)
#pragma unroll
        for (int sx = -1; sx <= 1; sx += 2) {
          T e = eps_cell<T, D>(L, x + (sx < 0 ? -1 : 0), y + (sy < 0 ? -1 : 0), 0);
          s += e * (T(2.0 / 3.0) * u0 - T(1.0 / 6.0) * (U(sx, 0, 0) + U(0, sy, 0)) - T(1.0 / 3.0) * U(sx, sy, 0));
          es += e;
        }
      dg = T(2.0 / 3.0) * es;
      return s;
    }
#pragma unroll
    for (int sz = -1; sz <= 1; sz += 2)
#pragma unroll
      for (int sy = -1; sy <= 1; sy += 2)
#pragma unroll
        for (int sx = -1; sx <= 1; sx += 2) {
          T e = eps_cell<T, D>(L, x + (sx < 0 ? -1 : 0), y + (sy < 0 ? -1 : 0), z + (sz < 0 ? -1 : 0));
          s += e * (T(1.0 / 3.0) * u0 - T(1.0 / 12.0) * (U(sx, sy, 0) + U(sx, 0, sz) + U(0, sy, sz) + U(sx, sy, sz)));
          es += e;
        }
    dg = L.h * T(1.0 / 3.0) * es;
    return L.h * s;
  }
  const size_t i = lin<D>(x, y, z, L.nv);
  const T* st = L.st + i * (D == 2 ? 9 : 27);
  T s = T(0);
#pragma unroll
  for (int t = 0; t < (D == 2 ? 9 : 27); ++t) s += st[t] * nb[t];
  dg = L.dg[i];
  return s;
}

// P(f <- c) of the transfer from the next coarser level into level F (R = P^T).
template <typename T, int D>
__device__ __forceinline__ T restrict_weight(const LevelView<T>& F, int fx, int fy, int fz, int cx, int cy,
                                             int cz) {
  if (!F.pw) {
    T w = (T(3) - T(abs(fx - 3 * cx))) * T(1.0 / 3.0);
    w *= (T(3) - T(abs(fy - 3 * cy))) * T(1.0 / 3.0);
    if (D == 3) w *= (T(3) - T(abs(fz - 3 * cz))) * T(1.0 / 3.0);
    return w;
  }
  if (!is_interior<D>(fx, fy, fz, F.nv)) return T(0);
  const int nc = (F.nv - 1) / 3;
  int ex = cx - min(fx / 3, nc - 1), ey = cy - min(fy / 3, nc - 1);
  int ez = D == 3 ? cz - min(fz / 3, nc - 1) : 0;
  if (ex < 0 || ex > 1 || ey < 0 || ey > 1 || ez < 0 || ez > 1) return T(0);
  return F.pw[lin<D>(fx, fy, fz, F.nv) * (1 << D) + (ex | (ey << 1) | (ez << 2))];
}

// sum_c P(f <- c) v(c) at fine vertex f (lattice of nvf vertices per axis, transfer weights pw
// into it or nullptr: d-linear) from the coarse lattice of nvc vertices per axis, with
// v(c) = fetch(cx, cy, cz).
template <typename T, int D, typename Fetch>
__device__ __forceinline__ T prolong_gather(const T* __restrict__ pw, int nvf, int nvc, int x, int y, int z,
                                            Fetch&& fetch) {
  const int nc = nvc - 1;
  const int cx = min(x / 3, nc - 1), cy = min(y / 3, nc - 1), cz = D == 3 ? min(z / 3, nc - 1) : 0;
  const int sx = x - 3 * cx, sy = y - 3 * cy, sz = z - 3 * cz;
  T acc = T(0);
#pragma unroll
  for (int e = 0; e < (1 << D); ++e) {
    const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
    T w;
    if (!pw) {
      w = (ex ? T(sx) : T(3 - sx)) * T(1.0 / 3.0);
      w *= (ey ? T(sy) : T(3 - sy)) * T(1.0 / 3.0);
      if (D == 3) w *= (ez ? T(sz) : T(3 - sz)) * T(1.0 / 3.0);
    } else {
      w = pw[lin<D>(x, y, z, nvf) * (1 << D) + e];
    }
    if (w != T(0)) acc += w * fetch(cx + ex, cy + ey, cz + ez);
  }
  return acc;
}

// sum_c P(f <- c) (src(c) - sub(c)) at fine vertex f of level F from level C.
template <typename T, int D>
__device__ __forceinline__ T prolong_value(const LevelView<T>& F, const LevelView<T>& C, int x, int y, int z,
                                           const T* __restrict__ src, const T* __restrict__ sub) {
  return prolong_gather<T, D>(F.pw, F.nv, C.nv, x, y, z, [&](int X, int Y, int Z) {
    const size_t ci = lin<D>(X, Y, Z, C.nv);
    T v = src[ci];
    if (sub) v -= sub[ci];
    return v;
  });
}

// FAS update of vertex i of coarse level C (next finer level F, next coarser level Cm).
template <typename T, int D>
__device__ __forceinline__ void level_update_vertex(const LevelView<T>& C, const LevelView<T>& F,
                                                    const LevelView<T>& Cm, const RtSep<T>& rts, T omega,
                                                    T omega_t, T cscale, int damping, int gather, size_t i) {
  const int nv = C.nv, nvf = F.nv;
  // coarse lattices stay far below 2^32 vertices: 32-bit index arithmetic
  const unsigned iu = unsigned(i), nvu = unsigned(nv), q = iu / nvu;
  const int x = int(iu - q * nvu), y = D == 3 ? int(q % nvu) : int(q), z = D == 3 ? int(q / nvu) : 0;
  if (!is_interior<D>(x, y, z, nv)) return;
  const bool jac = damping == ADAFAC_DAMP_JAC;
  T uv, rr, bt;
  T nb[27];
  if (gather) {
    const int X = 3 * x, Y = 3 * y, Z = 3 * z;
    uv = F.u[lin<D>(X, Y, Z, nvf)];
    rr = T(0);
    bt = T(0);
    // 5^d restriction gathers, one plane at a time with all its loads in flight
#pragma unroll
    for (int oz = (D == 3 ? -2 : 0); oz <= (D == 3 ? 2 : 0); ++oz) {
      T pl[25];
#pragma unroll
      for (int t = 0; t < 25; ++t) pl[t] = F.r[lin<D>(X + t % 5 - 2, Y + t / 5 - 2, Z + oz, nvf)];
      T W = T(0);
      if (!F.pw) {
#pragma unroll
        for (int t = 0; t < 25; ++t) W += restrict_weight<T, D>(F, X + t % 5 - 2, Y + t / 5 - 2, Z + oz, x, y, z) * pl[t];
      } else {
        for (int t = 0; t < 25; ++t) W += restrict_weight<T, D>(F, X + t % 5 - 2, Y + t / 5 - 2, Z + oz, x, y, z) * pl[t];
      }
      rr += W;
      if (jac && C.rtw) {
        // R~ built from the operator: this vertex's stored weights of the plane oz
        const T* rw = C.rtw + i * (D == 2 ? 25 : 125) + (D == 3 ? 25 * (oz + 2) : 0);
        T Bs = T(0);
#pragma unroll
        for (int t = 0; t < 25; ++t) Bs += rw[t] * pl[t];
        bt += Bs;
      } else if (jac) {
        // R~ = scale sum_a delta(o_a) prod_{b != a} m(o_b)
        T Xs = T(0), Ys = T(0), Qs = T(0);
#pragma unroll
        for (int o = 0; o < 5; ++o) {
          Xs += rts.m[o] * pl[10 + o];
          Ys += rts.m[o] * pl[5 * o + 2];
          T row = T(0);
#pragma unroll
          for (int q = 0; q < 5; ++q) row += rts.m[q] * pl[5 * o + q];
          Qs += rts.m[o] * row;
        }
        if (D == 2) bt += rts.scale * (Xs + Ys);
        else bt += rts.scale * (rts.m[oz + 2] * (Xs + Ys) + (oz == 0 ? Qs : T(0)));
      }
    }
    C.u[i] = uv;
    C.rr[i] = rr;
    C.bt[i] = bt;
#pragma unroll
    for (int t = 0; t < (D == 2 ? 9 : 27); ++t)
      nb[t] = F.u[lin<D>(3 * (x + t % 3 - 1), 3 * (y + (t / 3) % 3 - 1), 3 * (z + t / 9 - (D == 3 ? 1 : 0)), nvf)];
  } else {
    uv = C.u[i];
    rr = C.rr[i];
    bt = C.bt[i];
#pragma unroll
    for (int t = 0; t < (D == 2 ? 9 : 27); ++t)
      nb[t] = C.u[lin<D>(x + t % 3 - 1, y + (t / 3) % 3 - 1, z + t / 9 - (D == 3 ? 1 : 0), nv)];
  }
  T dg;
  T au = apply_level_op_nb<T, D>(C, x, y, z, nb, dg);
  // FAS right-hand side with the tau correction, b_l = R r_{l+1} + A_l I u_{l+1}.  The FAS
  // residual b_l - A_l u_l of this level is R r_{l+1} itself: taken from rr directly rather
  // than as (rr + au) - au, which would add a rounding of |A_l u_l| (large next to R r once the
  // iteration has converged far) to every coarse residual.
  T bf = rr + au;
  T res = rr;
  T c = cscale * omega * res / dg;
  T s = c;
  if (jac) s = c - omega_t * bt / dg;
  if (damping == ADAFAC_DAMP_PI && Cm.ic && x % 3 == 0 && y % 3 == 0 && (D == 2 || z % 3 == 0))
    Cm.ic[lin<D>(x / 3, y / 3, z / 3, Cm.nv)] = c;
  C.bf[i] = bf;
  C.r[i] = res;
  C.S[i] = s;
}

// A launch of a pipelined solve's cycle after the one that met the stopping rule does nothing
// (uniform over the launch).
__device__ __forceinline__ bool gated(const Gate& g) { return g.stop && g.need >= *g.stop; }

// The stopping rule on the norms (l2h, linf) a cycle has just formed (one thread); it is applied
// once (a later cycle, were its launch not gated, would leave *stop alone).
__device__ __forceinline__ void apply_stop_rule(const StopRule& r, const double* norm) {
  if (!r.stop || !r.apply || r.need >= *r.stop) return;
  const double l2 = norm[0];
  const double r0 = r.first ? l2 : r.r0[0];
  const bool diverged = !isfinite(l2) || l2 > 1e3 * r0;
  const bool met = r0 == 0.0 || l2 / r0 <= r.tol;
  if (diverged || met) *r.stop = r.need + 1;
}

// Block-wide (up to 1024 threads) sum and max; thread 0 writes (sum, max) to partials[2*blockIdx.x].
__device__ __forceinline__ void block_norm_partials(double ssum, double smax, double* partials) {
  __shared__ double ws[16], wm[16];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    ssum += __shfl_xor(ssum, off);
    smax = fmax(smax, __shfl_xor(smax, off));
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) { ws[wave] = ssum; wm[wave] = smax; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, m = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) { s += ws[w]; m = fmax(m, wm[w]); }
    partials[2 * blockIdx.x] = s;
    partials[2 * blockIdx.x + 1] = m;
  }
}

}  // namespace adafac
