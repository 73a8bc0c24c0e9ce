// Single-pass finest-level sweep of the adAFAC cycle for gfx950.
//
// One launch touches every finest-level vertex once per cycle and does, per vertex:
//   (a) u <- u + P S_{L-1}: the coarse corrections of the previous cycle, applied one sweep
//       late (the iterate shift of Sec. 4.3; the iterates equal those of the unshifted cycle),
//   (b) r = b - A u with the Q1 operator of -div(eps grad u) (element-wise, Sec. 4.2),
//   (c) u <- u + omega D^-1 r (damped Jacobi, Algorithm 1),
//   (d) the FAS injection u_{L-1} = I u, the restriction R r (the coarse level adds the tau
//       correction, Sec. 2.4) and the auxiliary right-hand side R~ r (Sec. 3.2) for every
//       coarse vertex the tile owns,
//   (e) per-block partial sums of h^d r^2 and max |r| (Sec. 5 residual norms).
//
// Tiling.  A workgroup owns a 27 x 27 (x tz in 3D, tz a multiple of 3) block of fine vertices,
// i.e. whole coarse cells, and every coarse vertex at a multiple of 3 inside it; the 3D sweep
// runs 1024 lanes (sixteen wave64), one per x/y column of the rings below, the 2D sweep 256.  The 5^d-point restriction of an owned coarse vertex reaches two fine vertices
// into the lower neighbour, so the tile recomputes the residual on a 29-wide ring and reads
// u on a 31-wide ring: every coarse value is written by exactly one workgroup, without atomics,
// and the result does not depend on scheduling.  3D tiles march through z with the current
// u plane and the current residual plane in LDS; the 27-point stencil is split into the two
// cell layers below and above a vertex, whose partial sums are carried in registers, and the
// global loads of the next plane are issued before the current plane is processed.  Both
// restrictions are tensor products (R = P^T of d-linear P; R~ a sum of d planar products,
// see the host setup) and are evaluated by an x pass over all rows and a y pass per coarse
// column.  Workgroup ids are remapped so that consecutive tiles (which share halo planes)
// run on the same XCD and hit the same L2.  adAFAC-PI reads and writes the injected fine
// correction in the same pass and therefore runs on the one-kernel-per-step path.
#include <hip/hip_runtime.h>

#include <type_traits>

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
constexpr int MAXTZ = 81;
constexpr int NU = UW * UW;
constexpr int NR = RW * RW;
// workgroup size of the 3D sweep and the occupancy it is compiled for (waves per SIMD)
#ifndef ADAFAC_SWEEP3D_THREADS
#define ADAFAC_SWEEP3D_THREADS 1024
#endif
#ifndef ADAFAC_SWEEP3D_MINWAVES
#define ADAFAC_SWEEP3D_MINWAVES 4
#endif
#ifndef ADAFAC_SWEEP3D_TZ
#define ADAFAC_SWEEP3D_TZ 0      // 0: choose per level
#endif
constexpr int NT3 = ADAFAC_SWEEP3D_THREADS;
#ifndef ADAFAC_SWEEP3D_RP
#define ADAFAC_SWEEP3D_RP 31
#endif
constexpr int RP = ADAFAC_SWEEP3D_RP;        // LDS row pitch of the 3D residual ring (>= RW)
constexpr int RB3 = RW * RP + (NT3 - NR);    // residual ring plus one slot per idle lane
static_assert(RP >= RW, "row pitch below the ring width");
constexpr int NUSLOT = (NU + 255) / 256;
constexpr int NSLOT = (NR + 255) / 256;
constexpr int NUSLOT3 = (NU + NT3 - 1) / NT3;
constexpr int NSLOT3 = (NR + NT3 - 1) / NT3;

__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  // blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous range of tiles
  const int q = nblk / 8, rem = nblk % 8;
  const int x = bid % 8, k = bid / 8;
  return x * q + min(x, rem) + k;
}

// The tile's block of a coarse-level array (CW x CW x nsz values from (cbx, cby, cbz), zero off
// the lattice of nc + 1 vertices per axis) into LDS.  Every lane issues all its loads before the
// first is needed (addresses clamped into the lattice), so the block costs one memory round
// trip, not one per lane slot.
template <typename T, int NTH>
__device__ __forceinline__ void stage_coarse_block(T* Sb, const T* __restrict__ S, int cbx, int cby, int cbz,
                                                   int nsz, int nc, int tid) {
  constexpr int NSB = ((MAXTZ / 3 + 3) * CW * CW + NTH - 1) / NTH;
  const int nsb = nsz * CW * CW, nvc = nc + 1;
  T sv[NSB];
#pragma unroll
  for (int k = 0; k < NSB; ++k) {
    const int i = tid + k * NTH;
    const int lx = i % CW, ly = (i / CW) % CW, lz = i / (CW * CW);
    const int cx = cbx + lx, cy = cby + ly, cz = cbz + lz;
    const int cxc = min(max(cx, 0), nc), cyc = min(max(cy, 0), nc), czc = min(max(cz, 0), nc);
    const T v = S[(size_t(czc) * nvc + cyc) * nvc + cxc];
    sv[k] = (i < nsb && cx == cxc && cy == cyc && cz == czc) ? v : T(0);
  }
#pragma unroll
  for (int k = 0; k < NSB; ++k)
    if (tid + k * NTH < nsb) Sb[tid + k * NTH] = sv[k];
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

// x pass of both tensor-product restrictions over the residual ring: for every row y and
// owned coarse column, the d-linear weighted and the R~ mass-weighted sums along x.
template <typename T, int NTH = 256>
__device__ __forceinline__ void restrict_x_pass(const T* Rb, T* Xw, T* Xm, const RtSep<T>& rts, int tid) {
  for (int t = tid; t < RW * NCO; t += NTH) {
    const int y = t / NCO, ccx = t % NCO;
    const T* rp = &Rb[y * RW + 3 * ccx + 2];
    T sw = T(0), sm = T(0);
#pragma unroll
    for (int o = -2; o <= 2; ++o) {
      sw += wlin<T>(o) * rp[o];
      sm += rts.m[o + 2] * rp[o];
    }
    Xw[t] = sw;
    Xm[t] = sm;
  }
}

// The 27-point Q1 operator on one z column, one plane at a time.  push() takes the 3 x 3
// neighbourhood of the column in the newest u plane (centre at up, row pitch W) and returns
// A u at the plane below it, z, with the diagonal D there; uz receives u(z).  Carried:
// Poisson (eps = 1): u(z), D4(z) = sum of the four in-plane diagonal neighbours, F(z-1) and
// F(z) with F = 2 A4 + D4 (A4: the four in-plane axis neighbours), and then
// A u(z) = h [8/3 u(z) - (2 D4(z) + F(z-1) + F(z+1)) / 12].  Variable eps: the contribution
// of the cell layer below z, the eps sum of that layer, and per quadrant the values the layer
// above needs; the eps of the four cells of layer z around the column come from the blocks.
template <typename T, bool VAREPS>
struct ColumnOp {
  T own = T(0), c1 = T(0), c2 = T(0), c3 = T(0), epsprev = T(0);
  // variable eps: the eps-weighted sums over the four quadrants of the diagonal neighbours and
  // of the in-plane neighbour sums of the plane below (weighted with the next push's cell layer,
  // so two values are carried instead of eight); the blocks of the four cells around the column
  // (fixed per column); the eps of the current block layer (reloaded only when z enters a new
  // layer, the same step for every lane); ceil(2^32 / bs) for the layer index
  T acar = T(0), bcar = T(0);
  int off4[4] = {0, 0, 0, 0};
  int bzc = -1;
  T e4c[4] = {T(0), T(0), T(0), T(0)}, eslc = T(0);
  unsigned long long bsm = 0;

  __device__ __forceinline__ void init(int x, int y, int n, int nb, int bs) {
    if constexpr (VAREPS) {
      const int bx0 = min(max(x - 1, 0), n - 1) / bs, bx1 = min(max(x, 0), n - 1) / bs;
      const int by0 = min(max(y - 1, 0), n - 1) / bs, by1 = min(max(y, 0), n - 1) / bs;
      off4[0] = by0 * nb + bx0;
      off4[1] = by0 * nb + bx1;
      off4[2] = by1 * nb + bx0;
      off4[3] = by1 * nb + bx1;
      bsm = 0xFFFFFFFFull / unsigned(bs) + 1;   // exact floor(z / bs) = (z bsm) >> 32 for z < 2^20
    }
  }

  template <int W>
  __device__ __forceinline__ T push(const T* up, T h, int z, int n, const T* eps, int nb, T& diag, T& uz) {
    const T o_n = up[0];
    const T ax_m = up[-1], ax_p = up[1], ay_m = up[-W], ay_p = up[W];
    const T d_0 = up[-W - 1], d_1 = up[-W + 1], d_2 = up[W - 1], d_3 = up[W + 1];
    T au;
    uz = own;
    if constexpr (!VAREPS) {
      const T d4 = (d_0 + d_1) + (d_2 + d_3);
      const T f = T(2) * ((ax_m + ax_p) + (ay_m + ay_p)) + d4;
      au = h * (T(8.0 / 3.0) * uz - T(1.0 / 12.0) * ((T(2) * c1 + c2) + f));
      diag = h * T(8.0 / 3.0);
      c1 = d4;
      c2 = c3;
      c3 = f;
    } else {
      // quadrants q = (sx, sy): 0 = (-,-), 1 = (+,-), 2 = (-,+), 3 = (+,+)
      const T d_n[4] = {d_0, d_1, d_2, d_3};
      const T e_n[4] = {ax_m + ay_m + d_0, ax_p + ay_m + d_1, ax_m + ay_p + d_2, ax_p + ay_p + d_3};
      // eps of the four cells of layer z (between planes z and z+1) around the column
      auto layer = [&](int zz) { return int((unsigned long long)unsigned(min(max(zz, 0), n - 1)) * bsm >> 32); };
      auto load = [&](int bz) {
        const T* eb = eps + size_t(bz) * nb * nb;
#pragma unroll
        for (int q = 0; q < 4; ++q) e4c[q] = eb[off4[q]];
        eslc = (e4c[0] + e4c[1]) + (e4c[2] + e4c[3]);
        bzc = bz;
      };
      const int bz = layer(z);
      if (bz != bzc) load(bz);
      T se = T(0), sd = T(0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        se += e4c[q] * e_n[q];
        sd += e4c[q] * d_n[q];
      }
      const T esl = eslc;
      // layer z's contributions to A u(z) (with the plane below) and to A u(z+1) (carried)
      const T bc = esl * (T(1.0 / 3.0) * uz) - T(1.0 / 12.0) * (acar + se);
      const T tn = esl * (T(1.0 / 3.0) * o_n) - T(1.0 / 12.0) * (sd + bcar);
      au = h * (bc + c1);
      diag = h * T(1.0 / 3.0) * (esl + epsprev);
      c1 = tn;
      epsprev = esl;
      // the next push (plane z+1) weights this plane's neighbours with layer z+1
      const int bzn = layer(z + 1);
      if (bzn != bz) {
        load(bzn);
        acar = T(0);
        bcar = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acar += e4c[q] * d_n[q];
          bcar += e4c[q] * e_n[q];
        }
      } else {
        acar = sd;
        bcar = se;
      }
    }
    own = o_n;
    return au;
  }
};

}  // namespace

// Arguments of the 3D sweep (only what it reads; passed in kernarg memory).
template <typename T>
struct Sweep3dArgs {
  const T* uin;
  T* uout;
  const T* b;
  const T* S;        // S_{L-1}
  T* cu;             // u_{L-1} (injection)
  T* crr;            // R r
  T* cbt;            // R~ r
  const T* eps;      // eps blocks (VAREPS)
  double* partials;
  T h, omega, hd;
  RtSep<T> rts;
  int n, nv, nc, nvc, nb, bs;
  int tz, ntx, ntz, damping, apply_pending;
  // coarse FAS level (coarse = 1): b holds R r of the finer level; the kernel forms the FAS
  // right-hand side bf = R r + A u (tau correction), the residual r = bf - A u (= R r), and writes
  // S = cscale omega D^-1 r - omega~ D^-1 b~ instead of updating u
  int coarse;
  const T* bt_in;
  T* sout;
  T* bfout;
  T* rout;
  T omega_t, cscale;
  // adAFAC-PI: the level's correction c at the c-points, I c, written to the next coarser level
  // (nullptr for the other damping forms)
  T* ic;
  // request server: the launch does nothing once *stop <= need (the request stopped)
  const unsigned long long* stop;
  unsigned long long need;
};

// Lattice loads and stores of the 3D sweep through a buffer resource: the per-lane column
// offset stays in one VGPR and the plane offset is a scalar, so no 64-bit address arithmetic
// is spent per plane.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
template <typename T>
struct Lattice;
template <>
struct Lattice<double> {
  __amdgpu_buffer_rsrc_t r;
  __device__ Lattice(const double* p, unsigned bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), 0, int(bytes), 0x00020000)) {}
  __device__ __forceinline__ double ld(unsigned voff, unsigned soff) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
  __device__ __forceinline__ void st_stream(double v, unsigned voff, unsigned soff) const {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, voff, soff, 2 /* nt */);
  }
};
template <>
struct Lattice<float> {
  __amdgpu_buffer_rsrc_t r;
  __device__ Lattice(const float* p, unsigned bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), 0, int(bytes), 0x00020000)) {}
  __device__ __forceinline__ float ld(unsigned voff, unsigned soff) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }
  __device__ __forceinline__ void st_stream(float v, unsigned voff, unsigned soff) const {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 2 /* nt */);
  }
};

template <int V>
using IC = std::integral_constant<int, V>;

// Lanes that run the per-plane restriction and interpolation passes: disjoint wavefronts, so
// that no wavefront carries more than one of them on top of its column.
constexpr int XP0 = 0;      // x pass: RW * NCO = 261 lanes, wavefronts 0-4
constexpr int YP0 = 320;    // y pass: NCO^2 = 81 lanes, wavefronts 5-6
constexpr int BL0 = 448;    // S interpolation: CW^2 = 144 lanes, wavefronts 7-9
static_assert(RW * NCO <= YP0 && YP0 + NCO * NCO <= BL0 && BL0 + CW * CW <= NT3, "pass lanes overlap");

// The sweep marches z in steps of one fine plane; three steps make one coarse layer.  Step p
// (ring slot K = (p - zs) mod 3, a compile-time constant because zs is a multiple of 3):
//   build u plane p in LDS (plus the pending S interpolated to it),
//   residual of plane p-2 (u planes p-3..p-1), Jacobi update, norm partials,
//   x pass of plane p-3, y pass of plane p-4 (coarse plane accumulation),
//   S interpolated to plane p+1,
// then one barrier.  Every per-plane LDS buffer is indexed by its plane's slot.  Steps of the
// pipeline's fill and drain carry the range checks (CK); the steady state carries none.
template <typename T, bool VAREPS, bool COARSE, bool PEND>
__global__ void __launch_bounds__(NT3, ADAFAC_SWEEP3D_MINWAVES) k_fine_sweep3d(Sweep3dArgs<T> a) {
  static_assert(NT3 >= NU, "one lane per ring column");
  __shared__ T Ub[3][NT3];               // u planes (padded: every lane writes its slot)
  __shared__ T Rb[3][RB3];               // residual planes, row pitch RP
  __shared__ T Xw[3][RW * NCO];          // x passes
  __shared__ T Xm[3][RW * NCO];
  __shared__ T Sb[PEND ? (MAXTZ / 3 + 3) * CW * CW : 1];
  __shared__ T Sz[3][CW * CW];           // S interpolated to a fine plane

  if (a.stop && a.need >= *a.stop) return;   // uniform over the launch
  const int n = a.n, nv = a.nv, nc = a.nc, nvc = a.nvc;
  const int plane = nv * nv;
  const unsigned planeb = unsigned(plane * sizeof(T));
  const unsigned latb = unsigned(size_t(plane) * nv * sizeof(T));
  const int nblk = a.ntx * a.ntx * a.ntz;
  const int t = xcd_remap(blockIdx.x, nblk);
  // x/y tiles fastest: the tiles of one XCD share their x/y halos in its L2 at the same time
  const int txi = t % a.ntx, tyi = (t / a.ntx) % a.ntx, tzi = t / (a.ntx * a.ntx);
  const int tz = a.tz;
  const int x0 = TX * txi, y0 = TX * tyi, z0 = tz * tzi;
  const int cbx = x0 / 3 - 1, cby = y0 / 3 - 1, cbz = z0 / 3 - 1;
  const int nsz = tz / 3 + 3;
  const int tid = threadIdx.x;
  const bool jac = a.damping == ADAFAC_DAMP_JAC;
  const T h = a.h;
  const Lattice<T> U(a.uin, latb), B(a.b, latb), UO(a.uout, latb);

  if constexpr (PEND) stage_coarse_block<T, NT3>(Sb, a.S, cbx, cby, cbz, nsz, nc, tid);

  // this lane's u-ring column (loads are clamped into the lattice: values off the lattice only
  // feed residuals of non-dof vertices, which are discarded)
  const int ui = tid < NU ? tid : 0;
  const int ux = x0 - 3 + ui % UW, uy = y0 - 3 + ui / UW;
  const int uxc = min(max(ux, 0), n), uyc = min(max(uy, 0), n);
  const unsigned uoffb = unsigned((uxc + nv * uyc) * sizeof(T));
  const int ucx = uxc / 3, ucy = uyc / 3;
  const int usi = (ucy - cby) * CW + ucx - cbx;
  const int usx = uxc - 3 * ucx, usy = uyc - 3 * ucy;
  const T wx0 = T(3 - usx) * T(1.0 / 3.0), wx1 = T(usx) * T(1.0 / 3.0);
  const T wy0 = T(3 - usy) * T(1.0 / 3.0), wy1 = T(usy) * T(1.0 / 3.0);
  // this lane's residual column
  const bool ract = tid < NR;
  const int rj = ract ? tid : 0;
  const int rx = rj % RW, ry = rj / RW;
  const int x = x0 - 2 + rx, y = y0 - 2 + ry;
  const bool rint = ract && x > 0 && x < n && y > 0 && y < n;
  const bool rown = rint && rx >= 2 && ry >= 2 && x < x0 + TX && y < y0 + TX;
  const bool rinj = rown && x % 3 == 0 && y % 3 == 0;
  const int roff = min(max(x, 0), n) + nv * min(max(y, 0), n);
  const unsigned roffb = unsigned(roff * sizeof(T));
  const int upos = (ry + 1) * UW + rx + 1;
  // residual slot: row pitch RP (bank spread of the strided x-pass reads), idle lanes past it
  const int rslot = ract ? ry * RP + rx : RW * RP + (tid - NR);

  ColumnOp<T, VAREPS> col;
  col.init(x, y, n, a.nb, a.bs);
  // prefetch ring: slot K holds u(p) and b(p-2) for the steps p of slot K
  T pu[3], pb[3];
  T accR[2] = {T(0), T(0)}, accT[2] = {T(0), T(0)};
  double ssum = 0.0, smax = 0.0;
  const T wdiag = a.omega / (h * T(8.0 / 3.0));     // omega / D for eps = 1

  const int zs = z0 - 3, ze = z0 + tz;
  auto uload = [&](int p) { return U.ld(uoffb, unsigned(min(max(p, 0), n)) * planeb); };
  auto bload = [&](int p) { return B.ld(roffb, unsigned(min(max(p, 0), n)) * planeb); };
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    pu[q] = uload(zs + q);
    pb[q] = bload(zs + q - 1);
  }

  // S interpolated along z to fine plane p, into slot KS (zero off the lattice)
  auto blend_s = [&](int p, auto ks) {
    constexpr int KS = decltype(ks)::value;
    if constexpr (PEND) {
      const int bt = tid - BL0;
      if (bt >= 0 && bt < CW * CW) {
        T v = T(0);
        if (p >= 0 && p <= n) {
          const int cz = p / 3, sz = p - 3 * cz;
          const T* s0 = &Sb[(cz - cbz) * CW * CW + bt];
          v = T(3 - sz) * T(1.0 / 3.0) * s0[0] + T(sz) * T(1.0 / 3.0) * s0[CW * CW];
        }
        Sz[KS][bt] = v;
      }
    }
  };
  if constexpr (PEND) __syncthreads();  // Sb ready
  blend_s(zs, IC<0>{});
  __syncthreads();                       // Sz[0] ready

  auto step = [&](int p, auto ck, auto kk) {
    constexpr bool CK = decltype(ck)::value != 0;
    constexpr int K = decltype(kk)::value;
    constexpr int K1 = (K + 1) % 3, K2 = (K + 2) % 3;
    // (1) u plane p into slot K, plus the pending correction
    if (!CK || p <= ze) {
      T v = pu[K];
      if constexpr (PEND) {
        const T* s0 = &Sz[K][usi];
        v += wy0 * (wx0 * s0[0] + wx1 * s0[1]) + wy1 * (wx0 * s0[CW] + wx1 * s0[CW + 1]);
      }
      Ub[K][tid] = v;
    }
    pu[K] = CK ? uload(min(p + 3, ze)) : U.ld(uoffb, unsigned(p + 3) * planeb);
    // (2) residual of plane z = p-2 from u planes p-3 (registers), p-2 (registers) and p-1 (slot K2)
    if (!CK || (p - 1 >= zs && p - 1 <= ze)) {
      const int z = p - 2;
      T diag, uz;
      const T au = col.template push<UW>(&Ub[K2][upos], h, z, n, a.eps, a.nb, diag, uz);
      const T dinv = VAREPS ? a.omega / diag : wdiag;
      T res = T(0);
      const bool zin = !CK || (p - 1 >= zs + 2 && z > 0 && z < n);
      if (zin && rint) {
        const bool own_pt = rown && (!CK || (z >= z0 && z < z0 + tz));
        if constexpr (!COARSE) {
          res = pb[K2] - au;
          if (own_pt) {
            UO.st_stream(uz + dinv * res, roffb, unsigned(z) * planeb);
            const double rd = double(res);
            ssum += rd * rd;
            smax = fabs(rd) > smax ? fabs(rd) : smax;
          }
        } else {
          // FAS right-hand side with the tau correction; the FAS residual bf - A u is R r
          // itself (taken directly: no rounding of |A u| enters it)
          const T bf = pb[K2] + au;
          res = pb[K2];
          if (own_pt) {
            const int gi = z * plane + roff;
            T sv = a.cscale * dinv * res;
            if (jac) sv -= (a.omega_t / a.omega) * dinv * a.bt_in[gi];
            a.sout[gi] = sv;
            a.bfout[gi] = bf;
            a.rout[gi] = res;
          }
        }
        // FAS injection u_{L-1} = I u: planes z = p-2 with z = 0 mod 3 are the steps K = 2
        if (K == 2 && own_pt && rinj) {
          const int ci = lin<3>(x / 3, y / 3, z / 3, nvc);
          a.cu[ci] = uz;
          if (a.ic) a.ic[ci] = (COARSE ? a.cscale : T(1)) * dinv * res;
        }
      }
      Rb[K1][rslot] = res;
    }
    pb[K2] = CK ? bload(min(p + 1, ze)) : B.ld(roffb, unsigned(p + 1) * planeb);
    // (3) x pass of residual plane p-3 (slot K)
    if (!CK || (p - 3 >= zs + 1 && p - 3 <= ze - 1)) {
      const int xt = tid - XP0;
      if (xt >= 0 && xt < RW * NCO) {
        // consecutive lanes take consecutive rows of one coarse column (conflict-free reads)
        const int yy = xt % RW, ccx = xt / RW;
        const T* rp = &Rb[K][yy * RP + 3 * ccx + 2];
        T sw = T(0), sm = T(0);
#pragma unroll
        for (int o = -2; o <= 2; ++o) {
          sw += wlin<T>(o) * rp[o];
          sm += a.rts.m[o + 2] * rp[o];
        }
        Xw[K][yy * NCO + ccx] = sw;
        Xm[K][yy * NCO + ccx] = sm;
      }
    }
    // (4) y pass of residual plane zr = p-4 (slot K2), accumulated into the coarse planes at
    // or below and above it; m = zr - 3 floor(zr / 3) = K2 because zs = 0 mod 3
    if (!CK || (p - 4 >= zs + 1 && p - 4 <= ze - 1)) {
      const int yt = tid - YP0;
      if (yt >= 0 && yt < NCO * NCO) {
        constexpr int m = K2;
        const int zr = p - 4;
        const T* xw = Xw[K2];
        const T* xm = Xm[K2];
        const T* rz = Rb[K2];
        const int ccx = yt % NCO, ccy = yt / NCO;
        T W = T(0), Q = T(0), Y = T(0);
#pragma unroll
        for (int o = -2; o <= 2; ++o) {
          const int row = 3 * ccy + 2 + o;
          W += wlin<T>(o) * xw[row * NCO + ccx];
          Q += a.rts.m[o + 2] * xm[row * NCO + ccx];
          Y += a.rts.m[o + 2] * rz[row * RP + 3 * ccx + 2];
        }
        const T X = xm[(3 * ccy + 2) * NCO + ccx];
        // R~: planar tensor products; the plane through the coarse vertex also carries Q
        accR[0] += wlin<T>(m) * W;
        if (jac) accT[0] += a.rts.scale * (a.rts.m[2 + m] * (X + Y) + (m == 0 ? Q : T(0)));
        if constexpr (m != 0) {
          accR[1] += wlin<T>(3 - m) * W;
          if (jac) accT[1] += a.rts.scale * a.rts.m[2 + 3 - m] * (X + Y);
        }
        if constexpr (m == 2) {
          const int cz = (zr - 2) / 3;        // coarse plane below zr (zr >= z0 - 1 >= -1)
          const int cx = x0 / 3 + ccx, cy = y0 / 3 + ccy;
          if (cz >= z0 / 3 && cz < (z0 + tz) / 3 && cx > 0 && cx < nc && cy > 0 && cy < nc &&
              cz > 0 && cz < nc) {
            const size_t ci = lin<3>(cx, cy, cz, nvc);
            a.crr[ci] = accR[0];
            a.cbt[ci] = accT[0];
          }
          accR[0] = accR[1];
          accT[0] = accT[1];
          accR[1] = accT[1] = T(0);
        }
      }
    }
    // (5) S interpolated to plane p+1 (slot K1)
    if (!CK || p + 1 <= ze) blend_s(p + 1, IC<K1>{});
    __syncthreads();
  };

  // steps zs .. ze+3 drain the pipeline (residuals end at plane ze-1, restriction two steps later)
  const int nit = (tz + 7 + 2) / 3;
  const int ihi = (tz - 2) / 3;          // iterations 2..ihi need no range checks
  int it = 0;
  for (; it < min(2, nit); ++it) {
    const int p = zs + 3 * it;
    step(p, IC<1>{}, IC<0>{});
    step(p + 1, IC<1>{}, IC<1>{});
    step(p + 2, IC<1>{}, IC<2>{});
  }
  for (; it <= ihi; ++it) {
    const int p = zs + 3 * it;
    step(p, IC<0>{}, IC<0>{});
    step(p + 1, IC<0>{}, IC<1>{});
    step(p + 2, IC<0>{}, IC<2>{});
  }
  for (; it < nit; ++it) {
    const int p = zs + 3 * it;
    step(p, IC<1>{}, IC<0>{});
    step(p + 1, IC<1>{}, IC<1>{});
    step(p + 2, IC<1>{}, IC<2>{});
  }
  if constexpr (!COARSE) block_norm_partials(double(a.hd) * ssum, smax, a.partials);
}

// ---------------------------------------------------------------------------
// The constant-coefficient (eps = 1) 3D sweep on a 32-wide ring.  Lane (lx, ly) =
// (tid mod 32, tid / 32) owns the ring column (x0-3+lx, y0-3+ly): it loads u and b there and,
// where the column lies on the 29 x 29 residual ring (lx, ly in 1..29), evaluates the residual
// too.  A ring row is half a wavefront, so the x neighbours of a column sit in the adjacent
// lanes: each lane forms the x-neighbour sum of its newest u value with two whole-wavefront
// lane shifts (DPP, no LDS traffic), and the stencil reads from LDS only the u values and x sums
// of the rows above and below (four values instead of the nine of the 3 x 3 neighbourhood).  The
// arithmetic is that of k_fine_sweep3d for eps = 1, term for term and in the same order.
// ---------------------------------------------------------------------------
namespace {
constexpr int W2 = 32;                      // ring pitch in lanes
constexpr int RQ = 33;                      // LDS row pitch of the residual planes (bank spread)
static_assert(W2 * W2 == NT3, "one lane per ring column");

typedef int i32x2_t __attribute__((ext_vector_type(2)));
// v of lane i-1 (CTRL = wave_shr:1) or lane i+1 (CTRL = wave_shl:1) of the wavefront; the lane
// without a source gets 0.  Must run with every lane of the wavefront active.
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
  const i32x2_t p = __builtin_bit_cast(i32x2_t, v);
  i32x2_t r;
  r.x = __builtin_amdgcn_update_dpp(0, p.x, CTRL, 0xf, 0xf, false);
  r.y = __builtin_amdgcn_update_dpp(0, p.y, CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, r);
}
template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveShl1 = 0x130;
}  // namespace

template <typename T, bool COARSE, bool PEND>
__global__ void __launch_bounds__(NT3, ADAFAC_SWEEP3D_MINWAVES) k_sweep3d_w32(Sweep3dArgs<T> a) {
  // newest u planes with their x-neighbour sums as (u, sum) pairs (one 16-byte access each in
  // FP64), one padding row above and below so that every lane reads its y neighbours in bounds
  // (the padding only feeds lanes without residual duty)
  typedef T T2 __attribute__((ext_vector_type(2)));
  __shared__ T2 UX[3][NT3 + 2 * W2];
  __shared__ T Rb[3][W2 * RQ];           // residual planes
  __shared__ T Xw[3][RW * NCO];          // x passes
  __shared__ T Xm[3][RW * NCO];
  __shared__ T Sb[PEND ? (MAXTZ / 3 + 3) * CW * CW : 1];
  __shared__ T Sz[3][CW * CW];           // S interpolated to a fine plane

  if (a.stop && a.need >= *a.stop) return;   // uniform over the launch
  const int n = a.n, nv = a.nv, nc = a.nc, nvc = a.nvc;
  const int plane = nv * nv;
  const unsigned planeb = unsigned(plane * sizeof(T));
  const unsigned latb = unsigned(size_t(plane) * nv * sizeof(T));
  const int nblk = a.ntx * a.ntx * a.ntz;
  const int t = xcd_remap(blockIdx.x, nblk);
  const int txi = t % a.ntx, tyi = (t / a.ntx) % a.ntx, tzi = t / (a.ntx * a.ntx);
  const int tz = a.tz;
  const int x0 = TX * txi, y0 = TX * tyi, z0 = tz * tzi;
  const int cbx = x0 / 3 - 1, cby = y0 / 3 - 1, cbz = z0 / 3 - 1;
  const int nsz = tz / 3 + 3;
  const int tid = threadIdx.x;
  const bool jac = a.damping == ADAFAC_DAMP_JAC;
  const T h = a.h;
  const Lattice<T> U(a.uin, latb), B(a.b, latb), UO(a.uout, latb);

  if constexpr (PEND) stage_coarse_block<T, NT3>(Sb, a.S, cbx, cby, cbz, nsz, nc, tid);

  // this lane's ring column (loads clamped into the lattice: values off the lattice only feed
  // residuals of non-dof vertices, which are discarded)
  const int lx = tid % W2, ly = tid / W2;
  const int x = x0 - 3 + lx, y = y0 - 3 + ly;
  const int xc = min(max(x, 0), n), yc = min(max(y, 0), n);
  const int roff = xc + nv * yc;
  const unsigned offb = unsigned(roff * sizeof(T));
  const int ucx = xc / 3, ucy = yc / 3;
  const int usi = (ucy - cby) * CW + ucx - cbx;
  const int usx = xc - 3 * ucx, usy = yc - 3 * ucy;
  const T wx0 = T(3 - usx) * T(1.0 / 3.0), wx1 = T(usx) * T(1.0 / 3.0);
  const T wy0 = T(3 - usy) * T(1.0 / 3.0), wy1 = T(usy) * T(1.0 / 3.0);
  // residual duty: the ring x0-2 .. x0+26 (lx, ly in 1..29)
  const bool ract = lx >= 1 && lx <= RW && ly >= 1 && ly <= RW;
  const bool rint = ract && x > 0 && x < n && y > 0 && y < n;
  const bool rown = rint && lx >= 3 && ly >= 3 && x < x0 + TX && y < y0 + TX;
  const bool rinj = rown && x % 3 == 0 && y % 3 == 0;
  const int rslot = ly * RQ + lx;

  // the column operator of k_fine_sweep3d (eps = 1): u(z), D4(z), F(z-1), F(z)
  T own = T(0), c1 = T(0), c2 = T(0), c3 = T(0);
  T vlast = T(0), xlast = T(0);          // this lane's newest u value and its x-neighbour sum
  // prefetch ring: slot K holds u(p) and b(p-2) for the steps p of slot K
  T pu[3], pb[3];
  T accR[2] = {T(0), T(0)}, accT[2] = {T(0), T(0)};
  double ssum = 0.0, smax = 0.0;
  const T wdiag = a.omega / (h * T(8.0 / 3.0));     // omega / D for eps = 1

  const int zs = z0 - 3, ze = z0 + tz;
  auto uload = [&](int p) { return U.ld(offb, unsigned(min(max(p, 0), n)) * planeb); };
  auto bload = [&](int p) { return B.ld(offb, unsigned(min(max(p, 0), n)) * planeb); };
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    pu[q] = uload(zs + q);
    pb[q] = bload(zs + q - 1);
  }

  auto blend_s = [&](int p, auto ks) {
    constexpr int KS = decltype(ks)::value;
    if constexpr (PEND) {
      const int bt = tid - BL0;
      if (bt >= 0 && bt < CW * CW) {
        T v = T(0);
        if (p >= 0 && p <= n) {
          const int cz = p / 3, sz = p - 3 * cz;
          const T* s0 = &Sb[(cz - cbz) * CW * CW + bt];
          v = T(3 - sz) * T(1.0 / 3.0) * s0[0] + T(sz) * T(1.0 / 3.0) * s0[CW * CW];
        }
        Sz[KS][bt] = v;
      }
    }
  };
  if constexpr (PEND) __syncthreads();  // Sb ready
  blend_s(zs, IC<0>{});
  __syncthreads();                       // Sz[0] ready

  auto step = [&](int p, auto ck, auto kk) {
    constexpr bool CK = decltype(ck)::value != 0;
    constexpr int K = decltype(kk)::value;
    constexpr int K1 = (K + 1) % 3, K2 = (K + 2) % 3;
    // (1) u plane p (plus the pending correction) and its x-neighbour sums into slot K; the
    // condition is uniform over the workgroup, so every lane takes part in the lane shifts
    T vnew = T(0), xnew = T(0);
    if (!CK || p <= ze) {
      vnew = pu[K];
      if constexpr (PEND) {
        const T* s0 = &Sz[K][usi];
        vnew += wy0 * (wx0 * s0[0] + wx1 * s0[1]) + wy1 * (wx0 * s0[CW] + wx1 * s0[CW + 1]);
      }
      xnew = lane_shift<kDppWaveShr1>(vnew) + lane_shift<kDppWaveShl1>(vnew);
      UX[K][W2 + tid] = T2{vnew, xnew};
    }
    pu[K] = CK ? uload(min(p + 3, ze)) : U.ld(offb, unsigned(p + 3) * planeb);
    // (2) residual of plane z = p-2 from u planes p-3, p-2 (registers) and p-1 (slot K2 and the
    // lane's own newest values)
    if (!CK || (p - 1 >= zs && p - 1 <= ze)) {
      const int z = p - 2;
      const T2 ym = UX[K2][tid], yp = UX[K2][tid + 2 * W2];
      const T ay = ym.x + yp.x;
      const T d4 = ym.y + yp.y;
      const T f = T(2) * (xlast + ay) + d4;
      const T uz = own;
      const T au = h * (T(8.0 / 3.0) * uz - T(1.0 / 12.0) * ((T(2) * c1 + c2) + f));
      c1 = d4;
      c2 = c3;
      c3 = f;
      own = vlast;
      T res = T(0);
      const bool zin = !CK || (p - 1 >= zs + 2 && z > 0 && z < n);
      if (zin && rint) {
        const bool own_pt = rown && (!CK || (z >= z0 && z < z0 + tz));
        if constexpr (!COARSE) {
          res = pb[K2] - au;
          if (own_pt) {
            UO.st_stream(uz + wdiag * res, offb, unsigned(z) * planeb);
            const double rd = double(res);
            ssum += rd * rd;
            smax = fabs(rd) > smax ? fabs(rd) : smax;
          }
        } else {
          // FAS right-hand side with the tau correction; the FAS residual bf - A u is R r
          // itself (taken directly: no rounding of |A u| enters it)
          const T bf = pb[K2] + au;
          res = pb[K2];
          if (own_pt) {
            const int gi = z * plane + roff;
            T sv = a.cscale * wdiag * res;
            if (jac) sv -= (a.omega_t / a.omega) * wdiag * a.bt_in[gi];
            a.sout[gi] = sv;
            a.bfout[gi] = bf;
            a.rout[gi] = res;
          }
        }
        // FAS injection u_{L-1} = I u: planes z = p-2 with z = 0 mod 3 are the steps K = 2
        if (K == 2 && own_pt && rinj) {
          const int ci = lin<3>(x / 3, y / 3, z / 3, nvc);
          a.cu[ci] = uz;
          if (a.ic) a.ic[ci] = (COARSE ? a.cscale : T(1)) * wdiag * res;
        }
      }
      Rb[K1][rslot] = res;
    }
    if (!CK || p <= ze) {
      vlast = vnew;
      xlast = xnew;
    }
    pb[K2] = CK ? bload(min(p + 1, ze)) : B.ld(offb, unsigned(p + 1) * planeb);
    // (3) x pass of residual plane p-3 (slot K)
    if (!CK || (p - 3 >= zs + 1 && p - 3 <= ze - 1)) {
      const int xt = tid - XP0;
      if (xt >= 0 && xt < RW * NCO) {
        // consecutive lanes take consecutive rows of one coarse column (conflict-free reads)
        const int yy = xt % RW, ccx = xt / RW;
        const T* rp = &Rb[K][(yy + 1) * RQ + 3 * ccx + 3];
        T sw = T(0), sm = T(0);
#pragma unroll
        for (int o = -2; o <= 2; ++o) {
          sw += wlin<T>(o) * rp[o];
          sm += a.rts.m[o + 2] * rp[o];
        }
        Xw[K][yy * NCO + ccx] = sw;
        Xm[K][yy * NCO + ccx] = sm;
      }
    }
    // (4) y pass of residual plane zr = p-4 (slot K2), accumulated into the coarse planes at
    // or below and above it; m = zr - 3 floor(zr / 3) = K2 because zs = 0 mod 3
    if (!CK || (p - 4 >= zs + 1 && p - 4 <= ze - 1)) {
      const int yt = tid - YP0;
      if (yt >= 0 && yt < NCO * NCO) {
        constexpr int m = K2;
        const int zr = p - 4;
        const T* xw = Xw[K2];
        const T* xm = Xm[K2];
        const T* rz = Rb[K2];
        const int ccx = yt % NCO, ccy = yt / NCO;
        T W = T(0), Q = T(0), Y = T(0);
#pragma unroll
        for (int o = -2; o <= 2; ++o) {
          const int row = 3 * ccy + 2 + o;
          W += wlin<T>(o) * xw[row * NCO + ccx];
          Q += a.rts.m[o + 2] * xm[row * NCO + ccx];
          Y += a.rts.m[o + 2] * rz[(row + 1) * RQ + 3 * ccx + 3];
        }
        const T X = xm[(3 * ccy + 2) * NCO + ccx];
        // R~: planar tensor products; the plane through the coarse vertex also carries Q
        accR[0] += wlin<T>(m) * W;
        if (jac) accT[0] += a.rts.scale * (a.rts.m[2 + m] * (X + Y) + (m == 0 ? Q : T(0)));
        if constexpr (m != 0) {
          accR[1] += wlin<T>(3 - m) * W;
          if (jac) accT[1] += a.rts.scale * a.rts.m[2 + 3 - m] * (X + Y);
        }
        if constexpr (m == 2) {
          const int cz = (zr - 2) / 3;        // coarse plane below zr (zr >= z0 - 1 >= -1)
          const int cx = x0 / 3 + ccx, cy = y0 / 3 + ccy;
          if (cz >= z0 / 3 && cz < (z0 + tz) / 3 && cx > 0 && cx < nc && cy > 0 && cy < nc &&
              cz > 0 && cz < nc) {
            const size_t ci = lin<3>(cx, cy, cz, nvc);
            a.crr[ci] = accR[0];
            a.cbt[ci] = accT[0];
          }
          accR[0] = accR[1];
          accT[0] = accT[1];
          accR[1] = accT[1] = T(0);
        }
      }
    }
    // (5) S interpolated to plane p+1 (slot K1)
    if (!CK || p + 1 <= ze) blend_s(p + 1, IC<K1>{});
    __syncthreads();
  };

  // steps zs .. ze+3 drain the pipeline (residuals end at plane ze-1, restriction two steps later)
  const int nit = (tz + 7 + 2) / 3;
  const int ihi = (tz - 2) / 3;          // iterations 2..ihi need no range checks
  int it = 0;
  for (; it < min(2, nit); ++it) {
    const int p = zs + 3 * it;
    step(p, IC<1>{}, IC<0>{});
    step(p + 1, IC<1>{}, IC<1>{});
    step(p + 2, IC<1>{}, IC<2>{});
  }
  for (; it <= ihi; ++it) {
    const int p = zs + 3 * it;
    step(p, IC<0>{}, IC<0>{});
    step(p + 1, IC<0>{}, IC<1>{});
    step(p + 2, IC<0>{}, IC<2>{});
  }
  for (; it < nit; ++it) {
    const int p = zs + 3 * it;
    step(p, IC<1>{}, IC<0>{});
    step(p + 1, IC<1>{}, IC<1>{});
    step(p + 2, IC<1>{}, IC<2>{});
  }
  if constexpr (!COARSE) block_norm_partials(double(a.hd) * ssum, smax, a.partials);
}

// ---------------------------------------------------------------------------
// FP64 step of defect correction on a 3D level (FP32 cycles inside FP64 defect correction):
//   u' = u + (e + P S_{L-1})     the FP32 inner correction with its pending prolongation
//                                (MODE 2), the correction alone (MODE 1) or nothing (MODE 0)
//   r  = b - A u'                in FP64, stored in FP32 as the next inner right-hand side,
//                                with the FP64 norm partials
// in one z march over 27 x 27 column tiles (u' on a 29 x 29 ring in LDS), u' into the other
// FP64 buffer.  Per dof: u, b read and u' written in FP64, e read and r written in FP32.
// ---------------------------------------------------------------------------
struct Defect3dArgs {
  const double* uin;
  double* uout;
  const float* e;
  const float* S;
  const double* b;
  float* r32;
  const double* eps;
  double* partials;
  double h, hd;
  int n, nv, nc, nvc, nb, bs, tz, ntx, ntz;
  // request server: the launch does nothing once *stop <= need (the request stopped)
  const unsigned long long* stop;
  unsigned long long need;
};

namespace {
constexpr int DW = TX + 2;          // u' ring: x0-1 .. x0+27
constexpr int ND = DW * DW;
constexpr int NTD = 1024;
}  // namespace

// One 1024-lane workgroup per CU: at 64 VGPRs (two per CU) the Poisson variant spills.
#ifndef ADAFAC_DEFECT3D_MINWAVES
#define ADAFAC_DEFECT3D_MINWAVES 4
#endif
template <bool VAREPS, int MODE>
__global__ void __launch_bounds__(NTD, VAREPS ? 4 : ADAFAC_DEFECT3D_MINWAVES) k_defect3d(Defect3dArgs a) {
  static_assert(NTD >= ND && NTD >= TX * TX, "one lane per ring column");
  __shared__ double Ub[3][NTD];
  __shared__ float Sb[MODE == 2 ? (MAXTZ / 3 + 3) * CW * CW : 1];
  __shared__ float Sz[3][CW * CW];

  if (a.stop && a.need >= *a.stop) return;   // uniform over the launch
  const int n = a.n, nv = a.nv, nc = a.nc, nvc = a.nvc;
  const int plane = nv * nv;
  const unsigned latb = unsigned(size_t(plane) * nv * sizeof(double));
  const unsigned latf = unsigned(size_t(plane) * nv * sizeof(float));
  const unsigned planeb = unsigned(plane * sizeof(double)), planef = unsigned(plane * sizeof(float));
  const int nblk = a.ntx * a.ntx * a.ntz;
  const int t = xcd_remap(blockIdx.x, nblk);
  const int txi = t % a.ntx, tyi = (t / a.ntx) % a.ntx, tzi = t / (a.ntx * a.ntx);
  const int tz = a.tz;
  const int x0 = TX * txi, y0 = TX * tyi, z0 = tz * tzi;
  const int cbx = x0 / 3 - 1, cby = y0 / 3 - 1, cbz = z0 / 3 - 1;
  const int nsz = tz / 3 + 3;
  const int tid = threadIdx.x;
  const double h = a.h;
  const Lattice<double> U(a.uin, latb), UO(a.uout, latb), B(a.b, latb);
  const Lattice<float> E(a.e, latf), R(a.r32, latf);

  if constexpr (MODE == 2) stage_coarse_block<float, NTD>(Sb, a.S, cbx, cby, cbz, nsz, nc, tid);
  // u' ring column of this lane (clamped into the lattice)
  const int ui = tid < ND ? tid : 0;
  const int ux = x0 - 1 + ui % DW, uy = y0 - 1 + ui / DW;
  const int uxc = min(max(ux, 0), n), uyc = min(max(uy, 0), n);
  const unsigned uoffd = unsigned(uxc + nv * uyc);
  const bool uown = tid < ND && ux == uxc && uy == uyc && ux > 0 && ux < n && uy > 0 && uy < n &&
                    ux >= x0 && ux < x0 + TX && uy >= y0 && uy < y0 + TX;
  const int ucx = uxc / 3, ucy = uyc / 3;
  const int usi = (ucy - cby) * CW + ucx - cbx;
  const int usx = uxc - 3 * ucx, usy = uyc - 3 * ucy;
  const float wx0 = float(3 - usx) * (1.f / 3.f), wx1 = float(usx) * (1.f / 3.f);
  const float wy0 = float(3 - usy) * (1.f / 3.f), wy1 = float(usy) * (1.f / 3.f);
  // residual column of this lane: the owned 27 x 27
  const bool ract = tid < TX * TX;
  const int rj = ract ? tid : 0;
  const int x = x0 + rj % TX, y = y0 + rj / TX;
  const bool rint = ract && x < n && y < n && x > 0 && y > 0;
  const int xc = min(x, n), yc = min(y, n);
  const unsigned roffd = unsigned(xc + nv * yc);
  const int upos = (rj / TX + 1) * DW + rj % TX + 1;

  ColumnOp<double, VAREPS> col;
  col.init(x, y, n, a.nb, a.bs);
  double pu[3], pb[3];
  float pe[3];
  double ssum = 0.0, smax = 0.0;
  const int zs = z0 - 1, ze = min(z0 + tz, n);
  auto pl = [&](int p) { return unsigned(min(max(p, 0), n)); };
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    pu[q] = U.ld(uoffd * 8u, pl(zs + q) * planeb);
    pe[q] = MODE ? E.ld(uoffd * 4u, pl(zs + q) * planef) : 0.f;
    pb[q] = B.ld(roffd * 8u, pl(zs + q - 1) * planeb);
  }
  auto blend_s = [&](int p, auto ks) {
    constexpr int KS = decltype(ks)::value;
    if constexpr (MODE == 2) {
      const int bt = tid - BL0;
      if (bt >= 0 && bt < CW * CW) {
        float v = 0.f;
        if (p >= 0 && p <= n) {
          const int cz = p / 3, sz = p - 3 * cz;
          const float* s0 = &Sb[(cz - cbz) * CW * CW + bt];
          v = float(3 - sz) * (1.f / 3.f) * s0[0] + float(sz) * (1.f / 3.f) * s0[CW * CW];
        }
        Sz[KS][bt] = v;
      }
    }
  };
  if constexpr (MODE == 2) __syncthreads();
  blend_s(zs, IC<0>{});
  __syncthreads();

  auto step = [&](int p, auto ck, auto kk) {
    constexpr bool CK = decltype(ck)::value != 0;
    constexpr int K = decltype(kk)::value;
    constexpr int K1 = (K + 1) % 3, K2 = (K + 2) % 3;
    // (1) u' plane p into slot K; owned interior values are the new FP64 solution
    if (!CK || p <= ze) {
      double v = pu[K];
      if constexpr (MODE >= 1) {
        float c = pe[K];
        if constexpr (MODE == 2) {
          const float* s0 = &Sz[K][usi];
          c += wy0 * (wx0 * s0[0] + wx1 * s0[1]) + wy1 * (wx0 * s0[CW] + wx1 * s0[CW + 1]);
        }
        v += double(c);
      }
      Ub[K][tid] = v;
      if (uown && (!CK || (p >= z0 && p < z0 + tz && p > 0 && p < n))) UO.st_stream(v, uoffd * 8u, unsigned(p) * planeb);
    }
    const unsigned nxt = (CK ? pl(min(p + 3, ze)) : unsigned(p + 3));
    pu[K] = U.ld(uoffd * 8u, nxt * planeb);
    if constexpr (MODE >= 1) pe[K] = E.ld(uoffd * 4u, nxt * planef);
    // (2) residual of plane z = p-2 from u' planes p-3, p-2 (registers) and p-1 (slot K2)
    if (!CK || (p - 1 >= zs && p - 1 <= ze)) {
      const int z = p - 2;
      double diag, uz;
      const double au = col.template push<DW>(&Ub[K2][upos], h, z, n, a.eps, a.nb, diag, uz);
      if (rint && (!CK || (z >= z0 && z < z0 + tz && z > 0 && z < n))) {
        const double res = pb[K2] - au;
        R.st_stream(float(res), roffd * 4u, unsigned(z) * planef);
        ssum += res * res;
        smax = fabs(res) > smax ? fabs(res) : smax;
      }
    }
    pb[K2] = B.ld(roffd * 8u, (CK ? pl(min(p + 1, ze)) : unsigned(p + 1)) * planeb);
    if (!CK || p + 1 <= ze) blend_s(p + 1, IC<K1>{});
    __syncthreads();
  };

  // steps zs .. ze+1: u' planes z0-1 .. z0+tz, residual planes z0 .. z0+tz-1
  const int nit = (tz + 3 + 2) / 3;
  const int ihi = (tz - 4) / 3;          // iterations 2..ihi need no range checks
  int it = 0;
  for (; it < min(2, nit); ++it) {
    const int p = zs + 3 * it;
    step(p, IC<1>{}, IC<0>{});
    step(p + 1, IC<1>{}, IC<1>{});
    step(p + 2, IC<1>{}, IC<2>{});
  }
  for (; it <= ihi; ++it) {
    const int p = zs + 3 * it;
    step(p, IC<0>{}, IC<0>{});
    step(p + 1, IC<0>{}, IC<1>{});
    step(p + 2, IC<0>{}, IC<2>{});
  }
  for (; it < nit; ++it) {
    const int p = zs + 3 * it;
    step(p, IC<1>{}, IC<0>{});
    step(p + 1, IC<1>{}, IC<1>{});
    step(p + 2, IC<1>{}, IC<2>{});
  }
  block_norm_partials(a.hd * ssum, smax, a.partials);
}

template <typename T, bool VAREPS>
__global__ void __launch_bounds__(256) k_fine_sweep2d(LevelView<T> F, LevelView<T> C,
                                                      const T* __restrict__ uin, T* __restrict__ uout,
                                                      const T* __restrict__ b, RtSep<T> rts, T omega,
                                                      int damping, int apply_pending, int ntx,
                                                      double* __restrict__ partials,
                                                      const unsigned long long* stop, unsigned long long need) {
  if (stop && need >= *stop) return;   // uniform over the launch (request server)
  __shared__ T Ub[NU];
  __shared__ T Rb[NR];
  __shared__ T Xw[RW * NCO];
  __shared__ T Xm[RW * NCO];
  __shared__ T Sb[CW * CW];
  const int nv = F.nv, n = F.n, nvc = C.nv, nc = C.n;
  const int t = xcd_remap(blockIdx.x, ntx * ntx);
  const int txi = t % ntx, tyi = t / ntx;
  const int x0 = TX * txi, y0 = TX * tyi;
  const int cbx = x0 / 3 - 1, cby = y0 / 3 - 1;
  const int tid = threadIdx.x;
  const bool jac = damping == ADAFAC_DAMP_JAC;
  // global loads first; the coarse block and the ring values are combined after one barrier
  T pu[NUSLOT];
#pragma unroll
  for (int k = 0; k < NUSLOT; ++k) {
    const int i = tid + 256 * k;
    const int x = x0 - 3 + i % UW, y = y0 - 3 + i / UW;
    pu[k] = (i < NU && x >= 0 && x <= n && y >= 0 && y <= n) ? uin[lin<2>(x, y, 0, nv)] : T(0);
  }
  if (apply_pending) {
    for (int i = tid; i < CW * CW; i += 256) {
      const int cx = cbx + i % CW, cy = cby + i / CW;
      T v = T(0);
      if (cx >= 0 && cx <= nc && cy >= 0 && cy <= nc) {
        v = C.S[lin<2>(cx, cy, 0, nvc)];
      }
      Sb[i] = v;
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NUSLOT; ++k) {
    const int i = tid + 256 * k;
    if (i >= NU) continue;
    const int x = x0 - 3 + i % UW, y = y0 - 3 + i / UW;
    T v = pu[k];
    if (apply_pending && x >= 0 && x <= n && y >= 0 && y <= n) {
      const int cx = x / 3, cy = y / 3, sx = x - 3 * cx, sy = y - 3 * cy;
      const T* s0 = &Sb[(cy - cby) * CW + cx - cbx];
      const T wx0 = T(3 - sx) * T(1.0 / 3.0), wx1 = T(sx) * T(1.0 / 3.0);
      const T wy0 = T(3 - sy) * T(1.0 / 3.0), wy1 = T(sy) * T(1.0 / 3.0);
      v += wy0 * (wx0 * s0[0] + wx1 * s0[1]) + wy1 * (wx0 * s0[CW] + wx1 * s0[CW + 1]);
    }
    Ub[i] = v;
  }
  __syncthreads();
  double ssum = 0.0, smax = 0.0;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int j = tid + 256 * s;
    if (j >= NR) continue;
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
          C.u[lin<2>(x / 3, y / 3, 0, nvc)] = u0;
          if (damping == ADAFAC_DAMP_PI) C.ic[lin<2>(x / 3, y / 3, 0, nvc)] = c;
        }
      }
    }
    Rb[j] = res;
  }
  __syncthreads();
  restrict_x_pass<T>(Rb, Xw, Xm, rts, tid);
  __syncthreads();
  if (tid < NCO * NCO) {
    const int ccx = tid % NCO, ccy = tid / NCO;
    const int cx = x0 / 3 + ccx, cy = y0 / 3 + ccy;
    if (cx > 0 && cx < nc && cy > 0 && cy < nc) {
      T W = T(0), Y = T(0);
#pragma unroll
      for (int o = -2; o <= 2; ++o) {
        const int row = 3 * ccy + 2 + o;
        W += wlin<T>(o) * Xw[row * NCO + ccx];
        Y += rts.m[o + 2] * Rb[row * RW + 3 * ccx + 2];
      }
      const T X = Xm[(3 * ccy + 2) * NCO + ccx];
      const size_t ci = lin<2>(cx, cy, 0, nvc);
      C.rr[ci] = W;
      C.bt[ci] = jac ? rts.scale * (X + Y) : T(0);
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

// Constant-coefficient 3D sweeps run on the 32-wide ring (k_sweep3d_w32) unless this is 0.
#ifndef ADAFAC_SWEEP3D_W32
#define ADAFAC_SWEEP3D_W32 1
#endif
constexpr bool kSweepW32 = ADAFAC_SWEEP3D_W32 != 0;

static int pick_tz(int n) {
  // longest z chunk (multiple of 3 dividing n, <= MAXTZ) that still gives one workgroup per CU
  // of the 256 (fewer, longer chunks re-read fewer halo planes)
  const int ntx = n / TX;
  if (ADAFAC_SWEEP3D_TZ > 0 && n % ADAFAC_SWEEP3D_TZ == 0) return ADAFAC_SWEEP3D_TZ;
  int best = 3;
  for (int tz = 3; tz <= MAXTZ; tz *= 3)
    if (n % tz == 0 && size_t(ntx) * ntx * (n / tz) >= 240) best = tz;
  return best;
}

template <typename T>
static hipError_t launch_sweep3d(const Sweep3dArgs<T>& a, bool var, hipStream_t s) {
  const unsigned nb = unsigned(a.ntx * a.ntx * a.ntz);
  const bool pend = a.apply_pending != 0;
  if (a.coarse) {
    if (var)
      k_fine_sweep3d<T, true, true, false><<<nb, NT3, 0, s>>>(a);
    else if (kSweepW32)
      k_sweep3d_w32<T, true, false><<<nb, NT3, 0, s>>>(a);
    else
      k_fine_sweep3d<T, false, true, false><<<nb, NT3, 0, s>>>(a);
  } else if (var) {
    if (pend)
      k_fine_sweep3d<T, true, false, true><<<nb, NT3, 0, s>>>(a);
    else
      k_fine_sweep3d<T, true, false, false><<<nb, NT3, 0, s>>>(a);
  } else if (kSweepW32) {
    if (pend)
      k_sweep3d_w32<T, false, true><<<nb, NT3, 0, s>>>(a);
    else
      k_sweep3d_w32<T, false, false><<<nb, NT3, 0, s>>>(a);
  } else {
    if (pend)
      k_fine_sweep3d<T, false, false, true><<<nb, NT3, 0, s>>>(a);
    else
      k_fine_sweep3d<T, false, false, false><<<nb, NT3, 0, s>>>(a);
  }
  return hipGetLastError();
}

bool sweep_level_ok(int d, int n, int fem, bool has_pw) {
  return d == 3 && fem && n % TX == 0 && !has_pw;
}

// FAS update of a coarse level L (3^l >= 27 cells per axis, Q1 operator, d-linear transfer
// into it) in one tiled pass that also restricts into the next coarser level C.
template <typename T>
hipError_t launch_coarse_sweep(int d, const LevelView<T>& L, const LevelView<T>& C, const RtSep<T>& rts,
                               T omega, T omega_t, T cscale, int damping, hipStream_t s,
                               const unsigned long long* stop, unsigned long long need) {
  if (d != 3 || L.n % TX || L.pw || !L.fem) return hipErrorInvalidValue;
  const int n = L.n, ntx = n / TX, tz = pick_tz(n), ntz = n / tz;
  Sweep3dArgs<T> a{L.u, nullptr, L.rr, C.S, C.u, C.rr, C.bt, L.eps, nullptr, L.h, omega, L.hd, rts,
                   n, L.nv, C.n, C.nv, L.nb, L.bs, tz, ntx, ntz, damping, 0,
                   1, L.bt, L.S, L.bf, L.r, omega_t, cscale, nullptr, stop, need};
  if (damping == ADAFAC_DAMP_PI) {
    if (!C.ic) return hipErrorInvalidValue;
    a.ic = C.ic;
  }
  return launch_sweep3d<T>(a, L.eps != nullptr, s);
}

int fine_sweep_nparts(int d, int n) {
  if (n % TX) return 0;
  const int ntx = n / TX;
  return d == 2 ? ntx * ntx : ntx * ntx * (n / pick_tz(n));
}

template <typename T>
hipError_t launch_fine_sweep(int d, const LevelView<T>& F, const LevelView<T>& C, const T* uin, T* uout,
                             const T* b, const RtSep<T>& rts, T omega, int damping, int apply_pending,
                             double* partials, int* nparts, hipStream_t s, const unsigned long long* stop,
                             unsigned long long need) {
  const int n = F.n;
  if (n % TX || F.pw) return hipErrorInvalidValue;   // needs 27 | n and d-linear transfer into L
  const int ntx = n / TX;
  const bool var = F.eps != nullptr;
  if (damping == ADAFAC_DAMP_PI && !C.ic) return hipErrorInvalidValue;
  if (d == 2) {
    const unsigned nb = unsigned(ntx * ntx);
    if (var)
      k_fine_sweep2d<T, true><<<nb, 256, 0, s>>>(F, C, uin, uout, b, rts, omega, damping, apply_pending, ntx, partials,
                                                 stop, need);
    else
      k_fine_sweep2d<T, false><<<nb, 256, 0, s>>>(F, C, uin, uout, b, rts, omega, damping, apply_pending, ntx, partials,
                                                  stop, need);
    *nparts = int(nb);
  } else {
    const int tz = pick_tz(n), ntz = n / tz;
    const unsigned nb = unsigned(ntx * ntx * ntz);
    Sweep3dArgs<T> a{uin, uout, b, C.S, C.u, C.rr, C.bt, F.eps, partials, F.h, omega, F.hd, rts,
                     n, F.nv, C.n, C.nv, F.nb, F.bs, tz, ntx, ntz, damping, apply_pending,
                     0, nullptr, nullptr, nullptr, nullptr, T(0), T(1), nullptr, stop, need};
    if (damping == ADAFAC_DAMP_PI) a.ic = C.ic;
    const hipError_t e = launch_sweep3d<T>(a, var, s);
    if (e != hipSuccess) return e;
    *nparts = int(nb);
  }
  return hipGetLastError();
}

// FP64 defect step of a 3D level with 27 | n (see k_defect3d).  mode: 0 u' = u, 1 u' = u + e,
// 2 u' = u + e + P S (d-linear P into the level).  *nparts receives the partial count.
hipError_t launch_defect3d(const LevelView<double>& F, int nc, int nvc, const double* uin, double* uout,
                           const float* e, const float* S, const double* b, float* r32, double* partials,
                           int mode, int* nparts, hipStream_t s, const unsigned long long* stop,
                           unsigned long long need) {
  const int n = F.n;
  if (n % TX) return hipErrorInvalidValue;
  const int ntx = n / TX, tz = pick_tz(n), ntz = n / tz;
  Defect3dArgs a{uin,  uout, e,  S,  b,    r32,  F.eps, partials, F.h, F.hd, n,   F.nv,
                 nc,   nvc,  F.nb, F.bs, tz, ntx, ntz,   stop,     need};
  const unsigned nb = unsigned(ntx * ntx * ntz);
  const bool var = F.eps != nullptr;
  if (mode == 2) {
    if (var) k_defect3d<true, 2><<<nb, NTD, 0, s>>>(a);
    else k_defect3d<false, 2><<<nb, NTD, 0, s>>>(a);
  } else if (mode == 1) {
    if (var) k_defect3d<true, 1><<<nb, NTD, 0, s>>>(a);
    else k_defect3d<false, 1><<<nb, NTD, 0, s>>>(a);
  } else {
    if (var) k_defect3d<true, 0><<<nb, NTD, 0, s>>>(a);
    else k_defect3d<false, 0><<<nb, NTD, 0, s>>>(a);
  }
  *nparts = int(nb);
  return hipGetLastError();
}

template hipError_t launch_coarse_sweep<double>(int, const LevelView<double>&, const LevelView<double>&,
                                                const RtSep<double>&, double, double, double, int, hipStream_t,
                                                const unsigned long long*, unsigned long long);
template hipError_t launch_coarse_sweep<float>(int, const LevelView<float>&, const LevelView<float>&,
                                               const RtSep<float>&, float, float, float, int, hipStream_t,
                                               const unsigned long long*, unsigned long long);
template hipError_t launch_fine_sweep<double>(int, const LevelView<double>&, const LevelView<double>&,
                                              const double*, double*, const double*, const RtSep<double>&,
                                              double, int, int, double*, int*, hipStream_t,
                                              const unsigned long long*, unsigned long long);
template hipError_t launch_fine_sweep<float>(int, const LevelView<float>&, const LevelView<float>&,
                                             const float*, float*, const float*, const RtSep<float>&, float,
                                             int, int, double*, int*, hipStream_t, const unsigned long long*,
                                             unsigned long long);

}  // namespace adafac
