// C ABI of the adAFAC solver (include/adafac.h): context, host setup, workspace layout and
// the sequencing of the gfx950 kernels of one cycle on the bound stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "adafac.h"
#include "adafac_internal.hpp"
#include "adaptive.hpp"

namespace adafac {

template <typename T>
hipError_t launch_fine_residual(int d, const LevelView<T>& F, const T* uin, T* uout, const T* b, T* r,
                                T* ic_coarse, int nvc, T omega, int pi, double* partials, int nblocks,
                                hipStream_t s, Gate g = Gate{});
template <typename T>
hipError_t launch_level_update(int d, const LevelView<T>& C, const LevelView<T>& F, const LevelView<T>& Cm,
                               const RtSep<T>& rt, T omega, T omega_t, T cscale, int damping, int gather,
                               hipStream_t s, Gate g = Gate{});
template <typename T>
hipError_t launch_prolong_add(int d, const LevelView<T>& F, const LevelView<T>& C, T* dst, const T* src,
                              const T* sub, hipStream_t s, const T* self = nullptr, Gate g = Gate{});
hipError_t launch_norm_finalize(const double* partials, int n, double* out, hipStream_t s, Gate g = Gate{},
                                StopRule rule = StopRule{});
hipError_t launch_stream_copy(const void* src, void* dst, size_t n16, hipStream_t s);
hipError_t launch_accumulate(int d, const LevelView<float>& F, const LevelView<float>& C, double* u,
                             const float* e, const float* S, hipStream_t s);
hipError_t launch_defect(int d, const LevelView<double>& F, const double* u, const double* b, float* r32,
                         double* partials, int nblocks, hipStream_t s);
template <typename T>
hipError_t launch_fine_sweep(int d, const LevelView<T>& F, const LevelView<T>& C, const T* uin, T* uout,
                             const T* b, const RtSep<T>& rt, T omega, int damping, int apply_pending,
                             double* partials, int* nparts, hipStream_t s, const unsigned long long* stop = nullptr,
                             unsigned long long need = 0);
size_t fine_sweep_partials(int d, int n);
int fine_sweep_nparts(int d, int n);
template <typename T>
hipError_t launch_coarse_sweep(int d, const LevelView<T>& L, const LevelView<T>& C, const RtSep<T>& rts,
                               T omega, T omega_t, T cscale, int damping, hipStream_t s,
                               const unsigned long long* stop = nullptr, unsigned long long need = 0);
bool sweep_level_ok(int d, int n, int fem, bool has_pw);
hipError_t launch_defect3d(const LevelView<double>& F, int nc, int nvc, const double* uin, double* uout,
                           const float* e, const float* S, const double* b, float* r32, double* partials,
                           int mode, int* nparts, hipStream_t s, const unsigned long long* stop = nullptr,
                           unsigned long long need = 0);
template <typename T>
hipError_t launch_small_levels(int d, const SmallLevelsArgs<T>& a, size_t lds_bytes, hipStream_t s);
template <typename T>
hipError_t launch_prolong_chain(int d, const ProlongChainArgs<T>& a, hipStream_t s);
hipError_t launch_zero_fill(void* p, size_t bytes, hipStream_t s);
void static_ws_forget(const adafac_ctx* c);

}  // namespace adafac

using namespace adafac;

namespace {
constexpr int kMaxHist = 1 << 14;
// Levels with at most this many vertices are updated together by one workgroup.
#ifndef ADAFAC_SMALL_VERTS
#define ADAFAC_SMALL_VERTS 256
#endif
constexpr size_t kSmallVerts = ADAFAC_SMALL_VERTS;
constexpr int kTimingPool = 256;
// Flags of the kernel-timing events.  These events only bracket the timed kernel on its own
// stream and are read after a stream synchronisation, so they need no system-scope fence: with
// the default flags every record writes back and invalidates the caches, a few microseconds of
// dead time per record that the timed cycle would otherwise carry.
#ifndef ADAFAC_TIMING_EVENT_FLAGS
#define ADAFAC_TIMING_EVENT_FLAGS hipEventDisableSystemFence
#endif

// The device hierarchy of one arithmetic precision: level views, the finest-level iterate
// (ping-pong, the Jacobi step reads the old neighbours), its right-hand side and residual.
template <typename T>
struct Hier {
  LevelView<T> v[kMaxLevel + 1]{};
  T* ufine[2] = {nullptr, nullptr};
  T* bfine = nullptr;
  T* rfine = nullptr;
  T* eps = nullptr;
  T* Salt[kMaxLevel + 1]{};  // second S of the levels below L-1: a prolongation chain's output
  int swap_lo = 0, swap_hi = 0;   // levels whose S and Salt the last cycle swapped
  RtSep<T> rts{};
  int cur = 0;
  bool pending = false;     // fused path: P S_{L-1} of the last cycle not yet added to the iterate
};
}  // namespace

struct adafac_ctx {
  int dim = 2, lmin = 1, L = 1;
  int nb = 1;
  std::vector<double> eps{1.0};
  std::vector<double> f;
  std::vector<double> gdir;     // Dirichlet data on the finest lattice (boundary entries; empty: u = 0 there)
  adafac_opts opts{};
  HostOps ops;
  bool built = false, bound = false;
  std::string err;
  // device
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t ws_need = 0;       // workspace size of the built hierarchy
  hipStream_t stream = nullptr;
  Hier<double> h64;         // FP64 form; for FP32_REFINED only the finest level (u, b, operator)
  Hier<float> h32;          // FP32_REFINED: inner cycles on A e = r, ufine = e, bfine = r
  float* ezero = nullptr;   // FP32_REFINED: e = 0, the iterate every inner solve starts from
  bool e_pending = false;   // FP32_REFINED: inner correction not yet added to the FP64 solution
  double* partials = nullptr;
  size_t npartials = 0;
  double* partials_inner = nullptr;   // adaptive FP32_REFINED: the inner cycles' norm partials
  double* norms = nullptr;  // (l2h, linf) per cycle or outer step, ring of kMaxHist
  double* scratch_norm = nullptr;
  double* norm0 = nullptr;  // (l2h, linf) of iterate 0, kept beyond the ring
  unsigned long long* stopseq = nullptr;   // pipelined solve: first cycle index whose launches do nothing
  double r0 = -1.0;         // l2h of iterate 0 (host copy, set by solve)
  int ncyc = 0;
  // adaptive spacetree (set_refinement / refine_ball)
  std::vector<RefineSpec> refine;
  double ball_c[3] = {0, 0, 0};
  double ball_r = 0.0;
  int ball_from = 0;
  bool adaptive = false;
  AdaptHost at;
  RtSep<double> ad_rts{};
  std::vector<AdaptLevel> ad;           // device views by level
  std::vector<size_t> ad_part;          // first norm-partial slot of each level's up launch
  std::vector<int> ad_tiled;            // level restricts from its finer level with the tiled kernel
  int ad_tiled_min = kAdaptTiledMinTiles;   // tiles from which it does (fixed at build_operators)
  double* ad_eps = nullptr;
  std::vector<AdaptLevelT<float>> ad32; // FP32_REFINED: inner cycles on the defect equation
  RtSep<float> ad_rts32{};
  float* ad_eps32 = nullptr;
  // right-hand side: a lattice (set_rhs_lattice) or a Gaussian source (set_rhs_gaussian)
  int src_gauss = 0;
  double (*src_fn)(const double*, void*) = nullptr;   // set_rhs_fn: f evaluated where the load is formed
  void* src_user = nullptr;
  double src_c[3] = {0, 0, 0}, src_sigma = 1.0, src_amp = 1.0;
  double next_src_c[3] = {0, 0, 0};
  AdaptHost at_next;                    // regrid: the prepared tree, its right-hand side and size
  std::vector<double> f_next;
  size_t next_need = 0;
  bool next_ready = false;
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
  double t_acc = 0.0;
  int t_launches = 0;
};

namespace {

int fail(adafac_ctx* c, int code, const std::string& m) {
  if (c) c->err = m;
  return code;
}

#define HIPCHK(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, ADAFAC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t nverts_of(int d, int l) {
  size_t nv = size_t(ipow3(l) + 1);
  return d == 2 ? nv * nv : nv * nv * nv;
}

bool mixed(const adafac_ctx* c) { return c->opts.precision == ADAFAC_PREC_FP32_REFINED; }

// f at the finest-lattice point (gx, gy, gz)
double source_at(const adafac_ctx* c, size_t gx, size_t gy, size_t gz) {
  const size_t nL = size_t(ipow3(c->L)) + 1;
  const double h = 1.0 / double(nL - 1);
  if (c->src_fn) {
    const double x[3] = {gx * h, gy * h, gz * h};
    return c->src_fn(x, c->src_user);
  }
  if (!c->src_gauss) return c->f[(gz * nL + gy) * nL + gx];
  const double x[3] = {gx * h, gy * h, gz * h};
  double r2 = 0.0;
  for (int a = 0; a < c->dim; ++a) r2 += (x[a] - c->src_c[a]) * (x[a] - c->src_c[a]);
  return c->src_amp * std::exp(-r2 / (2.0 * c->src_sigma * c->src_sigma));
}

// Lay out every device array inside the workspace; with base == nullptr only sizes.
size_t layout_adaptive(adafac_ctx* c, char* base);

size_t layout(adafac_ctx* c, char* base) {
  if (c->adaptive) return layout_adaptive(c, base);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) & ~size_t(255);
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const int d = c->dim;
  const int ns = d == 2 ? 9 : 27;
  const bool mp = mixed(c);
  auto views = [&](auto& H, auto tag, bool coarse_arrays) {
    using T = decltype(tag);
    const bool unit = c->ops.nb == 1 && c->ops.eps[0] == 1.0;
    H.eps = reinterpret_cast<T*>(take(sizeof(T) * c->ops.eps.size()));
    for (int l = c->lmin; l <= c->L; ++l) {
      const HostLevel& hl = c->ops.lev[l];
      LevelView<T>& v = H.v[l];
      v = LevelView<T>{};
      v.n = hl.n;
      v.nv = hl.nv;
      v.h = T(hl.h);
      v.hd = T(std::pow(hl.h, d));
      v.hdm2 = T(std::pow(hl.h, d - 2));
      v.fem = hl.fem ? 1 : 0;
      v.nb = c->ops.nb;
      v.bs = hl.fem ? ipow3(l - c->ops.k) : 1;
      v.bsm = v.bs > 1 ? unsigned(((uint64_t(1) << 32) + uint64_t(v.bs) - 1) / uint64_t(v.bs)) : 0u;
      v.eps = unit ? nullptr : H.eps;
      if (!coarse_arrays && l < c->L) continue;
      const size_t nvx = hl.nverts;
      if (!hl.fem) {
        v.st = reinterpret_cast<T*>(take(sizeof(T) * nvx * ns));
        v.dg = reinterpret_cast<T*>(take(sizeof(T) * nvx));
      }
      if (!hl.pw.empty()) v.pw = reinterpret_cast<T*>(take(sizeof(T) * nvx * (1u << d)));
      if (l < c->L) {
        v.u = reinterpret_cast<T*>(take(sizeof(T) * nvx));
        v.rr = reinterpret_cast<T*>(take(sizeof(T) * nvx));
        v.bt = reinterpret_cast<T*>(take(sizeof(T) * nvx));
        v.bf = reinterpret_cast<T*>(take(sizeof(T) * nvx));
        v.r = reinterpret_cast<T*>(take(sizeof(T) * nvx));
        v.S = reinterpret_cast<T*>(take(sizeof(T) * nvx));
        v.ic = reinterpret_cast<T*>(take(sizeof(T) * nvx));
        if (!hl.rtw.empty()) v.rtw = reinterpret_cast<T*>(take(sizeof(T) * hl.rtw.size()));
        H.Salt[l] = l < c->L - 1 ? reinterpret_cast<T*>(take(sizeof(T) * nvx)) : nullptr;
      }
    }
    const size_t nvL = c->ops.lev[c->L].nverts;
    H.ufine[0] = reinterpret_cast<T*>(take(sizeof(T) * nvL));
    H.ufine[1] = reinterpret_cast<T*>(take(sizeof(T) * nvL));
    H.bfine = reinterpret_cast<T*>(take(sizeof(T) * nvL));
  };
  views(c->h64, double{}, !mp);
  c->h64.rfine = mp ? nullptr : reinterpret_cast<double*>(take(sizeof(double) * c->ops.lev[c->L].nverts));
  if (mp) {
    views(c->h32, float{}, true);
    c->h32.rfine = reinterpret_cast<float*>(take(sizeof(float) * c->ops.lev[c->L].nverts));
    c->ezero = reinterpret_cast<float*>(take(sizeof(float) * c->ops.lev[c->L].nverts));
  } else {
    c->h32 = Hier<float>{};
    c->ezero = nullptr;
  }
  c->npartials = std::max<size_t>(kNormBlocks, fine_sweep_partials(d, ipow3(c->L)));
  c->partials = reinterpret_cast<double*>(take(sizeof(double) * 2 * c->npartials));
  c->norms = reinterpret_cast<double*>(take(sizeof(double) * 2 * kMaxHist));
  c->scratch_norm = reinterpret_cast<double*>(take(sizeof(double) * 2));
  c->norm0 = reinterpret_cast<double*>(take(sizeof(double) * 2));
  c->stopseq = reinterpret_cast<unsigned long long*>(take(sizeof(unsigned long long)));
  return (off + 255) & ~size_t(255);
}

bool ready(adafac_ctx* c) { return c && c->bound; }

// the single-pass sweep needs 27 | 3^L (L >= 3) and d-linear transfer into the finest level
bool fused_ok(const adafac_ctx* c) { return c->L >= 3 && c->ops.lev[c->L].pw.empty(); }

int record_start(adafac_ctx* c) {
  if (!c->timing) return ADAFAC_OK;
  if (c->ev_used + 2 > int(c->ev.size())) {
    // pool full: fold the finished pairs into the accumulator
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i + 1 < c->ev_used; i += 2) {
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
      c->t_acc += ms;
    }
    c->ev_used = 0;
  }
  HIPCHK(c, hipEventRecord(c->ev[c->ev_used], c->stream));
  return ADAFAC_OK;
}

int record_stop(adafac_ctx* c) {
  if (!c->timing) return ADAFAC_OK;
  HIPCHK(c, hipEventRecord(c->ev[c->ev_used + 1], c->stream));
  c->ev_used += 2;
  c->t_launches += 1;
  return ADAFAC_OK;
}

// Coarse levels are swept with the tiled kernel when they have at least this many cells per
// axis (fewer tiles than CUs otherwise, and the short z march is latency bound).
#ifndef ADAFAC_COARSE_SWEEP_MIN_N
#define ADAFAC_COARSE_SWEEP_MIN_N 81
#endif
constexpr int kCoarseSweepMinN = ADAFAC_COARSE_SWEEP_MIN_N;

// One adAFAC cycle in the arithmetic of T on hierarchy H: residual (and norms into norm_out)
// of the current finest iterate, FAS restriction cascade, coarse corrections, prolongation; the
// next iterate lands in H.ufine[1 - H.cur].  uin_zero (may be nullptr) replaces the current
// iterate by a zero lattice (first inner cycle of a defect-correction step).  rule (may be
// nullptr): a pipelined solve's cycle rule->need, every launch gated on rule->stop, the stopping
// rule applied where the norms are formed.
template <typename T>
int run_cycle(adafac_ctx* c, Hier<T>& H, double* norm_out, const T* uin_zero, const StopRule* rule = nullptr) {
  const int d = c->dim, L = c->L, lmin = c->lmin;
  const adafac_opts& o = c->opts;
  const int damping = o.damping;
  const int pi = damping == ADAFAC_DAMP_PI;
  const T omega = T(o.omega), omega_t = T(o.omega_tilde);
  const T* uin = uin_zero ? uin_zero : H.ufine[H.cur];
  T* uout = H.ufine[1 - H.cur];
  LevelView<T> F = H.v[L];
  F.u = const_cast<T*>(uin);
  F.r = H.rfine;
  LevelView<T> Lm1 = L > lmin ? H.v[L - 1] : LevelView<T>{};
  int nparts = kNormBlocks;
  int rc;
  // smallest levels lo..hi for the single-workgroup kernel
  int hi = lmin - 1;
  for (int l = lmin; l < L && l - lmin < kMaxSmall && nverts_of(d, l) <= kSmallVerts; ++l) hi = l;
  // The stored R~ of the OPERATOR form is a per-vertex gather: one kernel per step.  adAFAC-PI
  // (c~_l = P I c_l) in the single-pass form: the sweeps write I c_l to level l-1, and the last
  // prolongation into level L-1 subtracts I c_L there, so that S_{L-1} holds S_{L-1} - I c_L and
  // the pending P S_{L-1} of the next sweep is P (S_{L-1} - I c_L).  That needs a prolongation
  // launch into L-1 (L-1 above l_min and above the single-workgroup levels).
  const bool opr = o.rtilde == ADAFAC_RTILDE_OPERATOR;
  const bool fused = o.fused && L > lmin && !opr && fused_ok(c) && (!pi || (L - 1 > lmin && L - 1 > hi));
  const bool pend = H.pending && !uin_zero;
  const Gate gate = rule ? Gate{rule->stop, rule->need} : Gate{};
  const StopRule norm_rule = rule ? *rule : StopRule{};
  if ((rc = record_start(c))) return rc;
  if (fused) {
    HIPCHK(c, launch_fine_sweep<T>(d, F, Lm1, uin, uout, H.bfine, H.rts, omega, damping, pend ? 1 : 0,
                                   c->partials, &nparts, c->stream, gate.stop, gate.need));
  } else {
    HIPCHK(c, launch_fine_residual<T>(d, F, uin, uout, H.bfine, H.rfine, pi ? Lm1.ic : nullptr, Lm1.nv, omega,
                                      pi, c->partials, kNormBlocks, c->stream, gate));
  }
  if ((rc = record_stop(c))) return rc;
  auto cscale_of = [&](int l) { return T(damping == ADAFAC_DAMP_EXP ? std::pow(o.omega_hat, L - l) : 1.0); };
  bool fed = fused;               // level l's u, R r and R~ r already written by the finer level
  for (int l = L - 1; l > hi; --l) {
    const bool sweep = !opr && fed && l > lmin && H.v[l].n >= kCoarseSweepMinN &&
                       sweep_level_ok(d, H.v[l].n, H.v[l].fem, H.v[l].pw != nullptr);
    if (sweep) {
      HIPCHK(c, launch_coarse_sweep<T>(d, H.v[l], H.v[l - 1], H.rts, omega, omega_t, cscale_of(l), damping,
                                       c->stream, gate.stop, gate.need));
    } else {
      LevelView<T> Fv = H.v[l + 1];
      if (l + 1 == L) { Fv.u = const_cast<T*>(uin); Fv.r = H.rfine; }
      LevelView<T> Cm = l > lmin ? H.v[l - 1] : LevelView<T>{};
      HIPCHK(c, launch_level_update<T>(d, H.v[l], Fv, Cm, H.rts, omega, omega_t, cscale_of(l), damping,
                                       fed ? 0 : 1, c->stream, gate));
    }
    fed = sweep;
  }
  if (hi >= lmin) {
    SmallLevelsArgs<T> a{};
    a.lo = lmin;
    a.hi = hi;
    for (int l = lmin - 1; l <= hi + 1; ++l) {
      LevelView<T> v = (l >= lmin) ? H.v[l] : LevelView<T>{};
      if (l == L) { v.u = const_cast<T*>(uin); v.r = H.rfine; }
      a.lv[l - lmin + 1] = v;
    }
    for (int l = lmin; l <= hi; ++l) {
      a.gather[l - lmin] = (l == hi && fed) ? 0 : 1;
      a.cscale[l - lmin] = cscale_of(l);
    }
    a.rts = H.rts;
    a.omega = omega;
    a.omega_t = omega_t;
    a.damping = damping;
    a.partials = c->partials;
    a.nparts = nparts;
    a.norm_out = norm_out;
    a.gate = gate;
    a.rule = norm_rule;
    HIPCHK(c, launch_small_levels<T>(d, a, 0, c->stream));
  } else {
    HIPCHK(c, launch_norm_finalize(c->partials, nparts, norm_out, c->stream, gate, norm_rule));
  }
  const int l0 = std::max(hi + 1, lmin + 1), nt = L - l0;
  if (nt >= 2 && nt <= kMaxChain) {
    // S_l += P S_{l-1} for l = l0 .. L-1 in one launch; the levels below L-1 get their new S in
    // their second buffer, which then becomes their S
    ProlongChainArgs<T> a{};
    a.nt = nt;
    for (int k = 0; k <= nt; ++k) a.lv[k] = H.v[l0 - 1 + k];
    for (int k = 0; k < nt; ++k) {
      a.sub[k] = pi ? H.v[l0 - 1 + k].ic : nullptr;
      a.out[k] = k > 0 ? H.Salt[l0 - 1 + k] : nullptr;
    }
    a.self = (pi && fused) ? H.v[L - 1].ic : nullptr;
    a.gate = gate;
    HIPCHK(c, launch_prolong_chain<T>(d, a, c->stream));
    for (int l = l0; l < L - 1; ++l) std::swap(H.v[l].S, H.Salt[l]);
    H.swap_lo = l0;
    H.swap_hi = L - 1;
  } else {
    for (int l = l0; l < L; ++l)
      HIPCHK(c, launch_prolong_add<T>(d, H.v[l], H.v[l - 1], H.v[l].S, H.v[l - 1].S,
                                      pi ? H.v[l - 1].ic : nullptr, c->stream,
                                      (pi && fused && l == L - 1) ? H.v[l].ic : nullptr, gate));
  }
  if (fused) {
    H.pending = true;        // P S_{L-1} enters the next sweep (or the flush)
  } else {
    H.pending = false;
    if (L > lmin)
      HIPCHK(c, launch_prolong_add<T>(d, H.v[L], H.v[L - 1], uout, H.v[L - 1].S,
                                      pi ? H.v[L - 1].ic : nullptr, c->stream, nullptr, gate));
  }
  H.cur = 1 - H.cur;
  return ADAFAC_OK;
}

// Add the pending prolongated coarse correction to the current FP64 iterate (FP64 form), or
// the pending inner correction e + P S_{L-1} to the FP64 solution (FP32_REFINED).
int adapt_hang(adafac_ctx* c);
int adapt_accumulate(adafac_ctx* c);

int flush(adafac_ctx* c) {
  const int L = c->L;
  if (c->adaptive) {
    int rc = adapt_accumulate(c);
    return rc ? rc : adapt_hang(c);
  }
  if (mixed(c)) {
    if (!c->e_pending) return ADAFAC_OK;
    Hier<float>& H = c->h32;
    const float* S = (H.pending && L > c->lmin) ? H.v[L - 1].S : nullptr;
    LevelView<float> C = L > c->lmin ? H.v[L - 1] : LevelView<float>{};
    HIPCHK(c, launch_accumulate(c->dim, H.v[L], C, c->h64.ufine[c->h64.cur], H.ufine[H.cur], S, c->stream));
    H.pending = false;
    c->e_pending = false;
    return ADAFAC_OK;
  }
  Hier<double>& H = c->h64;
  if (!H.pending) return ADAFAC_OK;
  // pending only after a fused cycle, whose S_{L-1} already holds S_{L-1} - I c_L under adAFAC-PI
  HIPCHK(c, launch_prolong_add<double>(c->dim, H.v[L], H.v[L - 1], H.ufine[H.cur], H.v[L - 1].S, nullptr,
                                       c->stream));
  H.pending = false;
  return ADAFAC_OK;
}

// ---------------------------------------------------------------------------
// Adaptive spacetrees: per-level box arrays and the cycle over the ragged levels
// ---------------------------------------------------------------------------
// Does level l of an adaptive tree take BoxMG weights from the next coarser level (a complete
// level l <= k whose host transfer is stored)?
bool adapt_pw_level(const adafac_ctx* c, int l) {
  return l > c->lmin && l <= c->L && l < int(c->ops.lev.size()) && !c->ops.lev[l].pw.empty();
}

size_t layout_adaptive_tree(adafac_ctx* c, const AdaptHost& t, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) & ~size_t(255);
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const int d = c->dim;
  const bool mp = mixed(c);
  std::vector<AdaptLevel> ad(c->L + 1, AdaptLevel{});
  std::vector<AdaptLevelT<float>> ad32(mp ? c->L + 1 : 0, AdaptLevelT<float>{});
  double* eps = reinterpret_cast<double*>(take(sizeof(double) * c->ops.eps.size()));
  float* eps32 = mp ? reinterpret_cast<float*>(take(sizeof(float) * c->ops.eps.size())) : nullptr;
  const bool unit = c->ops.nb == 1 && c->ops.eps[0] == 1.0;
  for (int l = c->lmin; l <= c->L; ++l) {
    const AdaptHostLevel& H = t.lev[l];
    AdaptLevel& A = ad[l];
    A.ox = H.lo[0];
    A.oy = H.lo[1];
    A.oz = d == 3 ? H.lo[2] : 0;
    A.mx = H.nc[0] + 1;
    A.my = H.nc[1] + 1;
    A.mz = d == 3 ? H.nc[2] + 1 : 1;
    A.n = ipow3(l);
    A.h = 1.0 / A.n;
    A.hd = std::pow(A.h, d);
    A.hdm2 = std::pow(A.h, d - 2);
    A.fem = H.dg.empty() ? 1 : 0;
    A.nb = c->ops.nb;
    A.bs = A.fem ? ipow3(l - c->ops.k) : 1;
    A.eps = unit ? nullptr : eps;
    const size_t nv = H.nverts(), ncell = H.ncells();
    A.vcls = reinterpret_cast<uint8_t*>(take(nv));
    A.leaf = reinterpret_cast<uint8_t*>(take(ncell));
    A.dg = reinterpret_cast<double*>(take(sizeof(double) * nv));
    A.wc = reinterpret_cast<double*>(take(sizeof(double) * ncell));
    A.bleaf = reinterpret_cast<double*>(take(sizeof(double) * nv));
    A.u = reinterpret_cast<double*>(take(sizeof(double) * nv));
    A.bb = reinterpret_cast<double*>(take(sizeof(double) * nv));
    A.hh = reinterpret_cast<double*>(take(sizeof(double) * nv));
    A.nrun = unsigned(H.run.size() / 2);
    A.nhrun = unsigned(H.hrun.size() / 2);
    A.run = reinterpret_cast<const uint2*>(take(sizeof(uint2) * A.nrun));
    A.hrun = reinterpret_cast<const uint2*>(take(sizeof(uint2) * A.nhrun));
    const bool boxpw = adapt_pw_level(c, l);
    if (boxpw) A.pw = reinterpret_cast<double*>(take(sizeof(double) * nv << d));
    if (!mp) {
      A.s = reinterpret_cast<double*>(take(sizeof(double) * nv));
      A.S = reinterpret_cast<double*>(take(sizeof(double) * nv));
      continue;
    }
    // FP32_REFINED: the FP64 levels only hold u and the outer defect; the cycles run on E
    AdaptLevelT<float>& E = ad32[l];
    E.ox = A.ox, E.oy = A.oy, E.oz = A.oz, E.mx = A.mx, E.my = A.my, E.mz = A.mz;
    E.n = A.n;
    E.h = float(A.h);
    E.hd = float(A.hd);
    E.hdm2 = float(A.hdm2);
    E.fem = A.fem;
    E.nb = A.nb;
    E.bs = A.bs;
    E.eps = unit ? nullptr : eps32;
    E.vcls = A.vcls;
    E.leaf = A.leaf;
    E.run = A.run;
    E.hrun = A.hrun;
    E.nrun = A.nrun;
    E.nhrun = A.nhrun;
    E.dg = reinterpret_cast<float*>(take(sizeof(float) * nv));
    E.wc = reinterpret_cast<float*>(take(sizeof(float) * ncell));
    E.bleaf = reinterpret_cast<float*>(take(sizeof(float) * nv));
    E.u = reinterpret_cast<float*>(take(sizeof(float) * nv));
    E.bb = reinterpret_cast<float*>(take(sizeof(float) * nv));
    E.hh = reinterpret_cast<float*>(take(sizeof(float) * nv));
    E.s = reinterpret_cast<float*>(take(sizeof(float) * nv));
    E.S = reinterpret_cast<float*>(take(sizeof(float) * nv));
    if (boxpw) E.pw = reinterpret_cast<float*>(take(sizeof(float) * nv << d));
  }
  // norm partials: one slot per block of each level's up launch, levels packed
  std::vector<size_t> part(c->L + 1, 0);
  std::vector<int> tiled(c->L + 1, 0);
  const int min_tiles = c->ad_tiled_min;
  size_t npart = 0;
  for (int l = c->lmin; l <= c->L; ++l) {
    part[l] = npart;
    const AdaptHostLevel& H = t.lev[l];
    const int mx = H.nc[0] + 1, my = H.nc[1] + 1, mz = d == 3 ? H.nc[2] + 1 : 1;
    // the tiled kernel restricts with d-linear weights only
    tiled[l] = l < c->L && !adapt_pw_level(c, l + 1) && adapt_up_tiled(d, mx, my, mz, min_tiles);
    npart += adapt_up_slots(d, mx, my, mz, l < c->L, tiled[l] != 0);
  }
  double* partials = reinterpret_cast<double*>(take(sizeof(double) * 2 * npart));
  // the inner cycles run other kernels on some levels (so other slot counts): own partials, so
  // that the outer step's norms never read the inner cycles' slots
  double* partials_inner = mp ? reinterpret_cast<double*>(take(sizeof(double) * 2 * npart)) : nullptr;
  double* norms = reinterpret_cast<double*>(take(sizeof(double) * 2 * kMaxHist));
  double* scratch = reinterpret_cast<double*>(take(sizeof(double) * 2));
  double* norm0 = reinterpret_cast<double*>(take(sizeof(double) * 2));
  auto* stopseq = reinterpret_cast<unsigned long long*>(take(sizeof(unsigned long long)));
  if (base) {
    c->ad = std::move(ad);
    c->ad_part = std::move(part);
    c->ad_tiled = std::move(tiled);
    c->ad_eps = eps;
    c->ad32 = std::move(ad32);
    c->ad_eps32 = eps32;
    c->npartials = npart;
    c->partials = partials;
    c->partials_inner = partials_inner;
    c->norms = norms;
    c->scratch_norm = scratch;
    c->norm0 = norm0;
    c->stopseq = stopseq;
  }
  return (off + 255) & ~size_t(255);
}

size_t layout_adaptive(adafac_ctx* c, char* base) { return layout_adaptive_tree(c, c->at, base); }

// hanging vertices interpolated top-down from the current nodal values
template <typename T>
int adapt_hang_views(adafac_ctx* c, const std::vector<AdaptLevelT<T>>& ad, Gate g = Gate{}) {
  for (int l = c->lmin + 1; l <= c->L; ++l) HIPCHK(c, launch_ad_hang<T>(c->dim, ad[l], ad[l - 1], c->stream, g));
  return ADAFAC_OK;
}

int adapt_hang(adafac_ctx* c) { return adapt_hang_views(c, c->ad); }

// FP32_REFINED: the pending inner correction added to the FP64 nodal values
int adapt_accumulate(adafac_ctx* c) {
  if (!mixed(c) || !c->e_pending) return ADAFAC_OK;
  for (int l = c->lmin; l <= c->L; ++l) HIPCHK(c, launch_ad_accumulate(c->dim, c->ad[l], c->ad32[l], c->stream));
  c->e_pending = false;
  return ADAFAC_OK;
}

// One cycle on the levels ad (FP64 form, or an FP32 inner cycle whose leaf loads are the outer
// defect); norms of the composite residual of the input iterate into norm_out.
// rule (may be nullptr): a pipelined solve's cycle, every launch gated (see run_cycle).
template <typename T>
int run_adapt_cycle(adafac_ctx* c, const std::vector<AdaptLevelT<T>>& ad, const RtSep<T>& rts, double* norm_out,
                    const StopRule* rule = nullptr) {
  const Gate gate = rule ? Gate{rule->stop, rule->need} : Gate{};
  const StopRule norm_rule = rule ? *rule : StopRule{};
  const int d = c->dim, L = c->L, lmin = c->lmin;
  const adafac_opts& o = c->opts;
  const T omega = T(o.omega), omega_t = T(o.omega_tilde);
  const int pi = o.damping == ADAFAC_DAMP_PI;
  int rc = adapt_hang_views(c, ad, gate);
  if (rc) return rc;
  if ((rc = record_start(c))) return rc;
  double* partials = std::is_same<T, double>::value ? c->partials : c->partials_inner;
  HIPCHK(c, launch_ad_leaf_up<T>(d, ad[L], omega, omega_t, 0, partials + 2 * c->ad_part[L], c->stream, gate));
  if ((rc = record_stop(c))) return rc;
  for (int l = L - 1; l >= lmin; --l)
    HIPCHK(c, launch_ad_up<T>(d, ad[l], &ad[l + 1], rts, omega, omega_t, o.damping, 0,
                              std::is_same<T, double>::value ? c->ad_tiled[l] : 0, partials + 2 * c->ad_part[l],
                              c->stream, gate));
  HIPCHK(c, launch_ad_norm_finalize(partials, int(c->npartials), norm_out, c->stream, gate, norm_rule));
  // coarsest level first: S_l needs S_{l-1}; each level's updated composite dofs are copied into
  // the coinciding coarser dofs
  AdaptCopyView<T> V{};
  V.lmin = lmin;
  for (int l = lmin; l <= L; ++l)
    V.lv[l] = {ad[l].ox, ad[l].oy, ad[l].oz, ad[l].mx, ad[l].my, ad[l].mz, ad[l].vcls, ad[l].u};
  for (int l = lmin; l <= L; ++l)
    HIPCHK(c, launch_ad_down_update<T>(d, ad[l], l > lmin ? &ad[l - 1] : nullptr, V, l, pi, l < L, c->stream,
                                       gate));
  return ADAFAC_OK;
}

// FP32_REFINED on a tree: the pending correction added to u, then in FP64 the composite
// residual of u and its norms; the residual at the composite dofs (zero elsewhere), rounded to
// FP32, is the leaf load of the next inner solve, whose iterate restarts at zero.  It is the
// same functional as the per-level leaf residuals, without their large parts that cancel
// across refinement boundaries (rounded to FP32 first, they would leave an error of FP32 size
// relative to b, a floor near 1e-8 for the outer iteration).
int run_adapt_outer_mixed(adafac_ctx* c, double* norm_out) {
  const int d = c->dim, L = c->L, lmin = c->lmin;
  int rc = adapt_accumulate(c);
  if (rc || (rc = adapt_hang(c))) return rc;
  if ((rc = record_start(c))) return rc;
  HIPCHK(c, launch_ad_leaf_up<double>(d, c->ad[L], 0.0, 0.0, 1, c->partials + 2 * c->ad_part[L], c->stream));
  if ((rc = record_stop(c))) return rc;
  for (int l = L - 1; l >= lmin; --l)
    HIPCHK(c, launch_ad_up<double>(d, c->ad[l], &c->ad[l + 1], c->ad_rts, 0.0, 0.0, c->opts.damping, 1,
                                   c->ad_tiled[l], c->partials + 2 * c->ad_part[l], c->stream));
  HIPCHK(c, launch_ad_norm_finalize(c->partials, int(c->npartials), norm_out, c->stream));
  for (int l = lmin; l <= L; ++l) HIPCHK(c, launch_ad_to_inner(d, c->ad[l], c->ad32[l], c->stream));
  return ADAFAC_OK;
}

// FP64 form: one cycle.  FP32_REFINED: the FP64 part of an outer step, i.e. the pending inner
// correction added to u and the FP64 defect r = b - A u with its norms (the norms of the outer
// iterate), stored in FP32 as the right-hand side of the next inner solve.
// rule (may be nullptr): a pipelined solve's step (uniform FP64, or the one-pass 3D
// FP32_REFINED outer step), gated and applying the stopping rule.
int run_outer(adafac_ctx* c, const StopRule* rule = nullptr) {
  double* norm_out = c->norms + 2 * (c->ncyc % kMaxHist);
  const Gate gate = rule ? Gate{rule->stop, rule->need} : Gate{};
  const StopRule norm_rule = rule ? *rule : StopRule{};
  if (c->adaptive) {
    if (rule && mixed(c)) return fail(c, ADAFAC_EINVAL, "internal: this outer step is not pipelined");
    int rc = mixed(c) ? run_adapt_outer_mixed(c, norm_out)
                      : run_adapt_cycle<double>(c, c->ad, c->ad_rts, norm_out, rule);
    if (rc) return rc;
  } else if (!mixed(c)) {
    int rc = run_cycle<double>(c, c->h64, norm_out, nullptr, rule);
    if (rc) return rc;
  } else if (c->dim == 3 && c->opts.fused && fused_ok(c)) {
    // one pass: u' = u + e + P S into the other FP64 buffer, and the FP64 defect of u'
    Hier<double>& D = c->h64;
    Hier<float>& H = c->h32;
    const int L = c->L;
    const int mode = !c->e_pending ? 0 : (H.pending ? 2 : 1);
    const LevelView<float> C = L > c->lmin ? H.v[L - 1] : LevelView<float>{};
    int nparts = 0;
    HIPCHK(c, launch_defect3d(D.v[L], C.n, C.nv, D.ufine[D.cur], D.ufine[1 - D.cur], H.ufine[H.cur],
                              mode == 2 ? C.S : nullptr, D.bfine, H.bfine, c->partials, mode, &nparts, c->stream,
                              gate.stop, gate.need));
    HIPCHK(c, launch_norm_finalize(c->partials, nparts, norm_out, c->stream, gate, norm_rule));
    D.cur = 1 - D.cur;
    H.pending = false;
    c->e_pending = false;
  } else {
    if (rule) return fail(c, ADAFAC_EINVAL, "internal: this outer step is not pipelined");
    int rc = flush(c);
    if (rc) return rc;
    HIPCHK(c, launch_defect(c->dim, c->h64.v[c->L], c->h64.ufine[c->h64.cur], c->h64.bfine, c->h32.bfine,
                            c->partials, kNormBlocks, c->stream));
    HIPCHK(c, launch_norm_finalize(c->partials, kNormBlocks, norm_out, c->stream));
  }
  if (c->ncyc == 0)
    HIPCHK(c, hipMemcpyAsync(c->norm0, norm_out, 2 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  c->ncyc += 1;
  return ADAFAC_OK;
}

// FP32_REFINED: inner_k FP32 cycles on A e = r from e = 0; the correction stays pending.
// gate (may be nullptr): a pipelined solve's gate for these cycles (no stopping rule).
int run_inner(adafac_ctx* c, const StopRule* gate = nullptr) {
  if (c->adaptive) {
    for (int j = 0; j < c->opts.inner_k; ++j) {
      int rc = run_adapt_cycle<float>(c, c->ad32, c->ad_rts32, c->scratch_norm);
      if (rc) return rc;
    }
    c->e_pending = true;
    return ADAFAC_OK;
  }
  Hier<float>& H = c->h32;
  H.pending = false;
  for (int j = 0; j < c->opts.inner_k; ++j) {
    int rc = run_cycle<float>(c, H, c->scratch_norm, j == 0 ? c->ezero : nullptr, gate);
    if (rc) return rc;
  }
  c->e_pending = true;
  return ADAFAC_OK;
}

// One step as adafac_cycle defines it: a cycle, or an outer step with its inner solve.
int run_step(adafac_ctx* c) {
  int rc = run_outer(c);
  if (rc || !mixed(c)) return rc;
  return run_inner(c);
}

template <typename T>
int upload_ops(adafac_ctx* c, Hier<T>& H, bool coarse) {
  const int ns = c->dim == 2 ? 9 : 27;
  auto put = [&](T* dst, const std::vector<double>& src) -> int {
    if (std::is_same<T, double>::value) {
      HIPCHK(c, hipMemcpyAsync(dst, src.data(), sizeof(double) * src.size(), hipMemcpyHostToDevice, c->stream));
    } else {
      std::vector<T> tmp(src.begin(), src.end());
      HIPCHK(c, hipMemcpyAsync(dst, tmp.data(), sizeof(T) * tmp.size(), hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));   // tmp goes out of scope
    }
    return ADAFAC_OK;
  };
  int rc;
  if ((rc = put(H.eps, c->ops.eps))) return rc;
  for (int l = c->lmin; l <= c->L; ++l) {
    if (!coarse && l < c->L) continue;
    const HostLevel& hl = c->ops.lev[l];
    LevelView<T>& v = H.v[l];
    if (!hl.fem) {
      if ((rc = put(const_cast<T*>(v.st), hl.st))) return rc;
      if ((rc = put(const_cast<T*>(v.dg), hl.dg))) return rc;
    }
    if (!hl.pw.empty() && (rc = put(const_cast<T*>(v.pw), hl.pw))) return rc;
    if (v.rtw && (rc = put(const_cast<T*>(v.rtw), hl.rtw))) return rc;
    (void)ns;
  }
  for (int i = 0; i < 5; ++i) H.rts.m[i] = T(c->ops.rt_m[i]);
  H.rts.scale = T(c->ops.rt_scale);
  return ADAFAC_OK;
}

// Host set-up of an adaptive context: the tree, the Galerkin diagonals of the uniform levels
// below the coefficient blocks, and the factors of R~.
int build_adaptive(adafac_ctx* c) {
  const adafac_opts& o = c->opts;
  if (o.rtilde != ADAFAC_RTILDE_CONST_EPS1) return fail(c, ADAFAC_EUNSUPPORTED, "adaptive trees use the eps = 1 R~");
  if (o.damping == ADAFAC_DAMP_EXP)
    return fail(c, ADAFAC_EUNSUPPORTED, "adaptive trees support adAFAC-Jac, adAFAC-PI and plain additive damping");
  if (c->L <= c->lmin) return fail(c, ADAFAC_EINVAL, "an adaptive tree needs l_max > l_min");
  int first = c->L;
  for (const RefineSpec& r : c->refine) first = std::min(first, r.level);
  if (c->ball_r > 0.0) first = std::min(first, std::max(c->ball_from, c->lmin));
  if (c->ops.k > first)
    return fail(c, ADAFAC_EINVAL, "coefficient blocks finer than the first refined level of the tree");
  std::string m = build_adapt_tree(c->at, c->dim, c->lmin, c->L, c->refine, c->ball_c, c->ball_r, c->ball_from);
  if (!m.empty()) return fail(c, ADAFAC_EINVAL, m);
  // ADAFAC_AD_TILED_MIN_TILES overrides the tile count from which a 3D level restricts with the
  // tiled kernel (0: every level; tests use it to run that kernel on small trees)
  c->ad_tiled_min = kAdaptTiledMinTiles;
  if (const char* e = std::getenv("ADAFAC_AD_TILED_MIN_TILES")) c->ad_tiled_min = std::max(0, std::atoi(e));
  for (int l = c->lmin; l <= c->L; ++l)
    if (c->at.lev[l].nverts() > size_t(kAdaptMaxBox))
      return fail(c, ADAFAC_EUNSUPPORTED, "a level's bounding box exceeds 2^31 - 1 vertices");
  // uniform hierarchy up to max(k, lmin + 1): R~ factors and Galerkin diagonals below level k
  HostOps u;
  u.dim = c->dim;
  u.lmin = c->lmin;
  u.L = std::max(c->ops.k, c->lmin + 1);
  u.nb = c->nb;
  u.k = c->ops.k;
  u.eps = c->eps;
  // BoxMG (Sec. 2.5): the uniform hierarchy's operator-dependent P into the levels l <= k, which
  // are complete; above k every coarse cell lies inside one block and P is d-linear
  m = build_host_ops(u, o.transfer == ADAFAC_TRANSFER_BOXMG ? 1 : 0, o.omega);
  if (!m.empty()) return fail(c, ADAFAC_EINVAL, m);
  for (int i = 0; i < 5; ++i) {
    c->ad_rts.m[i] = u.rt_m[i];
    c->ad_rts32.m[i] = float(u.rt_m[i]);
  }
  c->ad_rts.scale = u.rt_scale;
  c->ad_rts32.scale = float(u.rt_scale);
  for (int l = c->lmin; l < c->ops.k; ++l) c->at.lev[l].dg = u.lev[l].dg;   // uniform levels: full box
  c->ops.lev = std::move(u.lev);     // kept for host_operator queries of the uniform part
  c->ops.rtilde = u.rtilde;
  c->ops.rt_scale = u.rt_scale;
  for (int i = 0; i < 5; ++i) c->ops.rt_m[i] = u.rt_m[i];
  return ADAFAC_OK;
}

// Uploads of an adaptive context: classes, leaf cells, stored diagonals, lumped loads.
// Dirichlet data at the domain-boundary vertices of level l's box (the values the kernels read
// there: no kernel writes a boundary vertex); other entries untouched.
void fill_boundary(const adafac_ctx* c, int l, std::vector<double>& box) {
  if (c->gdir.empty()) return;
  const int d = c->dim, L = c->L, n = ipow3(l), nL = ipow3(L) + 1, s = ipow3(L - l);
  const AdaptLevel& A = c->ad[l];
  for (int z = 0; z < A.mz; ++z)
    for (int y = 0; y < A.my; ++y)
      for (int x = 0; x < A.mx; ++x) {
        const int gx = A.ox + x, gy = A.oy + y, gz = d == 3 ? A.oz + z : 1;
        const bool bd = gx == 0 || gx == n || gy == 0 || gy == n || (d == 3 && (gz == 0 || gz == n));
        if (!bd) continue;
        const size_t fx = size_t(gx) * s, fy = size_t(gy) * s, fz = d == 3 ? size_t(gz) * s : 0;
        box[(size_t(z) * A.my + y) * A.mx + x] = c->gdir[(fz * nL + fy) * nL + fx];
      }
}

// Whether box vertex (x, y, z) of level l is a corner of an existing cell of that level.
bool vertex_of_cell(const AdaptHostLevel& H, int d, int x, int y, int z) {
  for (int e = 0; e < (1 << d); ++e) {
    const int cx = x - 1 + (e & 1), cy = y - 1 + ((e >> 1) & 1), cz = d == 3 ? z - 1 + ((e >> 2) & 1) : 0;
    if (cx < 0 || cy < 0 || cz < 0 || cx >= H.nc[0] || cy >= H.nc[1] || cz >= H.nc[2]) continue;
    if (H.exists[(size_t(cz) * H.nc[1] + cy) * H.nc[0] + cx]) return true;
  }
  return false;
}

int bind_adaptive(adafac_ctx* c) {
  const int d = c->dim, L = c->L;
  HIPCHK(c, hipMemcpyAsync(c->ad_eps, c->ops.eps.data(), sizeof(double) * c->ops.eps.size(), hipMemcpyHostToDevice,
                           c->stream));
  const bool mp = mixed(c);
  if (mp) {
    std::vector<float> e32(c->ops.eps.begin(), c->ops.eps.end());
    HIPCHK(c, hipMemcpyAsync(c->ad_eps32, e32.data(), sizeof(float) * e32.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  const int nL = ipow3(L) + 1;
  for (int l = c->lmin; l <= L; ++l) {
    const AdaptHostLevel& H = c->at.lev[l];
    const AdaptLevel& A = c->ad[l];
    std::vector<uint8_t> leaf(H.ncells());   // cell classes: 0 none, 1 leaf, 2 refined
    parallel_ranges(leaf.size(), [&](size_t i0, size_t i1) {
      for (size_t i = i0; i < i1; ++i) leaf[i] = H.exists[i] ? (H.refined[i] ? 2 : 1) : 0;
    });
    // lumped load: m_v f_v, m_v = |leaf cells around v| h^d / 2^d, f sampled from the finest lattice
    // (a Gaussian source is evaluated on the device after the uploads)
    std::vector<double> bl(c->src_gauss ? 0 : H.nverts(), 0.0);
    const int s = ipow3(L - l);
    const double share = A.hd / double(1 << d);
    // a user callback runs on the calling thread only
    auto ranges = [&](size_t n, auto&& f) { if (c->src_fn) f(size_t(0), n); else parallel_ranges(n, f); };
    if (!c->src_gauss) ranges(size_t(A.mz), [&](size_t z0, size_t z1) {
      for (int z = int(z0); z < int(z1); ++z)
        for (int y = 0; y < A.my; ++y)
          for (int x = 0; x < A.mx; ++x) {
            const size_t i = (size_t(z) * A.my + y) * A.mx + x;
            if (!(H.vcls[i] & (kDof | kHang))) continue;
            int nleaf = 0;
            for (int e = 0; e < (1 << d); ++e) {
              const int cx = x - 1 + (e & 1), cy = y - 1 + ((e >> 1) & 1), cz = d == 3 ? z - 1 + ((e >> 2) & 1) : 0;
              if (cx < 0 || cy < 0 || cz < 0 || cx >= H.nc[0] || cy >= H.nc[1] || cz >= H.nc[2]) continue;
              nleaf += leaf[(size_t(cz) * H.nc[1] + cy) * H.nc[0] + cx] == 1;
            }
            if (!nleaf) continue;
            const size_t gx = size_t(A.ox + x) * s, gy = size_t(A.oy + y) * s, gz = d == 3 ? size_t(A.oz + z) * s : 0;
            bl[i] = nleaf * share * source_at(c, gx, gy, gz);
          }
    });
    HIPCHK(c, hipMemcpyAsync(const_cast<uint8_t*>(A.vcls), H.vcls.data(), H.vcls.size(), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(const_cast<uint8_t*>(A.leaf), leaf.data(), leaf.size(), hipMemcpyHostToDevice, c->stream));
    if (A.nrun)
      HIPCHK(c, hipMemcpyAsync(const_cast<uint2*>(A.run), H.run.data(), sizeof(uint32_t) * H.run.size(),
                               hipMemcpyHostToDevice, c->stream));
    if (A.nhrun)
      HIPCHK(c, hipMemcpyAsync(const_cast<uint2*>(A.hrun), H.hrun.data(), sizeof(uint32_t) * H.hrun.size(),
                               hipMemcpyHostToDevice, c->stream));
    if (c->src_gauss) {
      GaussSource g{{c->src_c[0], c->src_c[1], c->src_c[2]}, c->src_sigma, c->src_amp};
      HIPCHK(c, launch_ad_gauss_load(d, A, g, c->stream));
    } else {
      HIPCHK(c, hipMemcpyAsync(const_cast<double*>(A.bleaf), bl.data(), sizeof(double) * bl.size(),
                               hipMemcpyHostToDevice, c->stream));
    }
    if (!A.fem)
      HIPCHK(c, hipMemcpyAsync(const_cast<double*>(A.dg), H.dg.data(), sizeof(double) * H.dg.size(),
                               hipMemcpyHostToDevice, c->stream));
    std::vector<double> ub;
    if (!c->gdir.empty()) {
      // the Dirichlet data on the level's boundary vertices, zero inside (the initial iterate,
      // or the zeros a regrid's transfer writes over at the dofs)
      ub.assign(H.nverts(), 0.0);
      fill_boundary(c, l, ub);
      HIPCHK(c, hipMemcpyAsync(A.u, ub.data(), sizeof(double) * ub.size(), hipMemcpyHostToDevice, c->stream));
    }
    std::vector<float> pw32;
    if (A.pw) {
      // a complete level: its box is the whole lattice, so box and lattice indices agree
      const std::vector<double>& pw = c->ops.lev[l].pw;
      if (A.ox || A.oy || A.oz || A.mx != A.n + 1 || pw.size() != (H.nverts() << d))
        return fail(c, ADAFAC_EINVAL, "internal: BoxMG weights on an incomplete level");
      HIPCHK(c, hipMemcpyAsync(const_cast<double*>(A.pw), pw.data(), sizeof(double) * pw.size(),
                               hipMemcpyHostToDevice, c->stream));
      if (mp) {
        pw32.assign(pw.begin(), pw.end());
        HIPCHK(c, hipMemcpyAsync(const_cast<float*>(c->ad32[l].pw), pw32.data(), sizeof(float) * pw32.size(),
                                 hipMemcpyHostToDevice, c->stream));
      }
    }
    std::vector<float> dg32;
    if (mp && !A.fem) {
      dg32.assign(H.dg.begin(), H.dg.end());
      HIPCHK(c, hipMemcpyAsync(const_cast<float*>(c->ad32[l].dg), dg32.data(), sizeof(float) * dg32.size(),
                               hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));   // host vectors go out of scope
  }
  for (int l = c->lmin; l <= L; ++l) {
    HIPCHK(c, launch_ad_setup<double>(d, c->ad[l], c->stream));
    if (mp) HIPCHK(c, launch_ad_setup<float>(d, c->ad32[l], c->stream));
  }
  return ADAFAC_OK;
}

// Composite FE function at every vertex of the finest lattice (host, from the level boxes).
int adaptive_finest(adafac_ctx* c, double* out) {
  const int d = c->dim, L = c->L, lmin = c->lmin;
  int rc = flush(c);
  if (rc) return rc;
  std::vector<double> cur, up;
  int ncur = 0;
  for (int l = lmin; l <= L; ++l) {
    const AdaptHostLevel& H = c->at.lev[l];
    const AdaptLevel& A = c->ad[l];
    std::vector<double> box(H.nverts());
    HIPCHK(c, hipMemcpyAsync(box.data(), A.u, sizeof(double) * box.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int n = ipow3(l), nv = n + 1;
    const size_t full = d == 2 ? size_t(nv) * nv : size_t(nv) * nv * nv;
    up.assign(full, 0.0);
    if (l > lmin) {
      // d-linear interpolation of the coarser level's composite function
      for (size_t i = 0; i < full; ++i) {
        const int x = int(i % nv), y = int((i / nv) % nv), z = d == 3 ? int(i / (size_t(nv) * nv)) : 0;
        const int cx = std::min(x / 3, ncur - 1), cy = std::min(y / 3, ncur - 1), cz = d == 3 ? std::min(z / 3, ncur - 1) : 0;
        const int sx = x - 3 * cx, sy = y - 3 * cy, sz = z - 3 * cz;
        double acc = 0.0;
        for (int e = 0; e < (1 << d); ++e) {
          const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
          double w = (ex ? sx : 3 - sx) / 3.0 * (ey ? sy : 3 - sy) / 3.0;
          if (d == 3) w *= (ez ? sz : 3 - sz) / 3.0;
          if (w == 0.0) continue;
          const size_t k = (size_t(cz + ez) * (ncur + 1) + (cy + ey)) * (ncur + 1) + (cx + ex);
          acc += w * cur[d == 2 ? size_t(cy + ey) * (ncur + 1) + (cx + ex) : k];
        }
        up[i] = acc;
      }
    }
    for (int z = 0; z < A.mz; ++z)
      for (int y = 0; y < A.my; ++y)
        for (int x = 0; x < A.mx; ++x) {
          const size_t i = (size_t(z) * A.my + y) * A.mx + x;
          if (!(H.vcls[i] & (kDof | kHang))) {
            // with Dirichlet data, the boundary vertices of existing cells hold it
            if (c->gdir.empty()) continue;
            const int gx = A.ox + x, gy = A.oy + y, gz = d == 3 ? A.oz + z : 1;
            const bool bd = gx == 0 || gx == n || gy == 0 || gy == n || (d == 3 && (gz == 0 || gz == n));
            if (!bd || !vertex_of_cell(H, d, x, y, z)) continue;
          }
          const size_t g = d == 2 ? size_t(A.oy + y) * nv + (A.ox + x)
                                  : (size_t(A.oz + z) * nv + (A.oy + y)) * nv + (A.ox + x);
          up[g] = box[i];
        }
    cur.swap(up);
    ncur = n;
  }
  std::memcpy(out, cur.data(), sizeof(double) * cur.size());
  return ADAFAC_OK;
}

// Nodal values at every dof of every level from values on the finest lattice.
int adaptive_set(adafac_ctx* c, const double* u) {
  const int d = c->dim, L = c->L;
  const int nL = ipow3(L) + 1;
  for (int l = c->lmin; l <= L; ++l) {
    const AdaptHostLevel& H = c->at.lev[l];
    const AdaptLevel& A = c->ad[l];
    const int s = ipow3(L - l);
    std::vector<double> box(H.nverts(), 0.0);
    for (int z = 0; z < A.mz; ++z)
      for (int y = 0; y < A.my; ++y)
        for (int x = 0; x < A.mx; ++x) {
          const size_t i = (size_t(z) * A.my + y) * A.mx + x;
          if (!(H.vcls[i] & kDof)) continue;
          const size_t gx = size_t(A.ox + x) * s, gy = size_t(A.oy + y) * s, gz = d == 3 ? size_t(A.oz + z) * s : 0;
          box[i] = u[(gz * nL + gy) * nL + gx];
        }
    fill_boundary(c, l, box);
    HIPCHK(c, hipMemcpyAsync(A.u, box.data(), sizeof(double) * box.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  c->e_pending = false;
  return adapt_hang(c);
}

}  // namespace

namespace adafac {

template <typename T>
static void describe_hier(const adafac_ctx* c, const Hier<T>& H, BatchHier<T>& B) {
  for (int l = 0; l <= kMaxLevel; ++l) B.v[l] = H.v[l];
  B.ufine[0] = H.ufine[H.cur];
  B.ufine[1] = H.ufine[1 - H.cur];
  B.bfine = H.bfine;
  B.rfine = H.rfine;
  B.rts = H.rts;
  (void)c;
}

// Device description of a bound context for the batched kernel.  Its iterate is taken as
// ufine[0] (FP64 form) and nothing may be pending.
int batch_describe(void* vc, BatchReq* out) {
  adafac_ctx* c = static_cast<adafac_ctx*>(vc);
  if (!c || !out || !c->bound) return ADAFAC_ESTATE;
  if (c->h64.pending || c->h32.pending || c->e_pending) return ADAFAC_ESTATE;
  *out = BatchReq{};
  out->dim = c->dim;
  out->L = c->L;
  out->lmin = c->lmin;
  out->damping = c->opts.damping;
  out->precision = c->opts.precision;
  out->inner_k = c->opts.inner_k;
  out->omega = c->opts.omega;
  out->omega_t = c->opts.omega_tilde;
  out->omega_hat = c->opts.omega_hat;
  describe_hier(c, c->h64, out->h64);
  if (mixed(c)) {
    describe_hier(c, c->h32, out->h32);
    out->h32.ufine[0] = c->h32.ufine[0];
    out->h32.ufine[1] = c->h32.ufine[1];
    out->ezero = c->ezero;
  }
  out->partials = c->partials;
  // the conditions of run_cycle's single-pass form, without the single-workgroup levels: under
  // adAFAC-PI the prolongation into level L-1 is a phase of its own when L-1 > l_min
  const int L = c->L;
  out->fusable = c->opts.fused && L > c->lmin && c->opts.rtilde != ADAFAC_RTILDE_OPERATOR && fused_ok(c) &&
                 (c->opts.damping != ADAFAC_DAMP_PI || L - 1 > c->lmin) && fine_sweep_nparts(c->dim, ipow3(L)) > 0;
  return ADAFAC_OK;
}

// Norms (l2h, linf) of cycles c0 .. c0+n-1 into out[2n], in one or two copies and one
// synchronisation (the server reads a lane's whole chunk at once).
int residual_range(void* vc, int c0, int n, double* out) {
  adafac_ctx* c = static_cast<adafac_ctx*>(vc);
  if (!c || !c->bound) return ADAFAC_ESTATE;
  if (n <= 0) return ADAFAC_OK;
  if (c0 < 0 || c0 + n > c->ncyc || c->ncyc - c0 > kMaxHist || !out) return ADAFAC_EINVAL;
  const int i0 = c0 % kMaxHist, first = std::min(n, kMaxHist - i0);
  HIPCHK(c, hipMemcpyAsync(out, c->norms + 2 * i0, sizeof(double) * 2 * first, hipMemcpyDeviceToHost, c->stream));
  if (first < n)
    HIPCHK(c, hipMemcpyAsync(out + 2 * first, c->norms, sizeof(double) * 2 * (n - first), hipMemcpyDeviceToHost,
                             c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return ADAFAC_OK;
}

// After batched cycles: ufine[cur] of the description holds the current FP64 iterate (also
// under FP32_REFINED, whose one-pass 3D defect alternates the two buffers); pending:
// (FP64 form) the last cycle swept the finest level and left P S_{L-1} to be added.
int batch_adopt(void* vc, int cur, int pending) {
  adafac_ctx* c = static_cast<adafac_ctx*>(vc);
  if (!c || !c->bound) return ADAFAC_ESTATE;
  if (cur == 1) c->h64.cur = 1 - c->h64.cur;
  c->h64.pending = c->h32.pending = c->e_pending = false;
  if (!mixed(c) && pending) c->h64.pending = true;
  return ADAFAC_OK;
}

}  // namespace adafac

extern "C" {

void adafac_default_opts(adafac_opts* o) {
  if (!o) return;
  o->transfer = ADAFAC_TRANSFER_DLINEAR;
  o->damping = ADAFAC_DAMP_JAC;
  o->rtilde = ADAFAC_RTILDE_CONST_EPS1;
  o->precision = ADAFAC_PREC_FP64;
  o->inner_k = 4;
  o->fused = 1;
  o->omega = 0.6;
  o->omega_tilde = 0.6;
  o->omega_hat = 0.5;
}

int adafac_create(adafac_ctx** out, int dim, int l_min, int l_max) {
  if (!out) return ADAFAC_EINVAL;
  *out = nullptr;
  if (dim != 2 && dim != 3) return ADAFAC_EINVAL;
  if (l_min < 1 || l_min > l_max) return ADAFAC_EINVAL;
  if ((dim == 2 && l_max > 9) || (dim == 3 && l_max > 6)) return ADAFAC_EINVAL;
  adafac_ctx* c = new (std::nothrow) adafac_ctx();
  if (!c) return ADAFAC_ENOMEM;
  c->dim = dim;
  c->lmin = l_min;
  c->L = l_max;
  c->eps.assign(1, 1.0);
  c->nb = 1;
  adafac_default_opts(&c->opts);
  *out = c;
  return ADAFAC_OK;
}

int adafac_set_coefficient_blocks(adafac_ctx* c, int blocks_per_axis, const double* eps) {
  if (!c) return ADAFAC_EINVAL;
  if (!eps || blocks_per_axis < 1) return fail(c, ADAFAC_EINVAL, "eps: null or blocks_per_axis < 1");
  int k = 0, b = 1;
  while (b < blocks_per_axis) { b *= 3; ++k; }
  if (b != blocks_per_axis || k > c->L) return fail(c, ADAFAC_EINVAL, "blocks_per_axis must be 3^k, k <= l_max");
  size_t n = c->dim == 2 ? size_t(b) * b : size_t(b) * b * b;
  for (size_t i = 0; i < n; ++i)
    if (!(eps[i] > 0.0) || !std::isfinite(eps[i])) return fail(c, ADAFAC_EINVAL, "eps must be finite and > 0");
  c->eps.assign(eps, eps + n);
  c->nb = b;
  c->built = c->bound = false;
  return ADAFAC_OK;
}

int adafac_set_rhs_lattice(adafac_ctx* c, const double* f, size_t n) {
  if (!c) return ADAFAC_EINVAL;
  if (!f || n != nverts_of(c->dim, c->L)) return fail(c, ADAFAC_EINVAL, "f: wrong size");
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(f[i])) return fail(c, ADAFAC_EINVAL, "f: non-finite value");
  c->f.assign(f, f + n);
  c->src_gauss = 0;
  c->src_fn = nullptr;
  c->bound = false;
  return ADAFAC_OK;
}

int adafac_set_rhs_gaussian(adafac_ctx* c, const double* centre, double sigma, double amplitude) {
  if (!c) return ADAFAC_EINVAL;
  if (!centre || !(sigma > 0.0) || !std::isfinite(sigma) || !std::isfinite(amplitude))
    return fail(c, ADAFAC_EINVAL, "bad Gaussian source");
  for (int a = 0; a < c->dim; ++a) {
    if (!std::isfinite(centre[a])) return fail(c, ADAFAC_EINVAL, "bad Gaussian centre");
    c->src_c[a] = centre[a];
  }
  c->src_sigma = sigma;
  c->src_amp = amplitude;
  c->src_gauss = 1;
  c->src_fn = nullptr;
  c->f.clear();
  c->bound = false;
  return ADAFAC_OK;
}

int adafac_build_operators(adafac_ctx* c, const adafac_opts* opts) {
  if (!c) return ADAFAC_EINVAL;
  adafac_opts o;
  adafac_default_opts(&o);
  if (opts) o = *opts;
  if (o.transfer != ADAFAC_TRANSFER_DLINEAR && o.transfer != ADAFAC_TRANSFER_BOXMG)
    return fail(c, ADAFAC_EINVAL, "unknown transfer");
  if (o.damping < ADAFAC_DAMP_JAC || o.damping > ADAFAC_DAMP_EXP) return fail(c, ADAFAC_EINVAL, "unknown damping");
  if (o.rtilde != ADAFAC_RTILDE_CONST_EPS1 && o.rtilde != ADAFAC_RTILDE_OPERATOR)
    return fail(c, ADAFAC_EINVAL, "unknown R~ form");
  if (o.precision != ADAFAC_PREC_FP64 && o.precision != ADAFAC_PREC_FP32_REFINED)
    return fail(c, ADAFAC_EINVAL, "unknown precision form");
  if (!(o.omega > 0.0) || !(o.omega_tilde >= 0.0) || !(o.omega_hat > 0.0) || o.inner_k < 1)
    return fail(c, ADAFAC_EINVAL, "bad damping parameters");
  c->opts = o;
  c->ops = HostOps{};
  c->ops.dim = c->dim;
  c->ops.lmin = c->lmin;
  c->ops.L = c->L;
  c->ops.nb = c->nb;
  c->ops.k = 0;
  for (int b = 1; b < c->nb; b *= 3) c->ops.k++;
  c->ops.eps = c->eps;
  c->adaptive = !c->refine.empty() || c->ball_r > 0.0;
  if (c->adaptive) {
    int rc = build_adaptive(c);
    if (rc) return rc;
    c->built = true;
    c->bound = false;
    c->ws_need = layout(c, nullptr);
    return ADAFAC_OK;
  }
  std::string m = build_host_ops(c->ops, o.transfer == ADAFAC_TRANSFER_BOXMG, o.omega,
                                 o.rtilde == ADAFAC_RTILDE_OPERATOR && o.damping == ADAFAC_DAMP_JAC);
  if (!m.empty()) return fail(c, ADAFAC_EINVAL, m);
  c->built = true;
  c->bound = false;
  c->ws_need = layout(c, nullptr);
  return ADAFAC_OK;
}

int adafac_workspace_bytes(const adafac_ctx* c, size_t* bytes) {
  if (!c || !bytes) return ADAFAC_EINVAL;
  if (!c->built) return ADAFAC_ESTATE;
  *bytes = c->ws_need;
  return ADAFAC_OK;
}

}  // extern "C"

namespace adafac {

// Binds c to the device memory ws (bytes >= ws_need, 256-byte aligned) and the stream, uploads
// the operators and the load and sets iterate 0.  clear_by_kernel: zero the workspace with a fill
// kernel instead of a memset node (the library's static workspace, for callers that capture).
int bind_workspace(adafac_ctx* c, void* ws, size_t bytes, void* stream, bool clear_by_kernel) {
  if (!c) return ADAFAC_EINVAL;
  if (!c->built) return fail(c, ADAFAC_ESTATE, "build_operators first");
  if (c->f.empty() && !c->src_gauss && !c->src_fn) return fail(c, ADAFAC_ESTATE, "set the right-hand side first");
  size_t need = c->ws_need;
  if (!ws || bytes < need) return fail(c, ADAFAC_ENOMEM, "workspace too small: need " + std::to_string(need));
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(c, ADAFAC_EINVAL, "workspace not 256-byte aligned");
  c->bound = false;
  c->ws = static_cast<char*>(ws);
  c->ws_bytes = bytes;
  c->stream = static_cast<hipStream_t>(stream);
  layout(c, c->ws);
  const int d = c->dim;
  if (clear_by_kernel)
    HIPCHK(c, launch_zero_fill(c->ws, need, c->stream));
  else
    HIPCHK(c, hipMemsetAsync(c->ws, 0, need, c->stream));
  if (c->adaptive) {
    int rc = bind_adaptive(c);
    if (rc) return rc;
    c->e_pending = false;
    c->ncyc = 0;
    c->r0 = -1.0;
    c->bound = true;
    return ADAFAC_OK;
  }
  int rc = upload_ops<double>(c, c->h64, !mixed(c));
  if (!rc && mixed(c)) rc = upload_ops<float>(c, c->h32, true);
  if (rc) return rc;
  // load vector with lumped mass: h^d f on interior vertices of the uniform finest level
  const HostLevel& fl = c->ops.lev[c->L];
  std::vector<double> b(fl.nverts, 0.0);
  const double hd = std::pow(fl.h, d);
  const int nv = fl.nv;
  const int z_lo = d == 3 ? 1 : 0, z_hi = d == 3 ? nv - 1 : 1;
  auto ranges = [&](size_t n, auto&& f) { if (c->src_fn) f(size_t(0), n); else parallel_ranges(n, f); };
  ranges(size_t(z_hi - z_lo), [&](size_t q0, size_t q1) {
    for (int z = z_lo + int(q0); z < z_lo + int(q1); ++z)
      for (int y = 1; y < nv - 1; ++y) {
        const size_t row = (size_t(z) * nv + y) * nv;
        for (int x = 1; x < nv - 1; ++x) b[row + x] = hd * source_at(c, x, y, z);
      }
  });
  HIPCHK(c, hipMemcpyAsync(c->h64.bfine, b.data(), sizeof(double) * b.size(), hipMemcpyHostToDevice, c->stream));
  if (!c->gdir.empty()) {
    // Dirichlet data: the boundary entries of both FP64 iterate buffers (no kernel writes them;
    // every residual reads them)
    HIPCHK(c, hipMemcpyAsync(c->h64.ufine[0], c->gdir.data(), sizeof(double) * c->gdir.size(), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->h64.ufine[1], c->gdir.data(), sizeof(double) * c->gdir.size(), hipMemcpyHostToDevice,
                             c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->h64.cur = c->h32.cur = 0;
  c->h64.pending = c->h32.pending = c->e_pending = false;
  c->ncyc = 0;
  c->r0 = -1.0;
  c->bound = true;
  return ADAFAC_OK;
}

const char* ctx_workspace(const adafac_ctx* c) { return c && c->bound ? c->ws : nullptr; }

void ctx_unbind(adafac_ctx* c, const char* why) {
  if (!c) return;
  c->bound = false;
  c->err = why;
}

int ctx_fail(adafac_ctx* c, int code, const char* msg) { return fail(c, code, msg); }

}  // namespace adafac

extern "C" {

int adafac_bind(adafac_ctx* c, void* ws, size_t bytes, void* stream) {
  if (c) static_ws_forget(c);
  return bind_workspace(c, ws, bytes, stream, false);
}

int adafac_cycle(adafac_ctx* c, int ncycles) {
  if (!c) return ADAFAC_EINVAL;
  if (!ready(c)) return fail(c, ADAFAC_ESTATE, "bind first");
  if (ncycles < 0) return fail(c, ADAFAC_EINVAL, "ncycles < 0");
  for (int i = 0; i < ncycles; ++i) {
    int rc = run_step(c);
    if (rc) return rc;
  }
  return ADAFAC_OK;
}

int adafac_cycles_run(const adafac_ctx* c) { return c ? c->ncyc : 0; }

int adafac_residual(adafac_ctx* c, int cycle, double* l2h, double* linf) {
  if (!c) return ADAFAC_EINVAL;
  if (!ready(c)) return fail(c, ADAFAC_ESTATE, "bind first");
  if (cycle < 0 || cycle >= c->ncyc || c->ncyc - cycle > kMaxHist)
    return fail(c, ADAFAC_EINVAL, "cycle not run (or no longer kept)");
  double nrm[2];
  HIPCHK(c, hipMemcpyAsync(nrm, c->norms + 2 * (cycle % kMaxHist), sizeof(nrm), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (l2h) *l2h = nrm[0];
  if (linf) *linf = nrm[1];
  return ADAFAC_OK;
}

// FP64 cycles on a uniform hierarchy, launched in batches without a host wait: the stopping rule
// is applied on the device where each cycle's norms are formed, and the launches of the cycles
// after the one that met it do nothing (Gate).  After each batch the host reads how many cycles
// ran and takes back its per-cycle bookkeeping of the skipped ones (iterate buffer, swapped S
// buffers).  The iterates are those of one cycle per host check.  The first batch has
// kSolveBatch cycles; the next ones as many as the contraction of the last cycles predicts until
// the tolerance (at most kSolveBatchMax), so that few batches end and few launches are skipped.
constexpr int kSolveBatch = 8, kSolveBatchMax = 64;

// cycles still needed after the last one of the history (norms of cycles n - k .. n - 1 in the ring)
int predict_cycles(const adafac_ctx* c, const double* nrm, int k, double rel_tol) {
  if (k < 2 || !(c->r0 > 0.0)) return kSolveBatch;
  const int j = std::min(k - 1, 4);
  const double last = nrm[2 * (k - 1)], prev = nrm[2 * (k - 1 - j)];
  if (!(last > 0.0) || !(prev > last)) return kSolveBatch;
  const double rho = std::pow(last / prev, 1.0 / j);
  const double need = std::log(rel_tol * c->r0 / last) / std::log(rho);
  if (!std::isfinite(need)) return kSolveBatch;
  return std::max(1, std::min(kSolveBatchMax, int(std::ceil(need))));
}

// Can adafac_solve pipeline this context?  FP64 on uniform hierarchies and on adaptive trees, and
// the one-pass 3D FP32_REFINED form (an outer step and its inner cycles per batch entry);
// ADAFAC_SOLVE_HOST_CHECK=1 forces the check on the host after every step (the tests compare both).
bool solve_pipelines(const adafac_ctx* c) {
  if (const char* e = std::getenv("ADAFAC_SOLVE_HOST_CHECK"))
    if (std::atoi(e) != 0) return false;
  if (c->adaptive) return !mixed(c);
  return !mixed(c) || (c->dim == 3 && c->opts.fused && fused_ok(c));
}

int solve_pipelined(adafac_ctx* c, double rel_tol, int max_cycles, int* done_out) {
  Hier<double>& D = c->h64;
  Hier<float>& H = c->h32;
  const bool mp = mixed(c);
  const int k = c->opts.inner_k;
  static const unsigned long long never = ~0ull;
  int done = 0, rc = ADAFAC_OK, next = kSolveBatch;
  if (!c->stopseq) return fail(c, ADAFAC_EINVAL, "internal: no stop counter in the workspace layout");
  HIPCHK(c, hipMemcpyAsync(c->stopseq, &never, sizeof(never), hipMemcpyHostToDevice, c->stream));
  while (done < max_cycles) {
    const int n0 = c->ncyc, batch = std::min({next, max_cycles - done, kMaxHist});
    for (int b = 0; b < batch; ++b) {
      const StopRule rule{c->stopseq, static_cast<unsigned long long>(c->ncyc), rel_tol, c->norm0, c->ncyc == 0, 1};
      if ((rc = run_outer(c, &rule))) break;
      if (mp) {
        // the inner solve of step n runs unless step n met the rule: gated as step n + 1
        const StopRule g{c->stopseq, static_cast<unsigned long long>(c->ncyc), 0.0, nullptr, 0, 0};
        if ((rc = run_inner(c, &g))) break;
      }
    }
    if (rc) break;
    unsigned long long stop = never;
    HIPCHK(c, hipMemcpyAsync(&stop, c->stopseq, sizeof(stop), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const bool stopped = stop != never;
    const int ran = stopped ? int(stop - static_cast<unsigned long long>(n0)) : batch;
    if (ran < 1 || ran > batch) return fail(c, ADAFAC_EINVAL, "internal: stop counter out of the batch");
    // take back the host bookkeeping of what the device skipped (an adaptive cycle keeps none)
    if (!c->adaptive && !mp) {
      if ((batch - ran) & 1) {
        D.cur = 1 - D.cur;
        for (int l = D.swap_lo; l < D.swap_hi; ++l) std::swap(D.v[l].S, D.Salt[l]);
      }
    } else if (!c->adaptive && stopped) {
      if ((batch - ran) & 1) D.cur = 1 - D.cur;                 // outer steps: one buffer flip each
      if (((batch - (ran - 1)) * k) & 1) {                      // inner cycles: one flip and swap each
        H.cur = 1 - H.cur;
        for (int l = H.swap_lo; l < H.swap_hi; ++l) std::swap(H.v[l].S, H.Salt[l]);
      }
      H.pending = false;                                        // the last step ran its outer part only
      c->e_pending = false;
    }
    c->ncyc = n0 + ran;
    done += ran;
    if (c->r0 < 0) {
      HIPCHK(c, hipMemcpyAsync(&c->r0, c->norm0, sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if (stopped) {
      double l2 = 0, li = 0;
      if ((rc = adafac_residual(c, c->ncyc - 1, &l2, &li))) break;
      if (!std::isfinite(l2) || l2 > 1e3 * c->r0) rc = fail(c, ADAFAC_EDIVERGED, "residual diverged");
      break;
    }
    // the norms of the batch's steps (consecutive slots of the ring, or two pieces)
    std::vector<double> nrm(2 * size_t(ran));
    const int s0 = n0 % kMaxHist, k1 = std::min(ran, kMaxHist - s0);
    HIPCHK(c, hipMemcpyAsync(nrm.data(), c->norms + 2 * s0, 2 * sizeof(double) * k1, hipMemcpyDeviceToHost,
                             c->stream));
    if (k1 < ran)
      HIPCHK(c, hipMemcpyAsync(&nrm[2 * size_t(k1)], c->norms, 2 * sizeof(double) * (ran - k1),
                               hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    next = predict_cycles(c, nrm.data(), ran, rel_tol);
  }
  *done_out = done;
  return rc;
}

int adafac_solve(adafac_ctx* c, double rel_tol, int max_cycles, int* cycles_done) {
  if (!c) return ADAFAC_EINVAL;
  if (!ready(c)) return fail(c, ADAFAC_ESTATE, "bind first");
  if (!(rel_tol >= 0.0) || max_cycles < 0) return fail(c, ADAFAC_EINVAL, "bad tolerance or cycle cap");
  int done = 0, rc = ADAFAC_OK;
  if (solve_pipelines(c)) {
    rc = solve_pipelined(c, rel_tol, max_cycles, &done);
    if (cycles_done) *cycles_done = done;
    int frc = flush(c);
    if (!rc) rc = frc;
    if (!rc) HIPCHK(c, hipStreamSynchronize(c->stream));
    return rc;
  }
  for (; done < max_cycles; ++done) {
    // norms of iterate ncyc (FP64 cycle or FP64 defect of the outer iterate)
    if ((rc = run_outer(c))) break;
    double l2 = 0, li = 0;
    if ((rc = adafac_residual(c, c->ncyc - 1, &l2, &li))) break;
    if (c->r0 < 0) {
      HIPCHK(c, hipMemcpyAsync(&c->r0, c->norm0, sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if (!std::isfinite(l2) || l2 > 1e3 * c->r0) {
      ++done;
      rc = fail(c, ADAFAC_EDIVERGED, "residual diverged");
      break;
    }
    if (c->r0 == 0.0 || l2 / c->r0 <= rel_tol) {
      // FP64: the cycle that measured iterate n also produced n+1; FP32_REFINED: the outer
      // iterate itself met the tolerance and no inner solve follows
      ++done;
      break;
    }
    if (mixed(c) && (rc = run_inner(c))) break;
  }
  if (cycles_done) *cycles_done = done;
  int frc = flush(c);
  if (!rc) rc = frc;
  if (!rc) HIPCHK(c, hipStreamSynchronize(c->stream));
  return rc;
}

int adafac_get_solution(adafac_ctx* c, double* u, size_t n) {
  if (!c) return ADAFAC_EINVAL;
  if (!ready(c)) return fail(c, ADAFAC_ESTATE, "bind first");
  if (!u || n != nverts_of(c->dim, c->L)) return fail(c, ADAFAC_EINVAL, "u: wrong size");
  if (c->adaptive) return adaptive_finest(c, u);
  int rc = flush(c);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(u, c->h64.ufine[c->h64.cur], sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return ADAFAC_OK;
}

int adafac_set_solution(adafac_ctx* c, const double* u, size_t n) {
  if (!c) return ADAFAC_EINVAL;
  if (!ready(c)) return fail(c, ADAFAC_ESTATE, "bind first");
  if (!u || n != nverts_of(c->dim, c->L)) return fail(c, ADAFAC_EINVAL, "u: wrong size");
  const int nv = ipow3(c->L) + 1;
  std::vector<double> v(u, u + n);
  for (size_t i = 0; i < n; ++i) {
    size_t t = i;
    for (int a = 0; a < c->dim; ++a) {
      int x = int(t % nv);
      t /= nv;
      if (x == 0 || x == nv - 1) v[i] = c->gdir.empty() ? 0.0 : c->gdir[i];
    }
    if (!std::isfinite(v[i])) return fail(c, ADAFAC_EINVAL, "u: non-finite value");
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->adaptive) {
    int rc = adaptive_set(c, v.data());
    if (rc) return rc;
    c->ncyc = 0;
    c->r0 = -1.0;
    return ADAFAC_OK;
  }
  HIPCHK(c, hipMemcpyAsync(c->h64.ufine[c->h64.cur], v.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->h64.pending = c->h32.pending = c->e_pending = false;
  c->ncyc = 0;
  c->r0 = -1.0;
  return ADAFAC_OK;
}

int adafac_get_level(adafac_ctx* c, int level, int which, double* out, size_t n) {
  if (!c) return ADAFAC_EINVAL;
  if (!ready(c)) return fail(c, ADAFAC_ESTATE, "bind first");
  if (c->adaptive) {
    // the level's box arrays on the full level lattice, zero outside the box
    if (level < c->lmin || level > c->L) return fail(c, ADAFAC_EINVAL, "level out of range");
    if (!out || n != nverts_of(c->dim, level)) return fail(c, ADAFAC_EINVAL, "out: wrong size");
    const AdaptLevel& A = c->ad[level];
    const double* src = nullptr;
    switch (which) {
      case 0: src = A.u; break;
      case 1: src = A.bb; break;
      case 4: src = A.S; break;
      default: return fail(c, ADAFAC_EINVAL, "which: 0 (u), 1 (b), 4 (S) on adaptive trees");
    }
    if (which == 4 && level == c->L)
      return fail(c, ADAFAC_EINVAL, "S is not kept on the finest level of a tree (it feeds no finer level)");
    if (mixed(c) && which != 0) return fail(c, ADAFAC_ESTATE, "FP32_REFINED keeps only u in FP64 on a tree");
    if (which == 0) {
      int rc = flush(c);
      if (rc) return rc;
    }
    const AdaptHostLevel& H = c->at.lev[level];
    std::vector<double> box(H.nverts());
    HIPCHK(c, hipMemcpyAsync(box.data(), src, sizeof(double) * box.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int nv = ipow3(level) + 1;
    std::fill(out, out + n, 0.0);
    for (int z = 0; z < A.mz; ++z)
      for (int y = 0; y < A.my; ++y)
        for (int x = 0; x < A.mx; ++x) {
          const size_t g = c->dim == 2 ? size_t(A.oy + y) * nv + (A.ox + x)
                                       : (size_t(A.oz + z) * nv + (A.oy + y)) * nv + (A.ox + x);
          out[g] = box[(size_t(z) * A.my + y) * A.mx + x];
        }
    return ADAFAC_OK;
  }
  if (level < c->lmin || level >= c->L) return fail(c, ADAFAC_EINVAL, "level out of range");
  if (!out || n != nverts_of(c->dim, level)) return fail(c, ADAFAC_EINVAL, "out: wrong size");
  if (mixed(c)) return fail(c, ADAFAC_ESTATE, "level arrays are kept in the FP64 form only");
  const LevelView<double>& v = c->h64.v[level];
  const double* src = nullptr;
  switch (which) {
    case 0: src = v.u; break;
    case 1: src = v.bf; break;
    case 2: src = v.bt; break;
    case 3: src = v.r; break;
    case 4: src = v.S; break;
    default: return fail(c, ADAFAC_EINVAL, "which out of range");
  }
  HIPCHK(c, hipMemcpyAsync(out, src, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return ADAFAC_OK;
}

int adafac_host_operator(const adafac_ctx* cc, int level, int which, double* out, size_t n) {
  adafac_ctx* c = const_cast<adafac_ctx*>(cc);
  if (!c || !out) return ADAFAC_EINVAL;
  if (!c->built) return fail(c, ADAFAC_ESTATE, "build_operators first");
  const int d = c->dim, ns = d == 2 ? 9 : 27;
  if (c->adaptive && which != 3) return fail(c, ADAFAC_EUNSUPPORTED, "host operators of uniform hierarchies only");
  if (which == 3) {
    if (n != c->ops.rtilde.size()) return fail(c, ADAFAC_EINVAL, "out: wrong size");
    std::memcpy(out, c->ops.rtilde.data(), sizeof(double) * n);
    return ADAFAC_OK;
  }
  if (level < c->lmin || level > c->L) return fail(c, ADAFAC_EINVAL, "level out of range");
  const HostLevel& hl = c->ops.lev[level];
  if (which == 4) {
    if (hl.rtw.empty()) return fail(c, ADAFAC_ESTATE, "no OPERATOR R~ on this level");
    if (n != hl.rtw.size()) return fail(c, ADAFAC_EINVAL, "out: wrong size");
    std::memcpy(out, hl.rtw.data(), sizeof(double) * n);
    return ADAFAC_OK;
  }
  const size_t nv = hl.nverts;
  auto coords = [&](size_t i, int* v) { for (int a = 0; a < d; ++a) { v[a] = int(i % hl.nv); i /= hl.nv; } };
  auto interior = [&](const int* v) { for (int a = 0; a < d; ++a) if (v[a] <= 0 || v[a] >= hl.nv - 1) return false; return true; };
  if (which == 0) {
    if (n != nv * ns) return fail(c, ADAFAC_EINVAL, "out: wrong size");
    if (!hl.st.empty()) { std::memcpy(out, hl.st.data(), sizeof(double) * n); return ADAFAC_OK; }
    for (size_t i = 0; i < nv; ++i) {
      int v[3] = {0, 0, 0};
      coords(i, v);
      for (int t = 0; t < ns; ++t) {
        int o[3] = {t % 3 - 1, (t / 3) % 3 - 1, d == 3 ? t / 9 - 1 : 0}, w[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) w[a] = v[a] + o[a];
        out[i * ns + t] = (interior(v) && interior(w)) ? fem_stencil_entry(c->ops, level, v, o) : 0.0;
      }
    }
    return ADAFAC_OK;
  }
  if (which == 1) {
    if (n != nv) return fail(c, ADAFAC_EINVAL, "out: wrong size");
    if (!hl.dg.empty()) {
      std::memcpy(out, hl.dg.data(), sizeof(double) * n);
      return ADAFAC_OK;
    }
    const int zero[3] = {0, 0, 0};
    for (size_t i = 0; i < nv; ++i) {
      int v[3] = {0, 0, 0};
      coords(i, v);
      out[i] = interior(v) ? fem_stencil_entry(c->ops, level, v, zero) : 0.0;
    }
    return ADAFAC_OK;
  }
  if (which == 2) {
    const size_t ne = size_t(1) << d;
    if (level <= c->lmin || n != nv * ne) return fail(c, ADAFAC_EINVAL, "level or size out of range");
    if (!hl.pw.empty()) { std::memcpy(out, hl.pw.data(), sizeof(double) * n); return ADAFAC_OK; }
    const int nc = hl.n / 3;
    for (size_t i = 0; i < nv; ++i) {
      int v[3] = {0, 0, 0};
      coords(i, v);
      for (size_t e = 0; e < ne; ++e) {
        double w = interior(v) ? 1.0 : 0.0;
        for (int a = 0; a < d; ++a) {
          int cell = std::min(v[a] / 3, nc - 1), s = v[a] - 3 * cell, cv = cell + int((e >> a) & 1);
          w *= ((e >> a) & 1) ? s / 3.0 : (3 - s) / 3.0;
          if (cv <= 0 || cv >= nc) w = 0.0;   // no shape function on a boundary coarse vertex
        }
        out[i * ne + e] = w;
      }
    }
    return ADAFAC_OK;
  }
  return fail(c, ADAFAC_EINVAL, "which out of range");
}

int64_t adafac_dofs_per_cycle(const adafac_ctx* c) {
  if (!c) return 0;
  int64_t s = 0;
  if (c->adaptive && c->built) {
    for (int l = c->lmin; l <= c->L; ++l)
      for (uint8_t v : c->at.lev[l].vcls) s += (v & kDof) ? 1 : 0;
    return s;
  }
  for (int l = c->lmin; l <= c->L; ++l) {
    int64_t m = ipow3(l) - 1;
    s += c->dim == 2 ? m * m : m * m * m;
  }
  return s;
}

int adafac_set_kernel_timing(adafac_ctx* c, int enable) {
  if (!c) return ADAFAC_EINVAL;
  if (c->stream || c->bound) HIPCHK(c, hipStreamSynchronize(c->stream));
  if (enable && c->ev.empty()) {
    c->ev.resize(2 * kTimingPool);
    for (auto& e : c->ev) HIPCHK(c, hipEventCreateWithFlags(&e, ADAFAC_TIMING_EVENT_FLAGS));
  }
  c->timing = enable != 0;
  c->ev_used = 0;
  c->t_acc = 0.0;
  c->t_launches = 0;
  return ADAFAC_OK;
}

int adafac_kernel_time(adafac_ctx* c, double* total_ms, int* launches) {
  if (!c) return ADAFAC_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i + 1 < c->ev_used; i += 2) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
    c->t_acc += ms;
  }
  c->ev_used = 0;
  if (total_ms) *total_ms = c->t_acc;
  if (launches) *launches = c->t_launches;
  return ADAFAC_OK;
}

int adafac_set_solution_coarse(adafac_ctx* c, const double* u, size_t n, int l_src) {
  if (!c) return ADAFAC_EINVAL;
  if (!ready(c)) return fail(c, ADAFAC_ESTATE, "bind first");
  if (l_src < 1 || l_src > c->L) return fail(c, ADAFAC_EINVAL, "l_src must lie in 1..l_max");
  const int d = c->dim;
  if (!u || n != nverts_of(d, l_src)) return fail(c, ADAFAC_EINVAL, "u: wrong size");
  // d-linear interpolation, one level at a time: fine index 3 i + s takes (1 - s/3) u_i + (s/3) u_{i+1}
  std::vector<double> cur(u, u + n), nxt;
  for (int l = l_src; l < c->L; ++l) {
    const int m = ipow3(l), M = 3 * m;   // cells per axis, coarse and fine
    const size_t nc = size_t(m) + 1, nf = size_t(M) + 1;
    nxt.assign(d == 2 ? nf * nf : nf * nf * nf, 0.0);
    const int zf = d == 3 ? M : 0;
    for (int z = 0; z <= zf; ++z)
      for (int y = 0; y <= M; ++y)
        for (int x = 0; x <= M; ++x) {
          const int cx = std::min(x / 3, m - 1), cy = std::min(y / 3, m - 1), cz = d == 3 ? std::min(z / 3, m - 1) : 0;
          const int sx = x - 3 * cx, sy = y - 3 * cy, sz = z - 3 * cz;
          double acc = 0.0;
          for (int e = 0; e < (1 << d); ++e) {
            const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
            double w = (ex ? sx : 3 - sx) / 3.0 * ((ey ? sy : 3 - sy) / 3.0);
            if (d == 3) w *= (ez ? sz : 3 - sz) / 3.0;
            if (w == 0.0) continue;
            acc += w * cur[(size_t(cz + ez) * nc + (cy + ey)) * nc + (cx + ex)];
          }
          nxt[(size_t(z) * nf + y) * nf + x] = acc;
        }
    cur.swap(nxt);
  }
  return adafac_set_solution(c, cur.data(), cur.size());
}

int adafac_amr_mark(adafac_ctx* c, double fraction, int l_uniform, int l_cap, uint8_t* flags, size_t n,
                    int* l_new) {
  if (!c) return ADAFAC_EINVAL;
  if (!ready(c)) return fail(c, ADAFAC_ESTATE, "bind first");
  const int d = c->dim, L = c->L;
  if (!(fraction >= 0.0 && fraction <= 1.0) || l_uniform < c->lmin || l_uniform > L || l_cap < L || l_cap > kMaxLevel ||
      (d == 3 && l_cap > 6))
    return fail(c, ADAFAC_EINVAL, "bad fraction, l_uniform or l_cap");
  if (!c->adaptive && l_uniform != L) return fail(c, ADAFAC_EINVAL, "a uniform tree has l_uniform = l_max");
  if (c->adaptive) {
    // the levels below l_uniform carry no flags: they must be complete and fully refined
    for (int l = c->lmin; l < l_uniform; ++l) {
      const AdaptHostLevel& H = c->at.lev[l];
      const size_t m = size_t(ipow3(l)), full = d == 2 ? m * m : m * m * m;
      bool ok = H.ncells() == full;
      for (size_t i = 0; ok && i < H.refined.size(); ++i) ok = H.exists[i] && H.refined[i];
      if (!ok) return fail(c, ADAFAC_EINVAL, "l_uniform above the current tree's complete levels");
    }
  }
  std::vector<size_t> off(size_t(l_cap) + 1, 0);
  size_t total = 0;
  for (int l = l_uniform; l < l_cap; ++l) {
    off[l] = total;
    const size_t m = size_t(ipow3(l));
    total += d == 2 ? m * m : m * m * m;
  }
  if (!flags || !l_new || n != total) return fail(c, ADAFAC_EINVAL, "flags: wrong size");
  std::fill(flags, flags + n, uint8_t(0));
  auto cell = [&](int l, int x, int y, int z) -> uint8_t& {
    const size_t m = size_t(ipow3(l));
    return flags[off[l] + (size_t(z) * m + y) * m + x];
  };
  int rc = flush(c);
  if (rc) return rc;
  // the current tree's refined cells, and every level's nodal values on the full lattice
  // (dofs, hanging values, boundary data; zero outside the level's cells)
  std::vector<std::vector<double>> u(L + 1);
  std::vector<std::vector<uint8_t>> comp(L + 1), exists(L + 1);
  for (int l = c->lmin; l <= L; ++l) {
    const int m = ipow3(l), nv = m + 1;
    const size_t nvert = d == 2 ? size_t(nv) * nv : size_t(nv) * nv * nv;
    const size_t ncell = d == 2 ? size_t(m) * m : size_t(m) * m * m;
    u[l].assign(nvert, 0.0);
    comp[l].assign(nvert, 0);
    exists[l].assign(ncell, 0);
  }
  if (c->adaptive) {
    for (int l = c->lmin; l <= L; ++l) {
      const AdaptHostLevel& H = c->at.lev[l];
      const AdaptLevel& A = c->ad[l];
      std::vector<double> box(H.nverts());
      HIPCHK(c, hipMemcpyAsync(box.data(), A.u, sizeof(double) * box.size(), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      const int m = ipow3(l), nv = m + 1;
      for (int z = 0; z < (d == 3 ? H.nc[2] + 1 : 1); ++z)
        for (int y = 0; y <= H.nc[1]; ++y)
          for (int x = 0; x <= H.nc[0]; ++x) {
            const size_t i = (size_t(z) * (H.nc[1] + 1) + y) * (H.nc[0] + 1) + x;
            const size_t g = (size_t(d == 3 ? H.lo[2] + z : 0) * nv + (H.lo[1] + y)) * nv + (H.lo[0] + x);
            u[l][g] = box[i];
            comp[l][g] = (H.vcls[i] & kComp) ? 1 : 0;
          }
      for (int z = 0; z < H.nc[2]; ++z)
        for (int y = 0; y < H.nc[1]; ++y)
          for (int x = 0; x < H.nc[0]; ++x) {
            const size_t i = (size_t(z) * H.nc[1] + y) * H.nc[0] + x;
            const size_t g = (size_t(d == 3 ? H.lo[2] + z : 0) * m + (H.lo[1] + y)) * m + (H.lo[0] + x);
            exists[l][g] = H.exists[i];
            if (l >= l_uniform && l < L && H.exists[i] && H.refined[i])
              cell(l, H.lo[0] + x, H.lo[1] + y, d == 3 ? H.lo[2] + z : 0) = 1;
          }
    }
  } else {
    std::vector<double> lat(nverts_of(d, L));
    if ((rc = adafac_get_solution(c, lat.data(), lat.size()))) return rc;
    u[L] = lat;
    const int m = ipow3(L), nv = m + 1;
    std::fill(exists[L].begin(), exists[L].end(), uint8_t(1));
    for (size_t i = 0; i < comp[L].size(); ++i) {
      const int x = int(i % nv), y = int((i / nv) % nv), z = d == 3 ? int(i / (size_t(nv) * nv)) : 1;
      comp[L][i] = x > 0 && x < m && y > 0 && y < m && (d == 2 || (z > 0 && z < m));
    }
  }
  // (i) the finest level's cells with a face on which the Dirichlet data are nonzero at every
  // vertex (the bottom boundary of the Sec. 5 set-ups), while the tree is below l_cap
  if (L < l_cap && !c->gdir.empty()) {
    const int m = ipow3(L), nv = m + 1;
    auto gv = [&](int x, int y, int z) { return c->gdir[(size_t(z) * nv + y) * nv + x]; };
    for (int z = 0; z < (d == 3 ? m : 1); ++z)
      for (int y = 0; y < m; ++y)
        for (int x = 0; x < m; ++x) {
          if (!exists[L][(size_t(z) * m + y) * m + x]) continue;
          const int q[3] = {x, y, z};
          bool mark = false;
          for (int a = 0; a < d && !mark; ++a)
            for (int side = 0; side < 2 && !mark; ++side) {
              // the cell's face at coordinate f along axis a lies on the boundary
              const int f = side ? m : 0;
              if (q[a] + side != f) continue;
              bool all = true;   // the data at the face's 2^(d-1) corners
              for (int e = 0; e < (1 << d) && all; ++e) {
                const int v[3] = {x + (e & 1), y + ((e >> 1) & 1), z + (d == 3 ? (e >> 2) & 1 : 0)};
                if (v[a] == f) all = gv(v[0], v[1], v[2]) != 0.0;
              }
              mark = all;
            }
          if (mark) cell(L, x, y, z) = 1;
        }
  }
  // (ii) the composite dofs carrying the (approximately) `fraction` largest directional second
  // derivatives |d^2 u / dx_i^2| (second differences on the dof's level), found by sorting the
  // values into 1024 equal bins over [0, max] and taking whole bins from the top until they
  // hold that fraction; their 2^d cells are refined unless the level is l_cap
  struct Dof { int l; int x, y, z; double v; };
  std::vector<Dof> dofs;
  for (int l = c->lmin; l <= L; ++l) {
    const int m = ipow3(l), nv = m + 1;
    const double h2 = 1.0 / (double(m) * m);
    for (size_t i = 0; i < comp[l].size(); ++i) {
      if (!comp[l][i]) continue;
      const int x = int(i % nv), y = int((i / nv) % nv), z = d == 3 ? int(i / (size_t(nv) * nv)) : 0;
      const size_t st[3] = {1, size_t(nv), size_t(nv) * nv};
      double v = 0.0;
      for (int a = 0; a < d; ++a)
        v = std::max(v, std::fabs(u[l][i + st[a]] - 2.0 * u[l][i] + u[l][i - st[a]]) / h2);
      dofs.push_back(Dof{l, x, y, z, v});
    }
  }
  if (!dofs.empty() && fraction > 0.0) {
    double vmax = 0.0;
    for (const Dof& q : dofs) vmax = std::max(vmax, q.v);
    constexpr int kBins = 1024;
    std::vector<size_t> cnt(kBins, 0);
    auto bin = [&](double v) { return vmax > 0.0 ? std::min(kBins - 1, int(v / vmax * kBins)) : 0; };
    for (const Dof& q : dofs) ++cnt[bin(q.v)];
    const double want = fraction * double(dofs.size());
    int cut = kBins;
    size_t have = 0;
    while (cut > 0 && double(have) < want) have += cnt[--cut];
    for (const Dof& q : dofs) {
      if (bin(q.v) < cut || q.l >= l_cap) continue;
      for (int e = 0; e < (1 << d); ++e) {
        const int cx = q.x - 1 + (e & 1), cy = q.y - 1 + ((e >> 1) & 1), cz = d == 3 ? q.z - 1 + ((e >> 2) & 1) : 0;
        if (q.l >= l_uniform) cell(q.l, cx, cy, cz) = 1;
      }
    }
  }
  int top = L;
  for (int l = l_uniform; l < l_cap; ++l) {
    const size_t m = size_t(ipow3(l)), nc = d == 2 ? m * m : m * m * m;
    for (size_t i = 0; i < nc; ++i)
      if (flags[off[l] + i]) {
        top = std::max(top, l + 1);
        break;
      }
  }
  *l_new = top;
  return ADAFAC_OK;
}

int adafac_set_refinement(adafac_ctx* c, int level, const uint8_t* flags, size_t ncells) {
  if (!c) return ADAFAC_EINVAL;
  if (level < c->lmin || level >= c->L) return fail(c, ADAFAC_EINVAL, "level must lie in l_min..l_max-1");
  const size_t n = size_t(ipow3(level));
  if (!flags || ncells != (c->dim == 2 ? n * n : n * n * n)) return fail(c, ADAFAC_EINVAL, "flags: wrong size");
  RefineSpec r;
  r.level = level;
  r.flags.assign(flags, flags + ncells);
  for (auto it = c->refine.begin(); it != c->refine.end(); ++it)
    if (it->level == level) {
      c->refine.erase(it);
      break;
    }
  c->refine.push_back(std::move(r));
  c->built = c->bound = false;
  return ADAFAC_OK;
}

int adafac_refine_ball(adafac_ctx* c, const double* centre, double radius, int l_from) {
  if (!c) return ADAFAC_EINVAL;
  if (!centre || !(radius >= 0.0) || !std::isfinite(radius)) return fail(c, ADAFAC_EINVAL, "bad ball");
  if (l_from < c->lmin || l_from >= c->L) return fail(c, ADAFAC_EINVAL, "l_from must lie in l_min..l_max-1");
  for (int a = 0; a < c->dim; ++a) {
    if (!std::isfinite(centre[a])) return fail(c, ADAFAC_EINVAL, "bad ball centre");
    c->ball_c[a] = centre[a];
  }
  c->ball_r = radius;
  c->ball_from = l_from;
  c->built = c->bound = false;
  return ADAFAC_OK;
}

int adafac_regrid_prepare(adafac_ctx* c, const double* centre, double radius, int l_from, const double* f, size_t n,
                          size_t* bytes) {
  if (!c) return ADAFAC_EINVAL;
  if (!ready(c) || !c->adaptive) return fail(c, ADAFAC_ESTATE, "regrid needs a bound adaptive context");
  if (!centre || !(radius > 0.0) || !std::isfinite(radius)) return fail(c, ADAFAC_EINVAL, "bad ball");
  if (l_from < c->lmin || l_from >= c->L) return fail(c, ADAFAC_EINVAL, "l_from must lie in l_min..l_max-1");
  if (c->ops.k > l_from) return fail(c, ADAFAC_EINVAL, "coefficient blocks finer than the first refined level");
  if (f) {
    if (n != nverts_of(c->dim, c->L)) return fail(c, ADAFAC_EINVAL, "f: wrong size");
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(f[i])) return fail(c, ADAFAC_EINVAL, "f: non-finite value");
  } else if (!c->src_gauss && !c->src_fn) {
    return fail(c, ADAFAC_EINVAL, "f: a lattice is needed unless the right-hand side is a Gaussian source or a function");
  }
  double cc[3] = {0, 0, 0};
  for (int a = 0; a < c->dim; ++a) cc[a] = centre[a];
  std::string m = build_adapt_tree(c->at_next, c->dim, c->lmin, c->L, {}, cc, radius, l_from);
  if (!m.empty()) return fail(c, ADAFAC_EINVAL, m);
  for (int l = c->lmin; l <= c->L; ++l)
    if (c->at_next.lev[l].nverts() > size_t(kAdaptMaxBox))
      return fail(c, ADAFAC_EUNSUPPORTED, "a level's bounding box exceeds 2^31 - 1 vertices");
  // the uniform levels below the coefficient blocks are those of the current tree
  for (int l = c->lmin; l < c->ops.k; ++l) c->at_next.lev[l].dg = c->at.lev[l].dg;
  if (f) c->f_next.assign(f, f + n);
  else c->f_next.clear();
  for (int a = 0; a < 3; ++a) c->next_src_c[a] = cc[a];
  c->next_need = layout_adaptive_tree(c, c->at_next, nullptr);
  c->next_ready = true;
  for (int a = 0; a < 3; ++a) c->ball_c[a] = cc[a];
  c->ball_r = radius;
  c->ball_from = l_from;
  c->refine.clear();
  if (bytes) *bytes = c->next_need;
  return ADAFAC_OK;
}

int adafac_regrid(adafac_ctx* c, void* ws, size_t bytes) {
  if (!c) return ADAFAC_EINVAL;
  if (!ready(c) || !c->adaptive || !c->next_ready) return fail(c, ADAFAC_ESTATE, "adafac_regrid_prepare first");
  if (!ws || bytes < c->next_need) return fail(c, ADAFAC_ENOMEM, "workspace too small: need " + std::to_string(c->next_need));
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(c, ADAFAC_EINVAL, "workspace not 256-byte aligned");
  // the old tree: pending correction added, hanging values current, then a view of its levels
  int rc = flush(c);
  if (rc) return rc;
  AdaptTreeView O{};
  O.lmin = c->lmin;
  O.L = c->L;
  for (int l = c->lmin; l <= c->L; ++l) {
    O.lv[l] = c->ad[l];
    O.scale[l] = ipow3(c->L - l);
  }
  double* old_norms = c->norms;
  double* old_norm0 = c->norm0;
  // switch to the new tree and its workspace
  std::swap(c->at, c->at_next);
  if (c->f_next.empty()) {
    // a Gaussian source moves with the ball; a function source stays as it is
    if (c->src_gauss)
      for (int a = 0; a < 3; ++a) c->src_c[a] = c->next_src_c[a];
  } else {
    c->f.swap(c->f_next);
    c->src_gauss = 0;
    c->src_fn = nullptr;
  }
  static_ws_forget(c);
  layout(c, static_cast<char*>(ws));
  HIPCHK(c, hipMemsetAsync(ws, 0, c->next_need, c->stream));
  if ((rc = bind_adaptive(c))) return rc;
  for (int l = c->lmin; l <= c->L; ++l)
    HIPCHK(c, launch_ad_transfer(c->dim, c->ad[l], ipow3(c->L - l), O, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->norms, old_norms, sizeof(double) * 2 * kMaxHist, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->norm0, old_norm0, sizeof(double) * 2, hipMemcpyDeviceToDevice, c->stream));
  if ((rc = adapt_hang(c))) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->ws = static_cast<char*>(ws);
  c->ws_bytes = bytes;
  c->ws_need = c->next_need;
  c->at_next = AdaptHost{};
  c->f_next.clear();
  c->next_ready = false;
  return ADAFAC_OK;
}

int64_t adafac_composite_dofs(const adafac_ctx* c) {
  if (!c || !c->built) return 0;
  if (c->adaptive) return int64_t(c->at.composite);
  const int64_t m = ipow3(c->L) - 1;
  return c->dim == 2 ? m * m : m * m * m;
}

void adafac_destroy(adafac_ctx* c) {
  if (!c) return;
  static_ws_forget(c);
  if (c->bound) (void)hipStreamSynchronize(c->stream);
  for (auto& e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

const char* adafac_last_error(const adafac_ctx* c) { return c ? c->err.c_str() : "null context"; }

int adafac_set_rhs_fn(adafac_ctx* c, double (*f)(const double* x, void* user), void* user) {
  if (!c) return ADAFAC_EINVAL;
  if (!f) return fail(c, ADAFAC_EINVAL, "f: null function");
  c->src_fn = f;
  c->src_user = user;
  c->src_gauss = 0;
  c->f.clear();
  c->bound = false;
  return ADAFAC_OK;
}

int adafac_set_dirichlet_lattice(adafac_ctx* c, const double* g, size_t n) {
  if (!c) return ADAFAC_EINVAL;
  if (!g || n != nverts_of(c->dim, c->L)) return fail(c, ADAFAC_EINVAL, "g: wrong size");
  const int nv = ipow3(c->L) + 1;
  std::vector<double> gd(n, 0.0);
  bool any = false;
  for (size_t i = 0; i < n; ++i) {
    size_t t = i;
    bool bd = false;
    for (int a = 0; a < c->dim; ++a) {
      const int x = int(t % nv);
      t /= nv;
      bd = bd || x == 0 || x == nv - 1;
    }
    if (!bd) continue;
    if (!std::isfinite(g[i])) return fail(c, ADAFAC_EINVAL, "g: non-finite boundary value");
    gd[i] = g[i];
    any = any || g[i] != 0.0;
  }
  if (any) c->gdir.swap(gd);
  else c->gdir.clear();
  return ADAFAC_OK;
}

int adafac_residual_normalised(adafac_ctx* c, int cycle, double* l2h_rel, double* linf_rel) {
  if (!c) return ADAFAC_EINVAL;
  if (!ready(c)) return fail(c, ADAFAC_ESTATE, "bind first");
  if (cycle < 0 || cycle >= c->ncyc || c->ncyc - cycle > kMaxHist)
    return fail(c, ADAFAC_EINVAL, "cycle not run (or no longer kept)");
  double nrm[2], n0[2];
  HIPCHK(c, hipMemcpyAsync(nrm, c->norms + 2 * (cycle % kMaxHist), sizeof(nrm), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(n0, c->norm0, sizeof(n0), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (l2h_rel) *l2h_rel = n0[0] > 0.0 ? nrm[0] / n0[0] : 0.0;
  if (linf_rel) *linf_rel = n0[1] > 0.0 ? nrm[1] / n0[1] : 0.0;
  return ADAFAC_OK;
}

}  // extern "C"

namespace {
// f(level, box-or-lattice index, finest-lattice coordinates) for every composite dof, in the
// composite order: uniform trees the interior finest vertices in lattice order; adaptive trees
// level by level from l_min, each level's composite dofs in the order of its box (x fastest).
template <class F>
void for_composite(const adafac_ctx* c, F&& f) {
  const int d = c->dim, L = c->L;
  if (!c->adaptive) {
    const int nv = ipow3(L) + 1;
    const int zl = d == 3 ? 1 : 0, zh = d == 3 ? nv - 1 : 1;
    for (int z = zl; z < zh; ++z)
      for (int y = 1; y < nv - 1; ++y)
        for (int x = 1; x < nv - 1; ++x) {
          const int g[3] = {x, y, z};
          f(L, (size_t(z) * nv + y) * nv + x, g);
        }
    return;
  }
  for (int l = c->lmin; l <= L; ++l) {
    const AdaptHostLevel& H = c->at.lev[l];
    const int s = ipow3(L - l);
    const int mx = H.nc[0] + 1, my = H.nc[1] + 1, mz = d == 3 ? H.nc[2] + 1 : 1;
    for (int z = 0; z < mz; ++z)
      for (int y = 0; y < my; ++y)
        for (int x = 0; x < mx; ++x) {
          const size_t i = (size_t(z) * my + y) * mx + x;
          if (!(H.vcls[i] & kComp)) continue;
          const int g[3] = {(H.lo[0] + x) * s, (H.lo[1] + y) * s, d == 3 ? (H.lo[2] + z) * s : 0};
          f(l, i, g);
        }
  }
}
}  // namespace

extern "C" {

int adafac_dof_coords(const adafac_ctx* cc, double* xyz, int* level, size_t n) {
  adafac_ctx* c = const_cast<adafac_ctx*>(cc);
  if (!c) return ADAFAC_EINVAL;
  if (!c->built) return fail(c, ADAFAC_ESTATE, "build_operators first");
  if (n != size_t(adafac_composite_dofs(c))) return fail(c, ADAFAC_EINVAL, "n must equal adafac_composite_dofs");
  const double hL = 1.0 / ipow3(c->L);
  const int d = c->dim;
  size_t k = 0;
  for_composite(c, [&](int l, size_t, const int* g) {
    if (xyz)
      for (int a = 0; a < d; ++a) xyz[k * d + a] = g[a] * hL;
    if (level) level[k] = l;
    ++k;
  });
  return ADAFAC_OK;
}

int adafac_get_composite(adafac_ctx* c, double* u, size_t n) {
  if (!c) return ADAFAC_EINVAL;
  if (!ready(c)) return fail(c, ADAFAC_ESTATE, "bind first");
  if (!u || n != size_t(adafac_composite_dofs(c))) return fail(c, ADAFAC_EINVAL, "n must equal adafac_composite_dofs");
  size_t k = 0;
  if (c->adaptive) {
    // the level boxes hold the composite dofs' values
    int rc = flush(c);
    if (rc) return rc;
    std::vector<std::vector<double>> box(c->L + 1);
    for (int l = c->lmin; l <= c->L; ++l) {
      box[l].resize(c->at.lev[l].nverts());
      HIPCHK(c, hipMemcpyAsync(box[l].data(), c->ad[l].u, sizeof(double) * box[l].size(), hipMemcpyDeviceToHost,
                               c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for_composite(c, [&](int l, size_t i, const int*) { u[k++] = box[l][i]; });
    return ADAFAC_OK;
  }
  std::vector<double> lat(nverts_of(c->dim, c->L));
  int rc = adafac_get_solution(c, lat.data(), lat.size());
  if (rc) return rc;
  for_composite(c, [&](int, size_t i, const int*) { u[k++] = lat[i]; });
  return ADAFAC_OK;
}

int adafac_set_composite(adafac_ctx* c, const double* u, size_t n) {
  if (!c) return ADAFAC_EINVAL;
  if (!ready(c)) return fail(c, ADAFAC_ESTATE, "bind first");
  if (!u || n != size_t(adafac_composite_dofs(c))) return fail(c, ADAFAC_EINVAL, "n must equal adafac_composite_dofs");
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(u[k])) return fail(c, ADAFAC_EINVAL, "u: non-finite value");
  size_t k = 0;
  if (c->adaptive) {
    // composite dofs take their values; a dof that is not composite copies the dof at its
    // position one level finer (filled first); hanging values are interpolated on the device
    const int d = c->dim, L = c->L;
    std::vector<std::vector<double>> box(L + 1);
    for (int l = c->lmin; l <= L; ++l) box[l].assign(c->at.lev[l].nverts(), 0.0);
    for_composite(c, [&](int l, size_t i, const int*) { box[l][i] = u[k++]; });
    for (int l = L - 1; l >= c->lmin; --l) {
      const AdaptHostLevel& H = c->at.lev[l];
      const AdaptHostLevel& F = c->at.lev[l + 1];
      const int mx = H.nc[0] + 1, my = H.nc[1] + 1, mz = d == 3 ? H.nc[2] + 1 : 1;
      const int fmx = F.nc[0] + 1, fmy = F.nc[1] + 1;
      for (int z = 0; z < mz; ++z)
        for (int y = 0; y < my; ++y)
          for (int x = 0; x < mx; ++x) {
            const size_t i = (size_t(z) * my + y) * mx + x;
            if ((H.vcls[i] & kDof) && !(H.vcls[i] & kComp)) {
              const int fx = 3 * (H.lo[0] + x) - F.lo[0], fy = 3 * (H.lo[1] + y) - F.lo[1];
              const int fz = d == 3 ? 3 * (H.lo[2] + z) - F.lo[2] : 0;
              box[l][i] = box[l + 1][(size_t(fz) * fmy + fy) * fmx + fx];
            }
          }
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int l = c->lmin; l <= L; ++l) {
      fill_boundary(c, l, box[l]);
      HIPCHK(c, hipMemcpyAsync(c->ad[l].u, box[l].data(), sizeof(double) * box[l].size(), hipMemcpyHostToDevice,
                               c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->e_pending = false;
    int rc = adapt_hang(c);
    if (rc) return rc;
    c->ncyc = 0;
    c->r0 = -1.0;
    return ADAFAC_OK;
  }
  std::vector<double> lat(nverts_of(c->dim, c->L), 0.0);
  for_composite(c, [&](int, size_t i, const int*) { lat[i] = u[k++]; });
  return adafac_set_solution(c, lat.data(), lat.size());
}

int adafac_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (!src || !dst || bytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
    return ADAFAC_EINVAL;
  if (bytes == 0) return ADAFAC_OK;
  return launch_stream_copy(src, dst, bytes / 16, static_cast<hipStream_t>(stream)) == hipSuccess ? ADAFAC_OK
                                                                                                 : ADAFAC_EDEVICE;
}

}  // extern "C"
