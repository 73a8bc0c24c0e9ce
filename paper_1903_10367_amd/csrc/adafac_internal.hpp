// Internal declarations shared by the host setup, the C ABI and the gfx950 kernels.
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace adafac {

constexpr int kMaxLevel = 9;    // 3^9 cells per axis in 2D, levels 0..9
constexpr int kNormBlocks = 2048;

inline int ipow3(int k) { int r = 1; while (k-- > 0) r *= 3; return r; }

// ---------------------------------------------------------------------------
// Host-side FP64 operators of one uniform level (full vertex lattice, x fastest)
// ---------------------------------------------------------------------------
struct HostLevel {
  int level = 0, n = 0, nv = 0;    // cells per axis, vertices per axis
  size_t nverts = 0;               // nv^d
  double h = 0;
  bool fem = true;                 // Q1 element operator from eps blocks (else stored stencil)
  std::vector<double> st;          // stored operator: 3^d entries per vertex (offset index o_x+3 o_y+9 o_z)
  std::vector<double> dg;          // diagonal of the operator (every level)
  std::vector<double> pw;          // transfer from level-1 to this level: 2^d weights per vertex, or empty = d-linear
  std::vector<double> rtw;         // OPERATOR R~ restricting the next finer level into this one: 5^d
                                   // weights per vertex (offset index (ox+2) + 5 (oy+2) + 25 (oz+2)), or empty
};

struct HostOps {
  int dim = 2, lmin = 1, L = 1;
  int nb = 1, k = 0;               // eps blocks per axis = 3^k
  std::vector<double> eps;         // nb^d
  std::vector<HostLevel> lev;      // indexed by level (0..L)
  std::vector<double> rtilde;      // 5^d weights of R~ (already times omega), offset index as st
  // R~ = scale * sum_a delta(o_a) prod_{b != a} m(o_b): the eps = 1 operator is a sum of tensor
  // products (1D stiffness x 1D masses) and the 1D stiffness annihilates the 1D hat except at
  // its centre, so R~ splits into d planar tensor-product stencils (checked against rtilde).
  double rt_m[5] = {0, 0, 0, 0, 0};
  double rt_scale = 0;
};

// Builds every operator of the hierarchy (FEM fine levels, BoxMG or d-linear
// transfers, Galerkin coarse operators below the coefficient-block level, R~; with
// rtilde_operator also the per-vertex R~ = omega trunc(P^T A D^-1) of every level below L).
// Returns an empty string on success, else a message.
std::string build_host_ops(HostOps& ops, int transfer_boxmg, double omega, int rtilde_operator = 0);

// Q1 stencil entry of a FEM level for vertex v and neighbour offset o (used by tests of the setup).
double fem_stencil_entry(const HostOps& ops, int level, const int* v, const int* o);

// ---------------------------------------------------------------------------
// Device views
// ---------------------------------------------------------------------------
template <typename T>
struct LevelView {
  int n, nv;                 // cells / vertices per axis
  T h;                       // mesh width
  T hd;                      // h^d (norm weight)
  T hdm2;                    // h^(d-2) (element scaling)
  int fem;                   // 1: operator from eps blocks, 0: stored stencil
  int nb;                    // eps blocks per axis
  int bs;                    // cells per block along an axis (>= 1) when fem
  unsigned bsm;              // ceil(2^32 / bs) when bs > 1 (cell / bs = umulhi(cell, bsm)), 0 when bs = 1
  const T* eps;              // nb^d block coefficients (nullptr: eps = 1)
  const T* st;               // stored stencil (3^d per vertex) when !fem
  const T* dg;               // stored diagonal when !fem
  const T* pw;               // transfer weights into this level (2^d per vertex) or nullptr: d-linear
  T* u;                      // FAS solution (coarse: injected); fine: unused here
  T* rr;                     // restricted residual R r_{l+1}
  T* bt;                     // auxiliary right-hand side R~ r_{l+1}
  T* bf;                     // FAS right-hand side R r_{l+1} + A_l I u_{l+1}
  T* r;                      // level residual
  T* S;                      // accumulated correction
  T* ic;                     // adAFAC-PI: injected correction of the next finer level
  const T* rtw;              // OPERATOR R~ into this level: 5^d weights per vertex, or nullptr (eps = 1 stencil)
};

// Tensor-product factors of R~ handed to the kernels.
template <typename T>
struct RtSep {
  T m[5];
  T scale;
};

// Pipelined solve: the cycles of a batch are launched without a host wait.  The launch of cycle
// `need` does nothing once *stop <= need; the kernel that forms a cycle's residual norms applies
// the stopping rule and, when it holds, writes *stop = that cycle's index + 1, so the cycle that
// met it still completes and every later one is skipped.  stop = nullptr: no gating.
struct Gate {
  const unsigned long long* stop;
  unsigned long long need;
};
// The stopping rule of a solve, applied on the device to the norms of cycle `need`: stop once
// ||r||_h <= tol ||r^0||_h (or ||r^0||_h = 0), or when ||r||_h is not finite or above 1e3 ||r^0||_h
// (the host then reports divergence).  r0 = nullptr with first = 1: this cycle's own norm is r^0.
struct StopRule {
  unsigned long long* stop;
  unsigned long long need;
  double tol;
  const double* r0;
  int first;
  int apply;               // 0: the launches are gated only (the inner cycles of FP32_REFINED)
};

// The smallest levels lo..hi handled by one workgroup (see k_small_levels).  lv[j] is the
// view of level lo-1+j (lv[0]: level lo-1, empty when lo is the coarsest; lv[hi-lo+2]: the
// next finer level hi+1).
constexpr int kMaxSmall = 4;
template <typename T>
struct SmallLevelsArgs {
  LevelView<T> lv[kMaxSmall + 2];
  int lo, hi;
  int gather[kMaxSmall];
  T cscale[kMaxSmall];
  RtSep<T> rts;
  T omega, omega_t;
  int damping;
  const double* partials;
  int nparts;
  double* norm_out;        // nullptr: no norms in this launch
  Gate gate;
  StopRule rule;           // rule.stop = nullptr: no stopping rule
};

// A chain of prolongations S_k <- S_k + P (S_{k-1} - sub_{k-1}) for k = 1 .. nt in one launch
// (see k_prolong_chain).  lv[0] is the source level (its S final), lv[k] the k-th target, lv[nt]
// the top one; sub[k] (may be null) is subtracted from lv[k]'s values where they feed the next
// prolongation, self (may be null) from the prolonged value at the top target's vertices.  The
// top target is updated in place; an intermediate target k reads lv[k].S and writes its new
// values to out[k] (other workgroups still read lv[k].S), whose boundary entries must hold
// those of lv[k].S.
constexpr int kMaxChain = 6;
template <typename T>
struct ProlongChainArgs {
  LevelView<T> lv[kMaxChain + 1];
  const T* sub[kMaxChain];
  T* out[kMaxChain];
  const T* self;
  int nt;
  Gate gate;
};

// ---------------------------------------------------------------------------
// Requests solved inside the batched work-queue kernel (continuous batching)
// ---------------------------------------------------------------------------
// One precision's hierarchy of a request: level views (v[L] describes the finest level; its
// iterate lives in ufine[cur], its right-hand side in bfine and its residual in rfine).
template <typename T>
struct BatchHier {
  LevelView<T> v[kMaxLevel + 1];
  T* ufine[2];
  T* bfine;
  T* rfine;
  RtSep<T> rts;
};

struct BatchReq {
  int dim, L, lmin, damping, precision, inner_k;
  double omega, omega_t, omega_hat;
  double tol;                // stop when ||r||_h / ||r^0||_h <= tol
  int max_cycles;            // cycles (FP64) or outer steps (FP32_REFINED)
  int fusable;               // the finest level can take the single-pass sweep (see run_cycle)
  BatchHier<double> h64;     // FP64 form: everything; FP32_REFINED: v[L], u (ufine[0]) and b
  BatchHier<float> h32;      // FP32_REFINED: the inner hierarchy (ufine = e, bfine = r)
  const float* ezero;        // FP32_REFINED: zero lattice, first inner iterate
  double* partials;          // norm partials of the finest level's work items, 2 per item
};

// Progress of a request across launches (device memory, written by the kernel).
struct BatchState {
  int cycles;                // cycles or outer steps run
  int status;                // 0 running, 1 converged, 2 diverged, 3 cycle cap reached
  int cur;                   // FP64 form: index of ufine holding the current iterate
  int pad;
  double r0, l2h, linf;      // norms of iterate 0 and of the last measured iterate
  unsigned long long stop_need;   // the request's items from this sequence number on do no work (stopped)
};

// Phase kinds of a serving step (one request's chain: FINE, FINAL, LEVEL l = L-1..lmin,
// PROLONG l = lmin+1..L for FP64; ADDE, DEFECT, FINAL, then per inner cycle FINE, LEVELs,
// PROLONGs in FP32 for FP32_REFINED).  Large requests replace FINE by SWEEP, the single-pass
// finest-level sweep launched on its own (it restricts to level L-1 and adds the previous
// cycle's pending prolongation), and leave the prolongation into level L pending; large 3D
// FP32_REFINED requests replace ADDE and DEFECT by DEFECT3, the one-pass u' = u + e + P S_{L-1}
// and FP64 defect of u' into the other FP64 buffer (also a launch of its own).
// A request's coarsest levels, up to `level` (each of at most kServeSmallVerts vertices), are one
// SMALL item: one workgroup runs their FAS updates (coarsest last) and then their
// prolongations, with a workgroup barrier between levels, as the per-level phases would.
enum {
  SERVE_FINE = 0, SERVE_FINAL, SERVE_LEVEL, SERVE_PROLONG, SERVE_ADDE, SERVE_DEFECT, SERVE_SWEEP, SERVE_DEFECT3,
  SERVE_SMALL
};
constexpr size_t kServeSmallVerts = 1024;
constexpr bool serve_own_launch(int kind) { return kind == SERVE_SWEEP || kind == SERVE_DEFECT3; }

// Kernel classes of the shared phase launches: a slot launches one kernel per class present.
// Light: prolongations and ADDE; heavy: the finest-level residuals (FINE, DEFECT), the coarse
// FAS updates (5^d gathers) and the stopping rule (which shares its slot with a heavy phase);
// small: the SMALL items (in the last restriction slot; a class of their own, since the two
// kernels together would spill).
enum { SERVE_CLS_LIGHT = 0, SERVE_CLS_HEAVY, SERVE_CLS_SMALL, SERVE_NCLS };
constexpr int serve_class(int kind) {
  return (kind == SERVE_PROLONG || kind == SERVE_ADDE) ? SERVE_CLS_LIGHT
                                                       : kind == SERVE_SMALL ? SERVE_CLS_SMALL : SERVE_CLS_HEAVY;
}

// One segment of a phase-slot launch's work list: the ntile items of one phase of one request.
struct ServeSeg {
  int req;                   // row of the request table
  int kind, level, sub;      // SERVE_*, the level it works on, inner cycle index (FP32 phases)
  int ntile, tile;           // items, vertices per item
  int need_off;              // items of the request in its earlier phases of the step
  int per_step;              // items of the request per step
  int item0;                 // first item of the segment within its launch
  int nparts;                // FINAL: norm partials to sum (items of the measured phase)
  int run_after;             // FINAL: items of the request after it that still run when it stops
  int cur0;                  // FP64: iterate index at the round's start
  int cps;                   // FP64: cycles per step (sub numbers them); 1 otherwise
  int gather;                // LEVEL, SMALL (its top level): 1 gathers R r, R~ r and I u from level + 1;
                             // 0: the sweep wrote them
  int pend;                  // ADDE: adds the pending P S_{L-1} with e; PROLONG into L-1 (SMALL: when it
                             // reaches L-1): subtracts I c_L;
                             // FINAL: the measured FP64 iterate is the other buffer (after DEFECT3)
  unsigned long long base;   // items of the request in earlier rounds (its sequence numbers start there)
};

// Internal hooks of the C ABI used by the request server (api.cpp).
int batch_describe(void* ctx, BatchReq* out);        // device description of a bound context
int batch_adopt(void* ctx, int cur, int pending);    // current iterate after batched cycles
int residual_range(void* ctx, int c0, int n, double* out);   // norms of cycles c0.., 2 per cycle

struct CycleParams {
  double omega, omega_t, omega_hat;
  int damping;               // ADAFAC_DAMP_*
  int L, lmin;
};

}  // namespace adafac
