// Request server of the C ABI (include/adafac.h): FIFO admission by device footprint into a
// pool inside the caller's workspace, batched advance of small requests in one work-queue
// launch, large requests on streams of their own, harvest of finished requests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <future>
#include <thread>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "adafac.h"
#include "adafac_internal.hpp"

namespace adafac {
hipError_t launch_serve_phase(int cls, const BatchReq* reqs, BatchState* states, const ServeSeg* segs, int nseg,
                              int nitems, int j, hipStream_t s);
template <typename T>
hipError_t launch_fine_sweep(int d, const LevelView<T>& F, const LevelView<T>& C, const T* uin, T* uout,
                             const T* b, const RtSep<T>& rt, T omega, int damping, int apply_pending,
                             double* partials, int* nparts, hipStream_t s, const unsigned long long* stop,
                             unsigned long long need);
int fine_sweep_nparts(int d, int n);
hipError_t launch_defect3d(const LevelView<double>& F, int nc, int nvc, const double* uin, double* uout,
                           const float* e, const float* S, const double* b, float* r32, double* partials,
                           int mode, int* nparts, hipStream_t s, const unsigned long long* stop,
                           unsigned long long need);
}  // namespace adafac

using namespace adafac;

namespace {

constexpr size_t kAlign = 256;
constexpr int kSegsPerSlot = 96;   // work-list segments held per request slot (on average)
// vertices per work item (whole lattice rows for the row-based phases): finest-level phases (at
// most kNormBlocks items, one norm partial each), coarse FAS updates (5^d gathers per vertex)
// and prolongations
constexpr size_t kFineItem = 2048, kLevelItem = 256, kProlongItem = 2048;
// requests with at least this many finest-level vertices sweep that level in one pass (when
// their options allow it): a launch of its own, which the smaller requests' phases do not share
constexpr size_t kSweepMinVerts = size_t(1) << 18;
constexpr int kPrepThreads = 4;    // host set-ups of queued requests running at once
constexpr int kPrepAhead = 16;     // queued requests set up ahead of admission (host memory bound)

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator of byte ranges [0, size).
class Pool {
 public:
  void reset(size_t size) {
    free_.clear();
    size_ = size;
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0;
};

struct Req {
  uint64_t ticket = 0;
  int dim = 2, lmin = 1, L = 1, nb = 0;
  std::vector<double> eps, f;
  adafac_opts opts{};
  double tol = 0;
  int max_cycles = 1;
  adafac_result res{};
  adafac_ctx* ctx = nullptr;
  size_t off = 0, bytes = 0;
  int slot = -1;          // batched: row of the request table
  int lane = -1;          // large: stream index
  int cycles_seen = 0;    // large: cycles whose norms were examined
  std::vector<double> u;  // solution once finished
  std::future<int> prep;  // host-side set-up on a worker thread
  bool prep_started = false;
  bool prepared = false;  // prep finished; its status is prep_rc
  int prep_rc = 0;
  unsigned long long items_base = 0;   // batched: work items of the request in earlier rounds
  int cur_next = 0;       // batched: iterate buffer at the start of its next round (see launch_batched)
  bool sweep = false;     // batched: its finest level takes the single-pass sweep
  // batched: binding (uploads and load vector) after admission, or finishing (solution to the
  // host) after the stopping rule, on a worker thread; the request holds its pool range meanwhile
  std::future<int> job;
  int bg = 0;             // 0 none, 1 binding, 2 finishing
  int fin_status = 0;     // finishing: the status it ends with
};

// A batched round in flight: its launches, then a copy of the state table to pinned host memory
// and an event.  kFlights rounds may be in flight; each has its own work-list buffers.
constexpr int kFlights = 3;
struct Flight {
  uint64_t id = 0;
  int buf = 0;                         // buffers of this flight (work lists, state copy, event)
  std::vector<uint64_t> members;       // requests of the round
};

size_t finest_vertices(int d, int L) {
  size_t nv = size_t(ipow3(L) + 1);
  return d == 2 ? nv * nv : nv * nv * nv;
}

}  // namespace

struct adafac_server {
  adafac_server_cfg cfg{};
  char* ws = nullptr;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  BatchReq* d_reqs = nullptr;
  BatchState* d_states = nullptr;
  ServeSeg* d_segs[kFlights] = {};     // work lists, one buffer per flight
  int seg_cap = 0;                     // segments per buffer
  char* pool_base = nullptr;
  Pool pool;
  std::vector<hipStream_t> lanes;
  hipStream_t setup = nullptr;         // uploads of newly admitted requests
  std::vector<int> lane_busy;          // a request holds the lane
  std::vector<int> lane_flight;        // its last chunk of cycles is enqueued and not harvested
  std::vector<uint64_t> lane_req;
  std::deque<Flight> flights;          // batched rounds enqueued and not harvested, oldest first
  uint64_t next_flight = 1, launched = 0, harvested = 0;   // flight ids
  BatchState* snap[kFlights] = {};     // pinned: the state table after each flight's round
  hipEvent_t done_ev[kFlights] = {};
  std::vector<ServeSeg> h_segs[kFlights];   // host sources of the work-list uploads
  bool buf_busy[kFlights] = {};
  std::vector<int> free_slots;
  // slots of finished requests, free again once every round launched before the finish (which
  // may still hold the request's no-op items) has been harvested: (last such flight id, slot)
  std::vector<std::pair<uint64_t, int>> quarantine;
  std::vector<BatchReq> h_desc;        // host copies of the table rows (kept for async copies)
  std::vector<BatchState> h_states;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Req> reqs;
  std::vector<uint64_t> active;
  std::vector<uint64_t> background;    // batched requests binding or finishing on worker threads
  uint64_t next_ticket = 1;
  std::chrono::steady_clock::time_point t0;
  std::string err;
  // host time spent per phase of adafac_server_step (seconds) and rounds run
  double t_harvest = 0, t_admit = 0, t_launch = 0;
  double t_issue = 0;             // part of t_launch spent issuing the round's copies and launches
  std::vector<double> norm_buf;   // a lane chunk's norms
  long rounds = 0;
  long launches = 0;              // kernel launches of batched rounds
};

namespace {

int sfail(adafac_server* s, int code, const std::string& m) {
  if (s) s->err = m;
  return code;
}

#define SHIP(srv, expr)                                                                     \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return sfail(srv, ADAFAC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

double now(const adafac_server* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

bool final_status(int st) { return st >= ADAFAC_REQ_CONVERGED; }

// Build (once) the host side of a request's hierarchy.
int build_ctx(Req* rp) {
  Req& r = *rp;
  adafac_ctx* c = nullptr;
  int rc = adafac_create(&c, r.dim, r.lmin, r.L);
  if (rc) return rc;
  if (r.nb > 0 && (rc = adafac_set_coefficient_blocks(c, r.nb, r.eps.data()))) {
    adafac_destroy(c);
    return rc;
  }
  if ((rc = adafac_set_rhs_lattice(c, r.f.data(), r.f.size())) || (rc = adafac_build_operators(c, &r.opts)) ||
      (rc = adafac_workspace_bytes(c, &r.bytes))) {
    adafac_destroy(c);
    return rc;
  }
  r.ctx = c;
  return ADAFAC_OK;
}

// Batched request: its solution to the host (with the pending prolongation of a swept FP64
// request added first) and its context released.  Runs on a worker thread.
int finish_batched_job(Req* rp, int cur, int pending) {
  Req& r = *rp;
  int rc = batch_adopt(r.ctx, cur, pending);
  r.u.assign(finest_vertices(r.dim, r.L), 0.0);
  if (!rc) rc = adafac_get_solution(r.ctx, r.u.data(), r.u.size());
  adafac_destroy(r.ctx);
  r.ctx = nullptr;
  return rc;
}

// Release a finished request's device resources, keeping its solution on the host.  A batched
// request does so on a worker thread (complete_background ends it); its status stays RUNNING
// until the solution is on the host.
int finish(adafac_server* s, Req& r, int status, int cur) {
  if (r.res.batched && r.ctx) {
    // an FP64 request whose cycles swept the finest level has the last P S_{L-1} pending
    const int pending = r.sweep && s->h_desc[r.slot].precision == ADAFAC_PREC_FP64;
    r.fin_status = status;
    r.bg = 2;
    r.job = std::async(std::launch::async, finish_batched_job, &r, cur, pending);
    s->background.push_back(r.ticket);
    // Its table row is read by the rounds still in flight (where its items find it stopped), so
    // the slot waits for those rounds.
    s->quarantine.emplace_back(s->launched, r.slot);
    r.slot = -1;
    return ADAFAC_OK;
  }
  r.res.status = status;
  r.res.t_done = now(s);
  if (r.ctx) {
    int rc = ADAFAC_OK;
    // an FP64 request whose cycles swept the finest level has the last P S_{L-1} pending
    if (r.res.batched) rc = batch_adopt(r.ctx, cur, r.sweep && s->h_desc[r.slot].precision == ADAFAC_PREC_FP64);
    r.u.assign(finest_vertices(r.dim, r.L), 0.0);
    if (!rc) rc = adafac_get_solution(r.ctx, r.u.data(), r.u.size());
    adafac_destroy(r.ctx);
    r.ctx = nullptr;
    if (rc) {
      r.res.status = ADAFAC_REQ_FAILED;
      r.res.error = rc;
    }
  }
  s->pool.release(r.off, r.bytes);
  if (r.lane >= 0) {
    s->lane_busy[r.lane] = 0;
    s->lane_flight[r.lane] = 0;
  }
  r.slot = r.lane = -1;
  r.f.clear();
  r.f.shrink_to_fit();
  return ADAFAC_OK;
}

// Whether the work enqueued on st has completed (any error counts as completed: the caller's
// synchronisation then reports it).  A not-ready query is cleared from the last-error state so
// that the next launch check does not see it.
bool ready(hipStream_t st, bool wait) {
  if (wait) return true;
  const hipError_t e = hipStreamQuery(st);
  if (e == hipErrorNotReady) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

void drop_active(adafac_server* s, uint64_t t) {
  for (size_t k = 0; k < s->active.size(); ++k)
    if (s->active[k] == t) {
      s->active.erase(s->active.begin() + long(k));
      return;
    }
}

// Batched group: when its oldest round in flight has completed, finish the requests that
// stopped (in it, or in the one before).
int harvest_batched(adafac_server* s, bool wait, bool* done) {
  *done = false;
  if (s->flights.empty()) return ADAFAC_OK;
  const Flight f = s->flights.front();
  if (wait) {
    SHIP(s, hipEventSynchronize(s->done_ev[f.buf]));
  } else {
    const hipError_t e = hipEventQuery(s->done_ev[f.buf]);
    if (e == hipErrorNotReady) {
      (void)hipGetLastError();
      return ADAFAC_OK;
    }
    SHIP(s, e);
  }
  s->flights.pop_front();
  s->buf_busy[f.buf] = false;
  s->harvested = f.id;
  *done = true;
  for (size_t k = 0; k < s->quarantine.size();) {
    if (s->quarantine[k].first <= s->harvested) {
      s->free_slots.push_back(s->quarantine[k].second);
      s->quarantine[k] = s->quarantine.back();
      s->quarantine.pop_back();
    } else {
      ++k;
    }
  }
  const BatchState* snap = s->snap[f.buf];
  for (uint64_t t : f.members) {
    auto it = s->reqs.find(t);
    if (it == s->reqs.end()) continue;
    Req& r = it->second;
    if (r.slot < 0 || final_status(r.res.status)) continue;   // finished at an earlier harvest
    const BatchState& st = snap[r.slot];
    r.res.cycles = st.cycles;
    r.res.l2h0 = st.r0;
    r.res.l2h = st.l2h;
    r.res.linf = st.linf;
    int status = ADAFAC_REQ_RUNNING;
    if (st.status == 1) status = ADAFAC_REQ_CONVERGED;
    else if (st.status == 2) status = ADAFAC_REQ_DIVERGED;
    else if (st.status == 3) status = ADAFAC_REQ_CAPPED;
    if (status != ADAFAC_REQ_RUNNING) {
      int rc = finish(s, r, status, st.cur);
      if (rc) return rc;
      drop_active(s, t);
    }
  }
  return ADAFAC_OK;
}

// Slot template of a round, shared by all its requests so that phases of one kind line up: a
// step is `prefix` slots (FP32_REFINED: ADDE, DEFECT, then the stopping rule, which shares the
// next slot; empty for FP64 requests) and `cps` cycle blocks of T = Dr + Pm slots.  In a block a
// request's restriction phases (the finest-level FINE or SWEEP, then LEVEL L-1 .. l_min) end at
// slot Dr - 1 and its prolongations start at slot Dr, so restriction slots hold heavy phases
// and prolongation slots light ones.  An FP64 step is cps cycles (each with its own stopping
// rule), so that FP64 requests move on as far per launch chain as FP32-refined ones whose steps
// hold inner_k cycles.
struct StepTemplate {
  int cps = 1, prefix = 0, Dr = 1, Pm = 0;
};

// The top level of a request's SMALL item: the largest l < L whose levels l_min .. l have at most
// kServeSmallVerts vertices each, when that covers at least two levels; else l_min - 1 (none).
int small_top(const BatchReq& d) {
  int hi = d.lmin - 1;
  for (int l = d.lmin; l < d.L; ++l) {
    const size_t n = size_t(ipow3(l) + 1);
    if ((d.dim == 2 ? n * n : n * n * n) > kServeSmallVerts) break;
    hi = l;
  }
  return hi - d.lmin + 1 >= 2 ? hi : d.lmin - 1;
}
// restriction: FINE or SWEEP, LEVEL L-1 .. hi+1 (or .. l_min), SMALL; prolongation: into hi+1 .. L
// (.. L-1 when the sweep leaves the finest one pending)
int restriction_phases(const BatchReq& d) {
  const int hi = small_top(d);
  return hi >= d.lmin ? 1 + (d.L - 1 - hi) + 1 : 1 + d.L - d.lmin;
}
int prolong_phases(const BatchReq& d, bool sweep) {
  const int top = (sweep && d.L > d.lmin) ? d.L - 1 : d.L;
  return top - std::max(d.lmin, small_top(d));
}

// The phases of one step of a request, in order (see ServeSeg), and slots[i], the launch (phase
// slot) of phase i.  The stopping rule's item shares its slot with the phase after it, which
// does not read its result (under FP64 that phase runs even when the request stops; under
// FP32_REFINED it only writes the inner correction, which a stopped request never adds).
// sweep: the finest level takes the single-pass sweep (SWEEP, one item in the request's sequence,
// launched on its own), level L-1 is fed by it, and the prolongation into level L is left
// pending for the next sweep (FP64) or the next outer step's ADDE (FP32_REFINED).
void step_program(const BatchReq& d, const StepTemplate& tp, bool sweep, std::vector<ServeSeg>& prog,
                  std::vector<int>& slots) {
  const int cps = tp.cps, T = tp.Dr + tp.Pm;
  prog.clear();
  slots.clear();
  auto nv_of = [&](int l) {
    const size_t n = size_t(ipow3(l) + 1);
    return d.dim == 2 ? n * n : n * n * n;
  };
  // lattice rows (nv vertices each) of level l: the unit of the row-based phases
  auto rows_of = [&](int l) {
    const size_t n = size_t(ipow3(l) + 1);
    return d.dim == 2 ? n : n * n;
  };
  auto add = [&](int kind, int level, int sub, size_t units, size_t tile, int slot) {
    slots.push_back(slot);
    ServeSeg g{};
    g.kind = kind;
    g.level = level;
    g.sub = sub;
    g.tile = int(tile);
    g.ntile = int((units + tile - 1) / tile);
    prog.push_back(g);
  };
  auto rows_per_item = [&](int l, size_t verts) {
    const size_t nv = size_t(ipow3(l) + 1);
    return std::max<size_t>(1, (verts + nv - 1) / nv);
  };
  // finest-level items: about kFineItem vertices, at most kNormBlocks of them (one norm partial each)
  const size_t rL = rows_of(d.L);
  const size_t tf = std::max(rows_per_item(d.L, kFineItem), (rL + size_t(kNormBlocks) - 1) / size_t(kNormBlocks));
  const int nf = int((rL + tf - 1) / tf);
  const bool fp64 = d.precision == ADAFAC_PREC_FP64;
  const bool pi = d.damping == ADAFAC_DAMP_PI;
  const int hi = small_top(d);
  auto cycle_phases = [&](int sub, int base) {
    const int s0 = base + tp.Dr - restriction_phases(d);   // this request's first restriction slot
    if (sweep) add(SERVE_SWEEP, d.L, sub, 1, 1, s0);
    else add(SERVE_FINE, d.L, sub, rL, tf, s0);
    if (fp64) add(SERVE_FINAL, d.L, sub, 1, 1, s0 + 1);
    for (int l = d.L - 1; l > hi && l >= d.lmin; --l) {
      add(SERVE_LEVEL, l, sub, nv_of(l), kLevelItem, s0 + d.L - l);
      prog.back().gather = (sweep && l == d.L - 1) ? 0 : 1;
    }
    if (hi >= d.lmin) {
      add(SERVE_SMALL, hi, sub, 1, 1, s0 + d.L - hi);
      prog.back().gather = (sweep && hi == d.L - 1) ? 0 : 1;
      prog.back().pend = (sweep && pi) ? 1 : 0;
    }
    int i = 0;
    for (int l = std::max(d.lmin, hi) + 1; l <= (sweep ? d.L - 1 : d.L); ++l, ++i) {
      add(SERVE_PROLONG, l, sub, rows_of(l), rows_per_item(l, kProlongItem), base + tp.Dr + i);
      prog.back().pend = (sweep && pi && l == d.L - 1) ? 1 : 0;
    }
  };
  if (fp64) {
    for (int c = 0; c < cps; ++c) cycle_phases(c, tp.prefix + c * T);
  } else if (sweep && d.dim == 3) {
    add(SERVE_DEFECT3, d.L, 0, 1, 1, 1);
    add(SERVE_FINAL, d.L, 0, 1, 1, 2);
    prog.back().pend = 1;
    for (int i = 0; i < d.inner_k; ++i) cycle_phases(i, tp.prefix + i * T);
  } else {
    add(SERVE_ADDE, d.L, 0, rL, tf, 0);
    prog.back().pend = sweep ? 1 : 0;
    add(SERVE_DEFECT, d.L, 0, rL, tf, 1);
    add(SERVE_FINAL, d.L, 0, 1, 1, 2);
    for (int i = 0; i < d.inner_k; ++i) cycle_phases(i, tp.prefix + i * T);
  }
  int off = 0;
  for (ServeSeg& g : prog) {
    g.need_off = off;
    off += g.ntile;
  }
  const int per_cycle = fp64 ? off / cps : 0;
  for (size_t p = 0; p < prog.size(); ++p) {
    ServeSeg& g = prog[p];
    g.per_step = off;
    g.cps = fp64 ? cps : 1;
    if (g.kind == SERVE_FINAL) {
      // the one-pass sweep and defect cut the finest level into the same tiles
      g.nparts = (sweep && (fp64 || d.dim == 3)) ? fine_sweep_nparts(d.dim, ipow3(d.L)) : nf;
      // FP64: the rest of its cycle still runs when it stops (that cycle produces the result)
      g.run_after = fp64 ? (g.sub + 1) * per_cycle - (g.need_off + 1) : 0;
    }
  }
}

// The phases with launches of their own (serve_own_launch), segment g in step j: each does
// nothing when the request stopped before this item of its sequence.  SWEEP: the single-pass
// finest-level sweep.  DEFECT3: u' = u + e + P S_{L-1} (nothing added before the first outer
// step) and the FP64 defect of u', into the other FP64 buffer.
hipError_t launch_own(adafac_server* s, const ServeSeg& g, int j, bool first) {
  const BatchReq& d = s->h_desc[g.req];
  const int L = d.L;
  const unsigned long long need =
      g.base + (unsigned long long)j * (unsigned long long)g.per_step + (unsigned long long)g.need_off;
  const unsigned long long* stop = &s->d_states[g.req].stop_need;
  int np = 0;
  if (g.kind == SERVE_DEFECT3) {
    const int cur = g.cur0 ^ (j & 1);
    const int mode = (first && j == 0) ? 0 : 2;
    const LevelView<float>& C = d.h32.v[L - 1];
    return launch_defect3d(d.h64.v[L], C.n, C.nv, d.h64.ufine[cur], d.h64.ufine[1 - cur], d.h32.ufine[d.inner_k & 1],
                           mode == 2 ? C.S : nullptr, d.h64.bfine, d.h32.bfine, d.partials, mode, &np, s->stream,
                           stop, need);
  }
  if (d.precision == ADAFAC_PREC_FP64) {
    const int cur = g.cur0 ^ ((j * g.cps + g.sub) & 1);
    const double* uin = d.h64.ufine[cur];
    LevelView<double> F = d.h64.v[L];
    F.u = const_cast<double*>(uin);
    F.r = d.h64.rfine;
    const int pend = (first && j == 0 && g.sub == 0) ? 0 : 1;
    return launch_fine_sweep<double>(d.dim, F, d.h64.v[L - 1], uin, d.h64.ufine[1 - cur], d.h64.bfine, d.h64.rts,
                                     d.omega, d.damping, pend, d.partials, &np, s->stream, stop, need);
  }
  // inner cycle g.sub of an outer step: e_0 = 0, e_{i+1} from e_i plus the pending P S_{L-1}
  const float* uin = g.sub == 0 ? d.ezero : d.h32.ufine[g.sub & 1];
  LevelView<float> F = d.h32.v[L];
  F.u = const_cast<float*>(uin);
  F.r = d.h32.rfine;
  return launch_fine_sweep<float>(d.dim, F, d.h32.v[L - 1], uin, d.h32.ufine[(g.sub + 1) & 1], d.h32.bfine,
                                  d.h32.rts, float(d.omega), d.damping, g.sub > 0 ? 1 : 0, d.partials, &np, s->stream,
                                  stop, need);
}

// One round advances every batched request by cycles_per_round steps.  Launch (j, p) runs the
// p-th phase of step j of every request whose chain has one, so the launch count per round is
// cycles_per_round x the longest chain, independent of the number of requests.
int launch_batched(adafac_server* s) {
  if (int(s->flights.size()) >= kFlights) return ADAFAC_OK;
  int buf = 0;
  while (s->buf_busy[buf]) ++buf;
  Flight fl;
  fl.buf = buf;
  std::vector<std::vector<ServeSeg>> progs;
  std::vector<std::vector<int>> pslots;
  std::vector<ServeSeg> prog;
  std::vector<int> slots;
  size_t nseg = 0, maxp = 0;
  const int steps = s->cfg.cycles_per_round;
  StepTemplate tp;
  for (uint64_t t : s->active) {
    const Req& r = s->reqs[t];
    if (!r.res.batched) continue;
    const BatchReq& d = s->h_desc[r.slot];
    if (d.precision != ADAFAC_PREC_FP64) {
      tp.cps = std::max(tp.cps, d.inner_k);
      tp.prefix = 2;
    }
    tp.Dr = std::max(tp.Dr, restriction_phases(d));
    tp.Pm = std::max(tp.Pm, prolong_phases(d, r.sweep));
  }
  struct SweepJob {
    size_t p;       // phase slot
    ServeSeg g;
    bool first;     // the request's first cycle has no pending prolongation
  };
  std::vector<SweepJob> sweeps;
  for (uint64_t t : s->active) {
    Req& r = s->reqs[t];
    if (!r.res.batched) continue;
    step_program(s->h_desc[r.slot], tp, r.sweep, prog, slots);
    if (nseg + prog.size() > size_t(s->seg_cap)) break;   // the rest joins a later round
    for (ServeSeg& g : prog) {
      g.req = r.slot;
      g.cur0 = r.cur_next;
      g.base = r.items_base;
    }
    for (size_t k = 0; k < prog.size(); ++k)
      if (serve_own_launch(prog[k].kind)) sweeps.push_back(SweepJob{size_t(slots[k]), prog[k], r.items_base == 0});
    r.items_base += (unsigned long long)steps * (unsigned long long)prog[0].per_step;
    // Where the round leaves the iterate if the request does not stop in it (when it stops, its
    // later rounds do nothing and their start does not matter): an FP64 cycle, and an outer step
    // with the one-pass 3D defect, swap the two FP64 buffers.
    const BatchReq& d = s->h_desc[r.slot];
    bool flips = d.precision == ADAFAC_PREC_FP64;
    for (const ServeSeg& g : prog) flips |= g.kind == SERVE_DEFECT3;
    if (flips) r.cur_next ^= (steps * prog[0].cps) & 1;
    nseg += prog.size();
    maxp = std::max(maxp, size_t(slots.back() + 1));
    progs.push_back(prog);
    pslots.push_back(slots);
    fl.members.push_back(t);
  }
  if (fl.members.empty()) return ADAFAC_OK;
  std::vector<ServeSeg>& hsegs = s->h_segs[buf];
  ServeSeg* dsegs = s->d_segs[buf];
  // work lists: per slot, one per kernel class (list q = p * SERVE_NCLS + class), each in
  // request order; a counting sort over all segments
  const size_t nlist = maxp * SERVE_NCLS;
  std::vector<int> list_off(nlist + 1, 0), list_items(nlist, 0);
  auto list_of = [&](size_t k, size_t a) { return size_t(pslots[k][a]) * SERVE_NCLS + size_t(serve_class(progs[k][a].kind)); };
  for (size_t k = 0; k < progs.size(); ++k)
    for (size_t a = 0; a < progs[k].size(); ++a)
      if (!serve_own_launch(progs[k][a].kind)) ++list_off[list_of(k, a) + 1];
  for (size_t q = 0; q < nlist; ++q) list_off[q + 1] += list_off[q];
  hsegs.resize(size_t(list_off[nlist]));
  std::vector<int> fill(list_off.begin(), list_off.end() - 1);
  for (size_t k = 0; k < progs.size(); ++k)
    for (size_t a = 0; a < progs[k].size(); ++a) {
      if (serve_own_launch(progs[k][a].kind)) continue;   // a launch of its own
      const size_t q = list_of(k, a);
      ServeSeg g = progs[k][a];
      g.item0 = list_items[q];
      list_items[q] += g.ntile;
      hsegs[size_t(fill[q]++)] = g;
    }
  // own launches by slot
  std::stable_sort(sweeps.begin(), sweeps.end(), [](const SweepJob& x, const SweepJob& y) { return x.p < y.p; });
  const double t_i0 = now(s);
  SHIP(s, hipMemcpyAsync(dsegs, hsegs.data(), sizeof(ServeSeg) * hsegs.size(), hipMemcpyHostToDevice,
                         s->stream));
  // Within a slot the shared launches go first: an FP32_REFINED request's stopping rule shares
  // the slot with its first inner sweep, which then sees the decision and does not overwrite the
  // norm partials before they are read.  The phases of a slot are independent of one another
  // (different requests, or a request's stopping rule and the phase after it, which does not
  // read its result), so the order of the class launches does not matter.
  for (int j = 0; j < steps; ++j) {
    size_t w = 0;
    for (size_t p = 0; p < maxp; ++p) {
      for (int cls = 0; cls < SERVE_NCLS; ++cls) {
        const size_t q = p * SERVE_NCLS + size_t(cls);
        if (list_items[q] == 0) continue;
        SHIP(s, launch_serve_phase(cls, s->d_reqs, s->d_states, dsegs + list_off[q], list_off[q + 1] - list_off[q],
                                   list_items[q], j, s->stream));
        ++s->launches;
      }
      for (; w < sweeps.size() && sweeps[w].p == p; ++w) {
        SHIP(s, launch_own(s, sweeps[w].g, j, sweeps[w].first));
        ++s->launches;
      }
    }
  }
  SHIP(s, hipMemcpyAsync(s->snap[buf], s->d_states, sizeof(BatchState) * size_t(s->cfg.max_active),
                         hipMemcpyDeviceToHost, s->stream));
  SHIP(s, hipEventRecord(s->done_ev[buf], s->stream));
  s->t_issue += now(s) - t_i0;
  fl.id = s->next_flight++;
  s->launched = fl.id;
  s->buf_busy[buf] = true;
  s->flights.push_back(std::move(fl));
  return ADAFAC_OK;
}

// Lane k: when its chunk has completed, assess the new cycles and finish or enqueue the next chunk.
int service_lane(adafac_server* s, int k, bool wait, bool* done) {
  *done = false;
  if (!s->lane_busy[k]) return ADAFAC_OK;
  Req& r = s->reqs[s->lane_req[k]];
  if (s->lane_flight[k]) {
    if (!ready(s->lanes[k], wait)) return ADAFAC_OK;
    s->lane_flight[k] = 0;
    *done = true;
    int status = ADAFAC_REQ_RUNNING;
    const int n = adafac_cycles_run(r.ctx);
    s->norm_buf.resize(2 * size_t(std::max(n - r.cycles_seen, 0)));
    if (n > r.cycles_seen) {
      int rc = residual_range(r.ctx, r.cycles_seen, n - r.cycles_seen, s->norm_buf.data());
      if (rc) return sfail(s, rc, adafac_last_error(r.ctx));
    }
    for (int c = r.cycles_seen; c < n && status == ADAFAC_REQ_RUNNING; ++c) {
      const double l2 = s->norm_buf[2 * size_t(c - r.cycles_seen)], li = s->norm_buf[2 * size_t(c - r.cycles_seen) + 1];
      if (c == 0) r.res.l2h0 = l2;
      r.res.l2h = l2;
      r.res.linf = li;
      if (!std::isfinite(l2) || l2 > 1e3 * r.res.l2h0) status = ADAFAC_REQ_DIVERGED;
      else if (r.res.l2h0 == 0.0 || l2 / r.res.l2h0 <= r.tol) status = ADAFAC_REQ_CONVERGED;
    }
    r.cycles_seen = n;
    r.res.cycles = n;
    if (status == ADAFAC_REQ_RUNNING && n >= r.max_cycles) status = ADAFAC_REQ_CAPPED;
    if (status != ADAFAC_REQ_RUNNING) {
      const uint64_t t = r.ticket;
      int rc = finish(s, r, status, 0);
      if (rc) return rc;
      drop_active(s, t);
      return ADAFAC_OK;
    }
  }
  // enqueue the next chunk of cycles
  const int n = std::min(s->cfg.cycles_per_round, r.max_cycles - adafac_cycles_run(r.ctx));
  if (n > 0) {
    int rc = adafac_cycle(r.ctx, n);
    if (rc) return sfail(s, rc, adafac_last_error(r.ctx));
    s->lane_flight[k] = 1;
  }
  return ADAFAC_OK;
}

// Batched requests on worker threads: a finished binding joins the next round enqueued (its
// table row uploaded here); a finished finishing releases the pool range (the request's items
// in rounds still in flight find it stopped and touch none of its memory) and ends the request.
int complete_background(adafac_server* s, bool wait) {
  bool rows = false;
  for (size_t k = 0; k < s->background.size();) {
    Req& r = s->reqs[s->background[k]];
    if (!wait && r.job.wait_for(std::chrono::seconds(0)) != std::future_status::ready) {
      ++k;
      continue;
    }
    int rc = r.job.get();
    s->background[k] = s->background.back();
    s->background.pop_back();
    if (r.bg == 2) {
      r.bg = 0;
      r.res.status = rc ? ADAFAC_REQ_FAILED : r.fin_status;
      if (rc) r.res.error = rc;
      r.res.t_done = now(s);
      s->pool.release(r.off, r.bytes);
      r.f.clear();
      r.f.shrink_to_fit();
      continue;
    }
    r.bg = 0;
    if (rc) {
      // the slot never entered a round
      s->pool.release(r.off, r.bytes);
      s->free_slots.push_back(r.slot);
      r.slot = -1;
      r.res.status = ADAFAC_REQ_FAILED;
      r.res.error = rc;
      r.res.t_done = now(s);
      adafac_destroy(r.ctx);
      r.ctx = nullptr;
      continue;
    }
    BatchReq& d = s->h_desc[r.slot];
    if ((rc = batch_describe(r.ctx, &d))) return sfail(s, rc, "batch_describe");
    r.sweep = d.fusable && finest_vertices(r.dim, r.L) >= kSweepMinVerts;
    d.tol = r.tol;
    d.max_cycles = r.max_cycles;
    s->h_states[r.slot] = BatchState{};
    s->h_states[r.slot].stop_need = ~0ull;
    SHIP(s, hipMemcpyAsync(&s->d_reqs[r.slot], &d, sizeof(BatchReq), hipMemcpyHostToDevice, s->setup));
    SHIP(s, hipMemcpyAsync(&s->d_states[r.slot], &s->h_states[r.slot], sizeof(BatchState), hipMemcpyHostToDevice,
                           s->setup));
    s->active.push_back(r.ticket);
    rows = true;
  }
  // the next batched launch reads the new table rows
  if (rows) SHIP(s, hipStreamSynchronize(s->setup));
  return ADAFAC_OK;
}

// Start the host-side set-up of queued requests, in arrival order, on worker threads: at most
// kPrepThreads at once and kPrepAhead set up (or being set up) ahead of admission.
void prepare(adafac_server* s) {
  int running = 0, ahead = 0;
  for (uint64_t t : s->queue) {
    Req& r = s->reqs[t];
    if (!r.prep_started) continue;
    ++ahead;
    if (!r.prepared && r.prep.wait_for(std::chrono::seconds(0)) != std::future_status::ready) ++running;
  }
  for (uint64_t t : s->queue) {
    if (running >= kPrepThreads || ahead >= kPrepAhead) break;
    Req& r = s->reqs[t];
    if (r.prep_started) continue;
    r.prep = std::async(std::launch::async, build_ctx, &r);
    r.prep_started = true;
    ++running;
    ++ahead;
  }
}

// Admit prepared requests in arrival order while slots and memory allow; their uploads go to
// the setup stream and they join the next round's launch.
int admit(adafac_server* s) {
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    if (int(s->active.size() + s->background.size()) >= s->cfg.max_active) break;
    Req& r = s->reqs[*it];
    if (!r.prep_started) {
      ++it;
      continue;
    }
    if (!r.prepared) {
      if (r.prep.wait_for(std::chrono::seconds(0)) != std::future_status::ready) {
        ++it;
        continue;
      }
      r.prep_rc = r.prep.get();
      r.prepared = true;
    }
    int rc = r.prep_rc;
    if (!rc && r.bytes > s->pool.size()) rc = ADAFAC_ENOMEM;
    if (rc) {
      if (r.ctx) adafac_destroy(r.ctx);
      r.ctx = nullptr;
      r.res.status = ADAFAC_REQ_FAILED;
      r.res.error = rc;
      r.res.t_done = now(s);
      it = s->queue.erase(it);
      continue;
    }
    const bool batched = finest_vertices(r.dim, r.L) <= s->cfg.batch_max_vertices;
    int lane = -1;
    if (!batched) {
      for (int k = 0; k < int(s->lanes.size()); ++k)
        if (!s->lane_busy[k]) { lane = k; break; }
      if (lane < 0) { ++it; continue; }
    } else if (s->free_slots.empty()) {
      ++it;
      continue;
    }
    size_t off = 0;
    if (!s->pool.alloc(r.bytes, &off)) { ++it; continue; }
    if (batched) {
      // binding (the load vector and the uploads) on a worker thread; the request joins a round
      // once it has finished (complete_background)
      r.off = off;
      r.res.footprint = align_up(r.bytes);
      r.res.batched = 1;
      r.res.t_admit = now(s);
      r.res.status = ADAFAC_REQ_RUNNING;
      r.slot = s->free_slots.back();
      s->free_slots.pop_back();
      r.bg = 1;
      r.job = std::async(std::launch::async, adafac_bind, r.ctx, static_cast<void*>(s->pool_base + off),
                         align_up(r.bytes), static_cast<void*>(s->setup));
      s->background.push_back(r.ticket);
      it = s->queue.erase(it);
      continue;
    }
    hipStream_t st = s->lanes[lane];
    rc = adafac_bind(r.ctx, s->pool_base + off, align_up(r.bytes), st);
    if (rc) {
      s->pool.release(off, r.bytes);
      r.res.status = ADAFAC_REQ_FAILED;
      r.res.error = rc;
      r.res.t_done = now(s);
      adafac_destroy(r.ctx);
      r.ctx = nullptr;
      it = s->queue.erase(it);
      continue;
    }
    r.off = off;
    r.res.footprint = align_up(r.bytes);
    r.res.batched = 0;
    r.res.t_admit = now(s);
    r.res.status = ADAFAC_REQ_RUNNING;
    r.lane = lane;
    s->lane_busy[lane] = 1;
    s->lane_flight[lane] = 0;
    s->lane_req[lane] = r.ticket;
    s->active.push_back(r.ticket);
    it = s->queue.erase(it);
  }
  prepare(s);
  return complete_background(s, false);
}

}  // namespace

extern "C" {

void adafac_server_default_cfg(adafac_server_cfg* c) {
  if (!c) return;
  c->max_active = 256;
  c->max_queued = 4096;
  c->cycles_per_round = 4;
  c->max_streams = 4;
  c->batch_max_vertices = SIZE_MAX;   // every request joins the batched launch
}

int adafac_server_create(const adafac_server_cfg* cfg, void* ws, size_t bytes, void* stream, adafac_server** out) {
  if (!out) return ADAFAC_EINVAL;
  *out = nullptr;
  adafac_server_cfg c;
  adafac_server_default_cfg(&c);
  if (cfg) c = *cfg;
  if (c.max_active < 1 || c.max_active > 4096 || c.max_queued < 1 || c.cycles_per_round < 1 || c.max_streams < 1 ||
      c.max_streams > 16)
    return ADAFAC_EINVAL;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % kAlign) return ADAFAC_EINVAL;
  const size_t head = align_up(sizeof(BatchReq) * c.max_active) + align_up(sizeof(BatchState) * c.max_active) +
                      kFlights * align_up(sizeof(ServeSeg) * size_t(kSegsPerSlot) * c.max_active);
  if (bytes < head) return ADAFAC_ENOMEM;
  adafac_server* s = new (std::nothrow) adafac_server();
  if (!s) return ADAFAC_ENOMEM;
  s->cfg = c;
  s->ws = static_cast<char*>(ws);
  s->bytes = bytes;
  s->stream = static_cast<hipStream_t>(stream);
  char* p = s->ws;
  s->d_reqs = reinterpret_cast<BatchReq*>(p);
  p += align_up(sizeof(BatchReq) * c.max_active);
  s->d_states = reinterpret_cast<BatchState*>(p);
  p += align_up(sizeof(BatchState) * c.max_active);
  s->seg_cap = kSegsPerSlot * c.max_active;
  for (int b = 0; b < kFlights; ++b) {
    s->d_segs[b] = reinterpret_cast<ServeSeg*>(p);
    p += align_up(sizeof(ServeSeg) * size_t(s->seg_cap));
  }
  s->pool_base = p;
  s->pool.reset((bytes - head) & ~(kAlign - 1));
  s->h_desc.resize(c.max_active);
  s->h_states.resize(c.max_active);
  for (int k = c.max_active - 1; k >= 0; --k) s->free_slots.push_back(k);
  s->lanes.resize(c.max_streams, nullptr);
  s->lane_busy.assign(c.max_streams, 0);
  s->lane_flight.assign(c.max_streams, 0);
  s->lane_req.assign(c.max_streams, 0);
  for (auto& l : s->lanes) {
    if (hipStreamCreateWithFlags(&l, hipStreamNonBlocking) != hipSuccess) {
      adafac_server_destroy(s);
      return ADAFAC_EDEVICE;
    }
  }
  if (hipStreamCreateWithFlags(&s->setup, hipStreamNonBlocking) != hipSuccess) {
    adafac_server_destroy(s);
    return ADAFAC_EDEVICE;
  }
  for (int b = 0; b < kFlights; ++b) {
    void* h = nullptr;
    if (hipHostMalloc(&h, sizeof(BatchState) * size_t(c.max_active), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&s->done_ev[b], hipEventDisableTiming) != hipSuccess) {
      if (h) (void)hipHostFree(h);
      adafac_server_destroy(s);
      return ADAFAC_EDEVICE;
    }
    s->snap[b] = static_cast<BatchState*>(h);
  }
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return ADAFAC_OK;
}

int adafac_server_submit(adafac_server* s, const adafac_request* q, uint64_t* ticket) {
  if (!s || !q || !ticket) return ADAFAC_EINVAL;
  if (int(s->queue.size()) >= s->cfg.max_queued) return sfail(s, ADAFAC_EAGAIN, "queue full");
  if ((q->dim != 2 && q->dim != 3) || q->l_min < 1 || q->l_min > q->l_max ||
      (q->dim == 2 && q->l_max > 9) || (q->dim == 3 && q->l_max > 6))
    return sfail(s, ADAFAC_EINVAL, "bad dimension or levels");
  if (!q->f || q->max_cycles < 1 || !(q->rel_tol >= 0.0)) return sfail(s, ADAFAC_EINVAL, "bad f, tolerance or cycle cap");
  if (q->blocks_per_axis < 0 || (q->blocks_per_axis > 0 && !q->eps)) return sfail(s, ADAFAC_EINVAL, "bad eps");
  Req r;
  r.ticket = s->next_ticket++;
  r.dim = q->dim;
  r.lmin = q->l_min;
  r.L = q->l_max;
  r.nb = q->blocks_per_axis;
  if (r.nb > 0) {
    const size_t ne = q->dim == 2 ? size_t(r.nb) * r.nb : size_t(r.nb) * r.nb * r.nb;
    r.eps.assign(q->eps, q->eps + ne);
  }
  r.f.assign(q->f, q->f + finest_vertices(q->dim, q->l_max));
  r.opts = q->opts;
  r.tol = q->rel_tol;
  r.max_cycles = q->max_cycles;
  r.res.status = ADAFAC_REQ_QUEUED;
  r.res.t_submit = now(s);
  *ticket = r.ticket;
  s->queue.push_back(r.ticket);
  s->reqs.emplace(r.ticket, std::move(r));
  prepare(s);
  return ADAFAC_OK;
}

int adafac_server_step(adafac_server* s, int* active, int* queued) {
  if (!s) return ADAFAC_EINVAL;
  // Each group (the batched launch, every lane) is harvested and relaunched as soon as its own
  // work completes; newly admitted requests start right away (lanes) or with the next batched
  // launch.  When nothing has completed yet, wait a little for the first completion.
  int rc = ADAFAC_OK;
  const double t_a = now(s);
  bool progress = false;
  for (int spin = 0; spin < 200 && !rc; ++spin) {
    bool done = false;
    rc = harvest_batched(s, false, &done);
    progress |= done;
    for (int k = 0; k < int(s->lanes.size()) && !rc; ++k) {
      rc = service_lane(s, k, false, &done);
      progress |= done;
    }
    bool busy = !s->flights.empty() || !s->background.empty();
    for (int k = 0; k < int(s->lanes.size()); ++k) busy |= s->lane_flight[k] != 0;
    for (uint64_t t : s->background)
      if (s->reqs[t].job.wait_for(std::chrono::seconds(0)) == std::future_status::ready) progress = true;
    if (progress) break;
    if (!busy) {
      // nothing on the device: wait (a little) only for a queued request's host set-up
      bool preparing = false;
      for (uint64_t t : s->queue) {
        Req& r = s->reqs[t];
        if (r.prep_started && !r.prepared) {
          preparing = r.prep.wait_for(std::chrono::seconds(0)) != std::future_status::ready;
          break;   // admission is in arrival order: the first started set-up decides
        }
      }
      if (!preparing) break;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(25));
  }
  const double t_b = now(s);
  if (!rc) rc = admit(s);
  const double t_c = now(s);
  // start newly admitted lanes and an idle batched group
  bool done = false;
  for (int k = 0; k < int(s->lanes.size()) && !rc; ++k)
    if (s->lane_busy[k] && !s->lane_flight[k]) rc = service_lane(s, k, false, &done);
  // keep kFlights batched rounds in flight: the host harvests one while the device runs the others
  for (int k = 0; k < kFlights && !rc && int(s->flights.size()) < kFlights; ++k) {
    const size_t before = s->flights.size();
    rc = launch_batched(s);
    if (s->flights.size() == before) break;
  }
  const double t_d = now(s);
  s->t_harvest += t_b - t_a;
  s->t_admit += t_c - t_b;
  s->t_launch += t_d - t_c;
  s->rounds += 1;
  if (active) *active = int(s->active.size() + s->background.size());
  if (queued) *queued = int(s->queue.size());
  return rc;
}

int adafac_server_poll(const adafac_server* s, uint64_t ticket, adafac_result* out) {
  if (!s || !out) return ADAFAC_EINVAL;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return ADAFAC_EINVAL;
  *out = it->second.res;
  return ADAFAC_OK;
}

int adafac_server_fetch(adafac_server* s, uint64_t ticket, double* u, size_t n) {
  if (!s) return ADAFAC_EINVAL;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return sfail(s, ADAFAC_EINVAL, "unknown ticket");
  Req& r = it->second;
  if (!final_status(r.res.status)) return sfail(s, ADAFAC_ESTATE, "request not finished");
  if (r.res.status != ADAFAC_REQ_FAILED) {
    if (!u || n != r.u.size()) return sfail(s, ADAFAC_EINVAL, "u: wrong size");
    std::memcpy(u, r.u.data(), sizeof(double) * n);
  }
  s->reqs.erase(it);
  return ADAFAC_OK;
}

void adafac_server_destroy(adafac_server* s) {
  if (!s) return;
  if (std::getenv("ADAFAC_SERVER_STATS"))
    std::fprintf(stderr, "adafac server: %ld steps, %lu rounds, %ld launches, host seconds harvest %.3f admit %.3f "
                 "launch %.3f (issue %.3f)\n", s->rounds, (unsigned long)s->launched, s->launches, s->t_harvest,
                 s->t_admit, s->t_launch, s->t_issue);
  (void)hipStreamSynchronize(s->stream);
  for (hipStream_t l : s->lanes)
    if (l) (void)hipStreamSynchronize(l);
  for (auto& kv : s->reqs) {
    Req& r = kv.second;
    if (r.prep_started && !r.prepared && r.prep.valid()) (void)r.prep.get();
    if (r.bg && r.job.valid()) (void)r.job.get();   // a finishing job releases its context itself
    if (r.ctx) adafac_destroy(r.ctx);
  }
  for (hipStream_t l : s->lanes)
    if (l) (void)hipStreamDestroy(l);
  if (s->setup) (void)hipStreamDestroy(s->setup);
  for (int b = 0; b < kFlights; ++b) {
    if (s->snap[b]) (void)hipHostFree(s->snap[b]);
    if (s->done_ev[b]) (void)hipEventDestroy(s->done_ev[b]);
  }
  delete s;
}

const char* adafac_server_last_error(const adafac_server* s) { return s ? s->err.c_str() : "null server"; }

}  // extern "C"
