// Host orchestration of the solver: binds a plan to the caller's device arena and enqueues the
// kernels of kernels.hip on the caller's stream (one forward pass, one backward pass and the bound
// per iteration of Alg. "Min-marginal averaging").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <initializer_list>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "solver.h"

namespace bddmp {

// ---------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------

struct Solver {
  const Plan *plan = nullptr;
  char *arena = nullptr;
  hipStream_t stream = nullptr;
  Dev D{};
  int64_t n_hist = 0;  // bounds recorded so far (the device counter holds the same count)
  int64_t iters = 0;
  // one update iteration captured as a HIP graph and replayed by iterate (the kernel arguments,
  // including the group selection, are baked in: a change of D.gsel re-captures)
  // With a wrap-around plan a run of n iterations is the first forward wave, n - 1 replays of
  // gexec_wrap (which ends with the wrap-around launch: the last backward wave and the next
  // iteration's first forward wave) and one replay of gexec (which ends with the plain last backward
  // wave), so that the state between calls is always that after whole iterations.
  bool use_graph = true;
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec = nullptr, gexec_wrap = nullptr;
  uint32_t graph_gsel = 0;
  bool costs_replaced = false;  // bddmp_solver_set_costs was called (instance constants are stale)
  // dataflow launch of the update passes (one launch per pass, see pass_kernel): on or off, the
  // arguments per pass (forward, backward) and the resident grid
  bool dataflow = false;
  PassArgs pass[2]{};
  int pass_grid[2] = {0, 0};
  // two-branch wave launches: on or off, the second stream of eager launches and of captures, and
  // the events ordering the branches (per pass: fork, join, then one per wave after its A part)
  bool pipe = false;
  hipStream_t side = nullptr, cap_side = nullptr;
  std::vector<hipEvent_t> pipe_ev;
  // wave-group launches: waves per launch (0: off), two tiles per workgroup (plans whose layers
  // are all narrow) and the bound of one dependency wait
  int group_waves = 0;
  bool group_pairs = false;
  uint32_t group_spin = 0;
  ~Solver() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (gexec_wrap) (void)hipGraphExecDestroy(gexec_wrap);
    if (cap) (void)hipStreamDestroy(cap);
    if (side) (void)hipStreamDestroy(side);
    if (cap_side) (void)hipStreamDestroy(cap_side);
    for (hipEvent_t e : pipe_ev) (void)hipEventDestroy(e);
  }
};

namespace {

int32_t hip_fail(hipError_t e, const char *what) {
  return set_error(BDDMP_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

int32_t launched(hipError_t e, const char *what) { return e == hipSuccess ? BDDMP_OK : hip_fail(e, what); }

// polls of one dependency flag before a wait of the dataflow launch gives up (each poll is a load
// and a short sleep, about a microsecond: several seconds in all, far beyond any real wait)
constexpr uint32_t kPassSpinLimit = 1u << 23;
// The same for the wave-group launch, whose waits are for tiles of the same launch that were
// dispatched before the waiting one (a quarter of a second or so), and the default waves per launch
constexpr uint32_t kGroupSpinLimit = 1u << 18;
constexpr int kGroupDefaultWaves = 4;

// BDDMP_DEVICE if a dataflow launch gave up a wait (its error word is set; the stream is
// synchronised by the caller before *err is read)
int32_t pass_error(uint32_t err) {
  if (!err) return BDDMP_OK;
  return set_error(BDDMP_DEVICE, "a dependency wait of the dataflow pass launch exceeded its bound; the results since the "
                                 "last reset are invalid");
}

// the turnaround and wrap-around launches fuse wave launches; the dataflow, two-branch and
// wave-group launches have none
bool use_turn(const Solver &S) { return S.plan->fuse_turn && !S.dataflow && !S.pipe && !S.group_waves; }
bool use_wrap(const Solver &S) { return S.plan->fuse_wrap && !S.dataflow && !S.pipe && !S.group_waves; }

// NONFINITE unless every value of the device arrays (float or double, n each) is finite; checked on
// the device, then the stream is synchronised to read the result.
template <class T>
int32_t check_finite(Solver &S, std::initializer_list<const T *> arrays, int64_t n, const char *what) {
  if (n <= 0) return BDDMP_OK;
  if (int32_t rc = launched(launch_flag_clear(S.D, S.stream), "flag_clear")) return rc;
  for (const T *p : arrays)
    if (int32_t rc = launched(launch_nonfinite(S.D, p, n, S.stream), "nonfinite check")) return rc;
  unsigned bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, S.D.flag, sizeof bad, hipMemcpyDeviceToHost, S.stream), "hipMemcpyAsync");
  HIP_TRY(hipStreamSynchronize(S.stream), "hipStreamSynchronize");
  if (bad) return set_error(BDDMP_NONFINITE, std::string(what) + " holds NaN or infinite values");
  return BDDMP_OK;
}

// Events around the pieces of an iteration for the timing entry point: the forward pass, the
// backward pass and the bound, each bracketed as a whole (cls 0, 1, 2), so that the events add no
// gap between the wave launches of a pass.
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  int cls = 0;
  int launches = 0;
};

struct Timer {
  std::vector<EventPair> *ev;
  EventPair e{};
  int32_t start(hipStream_t s, int cls) {
    if (!ev) return BDDMP_OK;
    e.cls = cls;
    HIP_TRY(hipEventCreate(&e.a), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e.b), "hipEventCreate");
    HIP_TRY(hipEventRecord(e.a, s), "hipEventRecord");
    return BDDMP_OK;
  }
  int32_t stop(hipStream_t s, int launches) {
    if (!ev) return BDDMP_OK;
    e.launches = launches;
    HIP_TRY(hipEventRecord(e.b, s), "hipEventRecord");
    ev->push_back(e);
    return BDDMP_OK;
  }
};

// Two-branch launch of an update pass: the A part of every wave on st, the B parts on the second
// stream (the capture's own while st is captured), forked from st at the start and joined back at
// the end; part B of wave w waits for the event recorded after part A of wave b_wait.
int32_t pipe_pass(Solver &S, int dir, hipStream_t st) {
  const Plan &P = *S.plan;
  const int p = dir == kFwd ? 0 : 1;
  const auto &waves = p ? P.bwd_waves : P.fwd_waves;
  const auto &split = p ? P.bsplit : P.fsplit;
  hipStream_t side = st == S.cap ? S.cap_side : S.side;
  hipEvent_t *ev = S.pipe_ev.data() + (p ? 2 + P.fwd_waves.size() : 0);
  HIP_TRY(hipEventRecord(ev[0], st), "hipEventRecord");
  HIP_TRY(hipStreamWaitEvent(side, ev[0], 0), "hipStreamWaitEvent");
  for (size_t w = 0; w < waves.size(); ++w) {
    const WaveRange &wr = waves[w];
    const int32_t mid = split[w].mid;
    const bool list = dir == kBwd && wr.list;
    if (mid > wr.tile_begin)
      if (int32_t rc = launched(launch_wave(dir, kUpdate, wr.narrow_only, list, mid - wr.tile_begin, wr.tile_begin, S.D, st),
                                "wave kernel (part A)"))
        return rc;
    HIP_TRY(hipEventRecord(ev[2 + w], st), "hipEventRecord");
    if (split[w].b_wait >= 0) HIP_TRY(hipStreamWaitEvent(side, ev[2 + split[w].b_wait], 0), "hipStreamWaitEvent");
    if (wr.tile_end > mid)
      if (int32_t rc = launched(launch_wave(dir, kUpdate, wr.narrow_only, list, wr.tile_end - mid, mid, S.D, side),
                                "wave kernel (part B)"))
        return rc;
  }
  HIP_TRY(hipEventRecord(ev[1], side), "hipEventRecord");
  HIP_TRY(hipStreamWaitEvent(st, ev[1], 0), "hipStreamWaitEvent");
  return BDDMP_OK;
}

// One pass: every wave in order, one launch per wave (plus one for the wave's big tiles if any).
// turn (plans with fuse_turn, update mode): the forward pass stops before its last wave and the
// backward pass's first launch runs that wave's forward update before its own (kTurn).
// skip_first: the forward pass starts at its second wave (the first ran already); wrap: the backward
// pass's last wave is the wrap-around launch (kWrap), which also runs the next iteration's first
// forward wave.
int32_t run_pass(Solver &S, int dir, int mode, std::vector<EventPair> *ev, hipStream_t st, bool turn = false,
                 bool skip_first = false, bool wrap = false) {
  const Plan &P = *S.plan;
  const auto &waves = dir == kFwd ? P.fwd_waves : P.bwd_waves;
  const size_t nw = waves.size() - ((turn && dir == kFwd) ? 1 : 0);
  const size_t w0 = (skip_first && dir == kFwd) ? 1 : 0;
  Timer tm{ev};
  if (int32_t rc = tm.start(st, dir)) return rc;
  if (S.dataflow && mode == kUpdate) {
    const int p = dir == kFwd ? 0 : 1;
    if (int32_t rc = launched(launch_pass(dir, P.n_general == 0, S.pass_grid[p], S.D, S.pass[p], st), "pass kernel"))
      return rc;
    return tm.stop(st, S.pass[p].n_tiles > 0 ? 1 : 0);
  }
  if (S.group_waves && mode == kUpdate) {
    // group_waves consecutive waves per launch, one workgroup per tile (per two tiles with group_pairs)
    const int p = dir == kFwd ? 0 : 1;
    int launches = 0;
    for (size_t w = 0; w < waves.size(); w += size_t(S.group_waves)) {
      const size_t wl = std::min(waves.size(), w + size_t(S.group_waves)) - 1;
      GroupArgs ga{};
      ga.trec = S.pass[p].trec;
      ga.dep_list = S.pass[p].dep_list;
      ga.flags = S.pass[p].flags;
      ga.ctl = S.pass[p].ctl;
      ga.spin_limit = S.group_spin;
      ga.t0 = waves[w].tile_begin;
      ga.t_first = waves[w].tile_end;
      ga.t_last = waves[wl].tile_begin;
      ga.t_end = waves[wl].tile_end;
      if (int32_t rc = launched(launch_group(dir, P.n_general == 0, S.group_pairs, S.D, ga, st), "wave-group kernel"))
        return rc;
      launches += ga.t_end > ga.t0 ? 1 : 0;
    }
    return tm.stop(st, launches);
  }
  if (S.pipe && mode == kUpdate) {
    if (int32_t rc = pipe_pass(S, dir, st)) return rc;
    const auto &split = dir == kFwd ? P.fsplit : P.bsplit;
    int parts = 0;
    for (size_t w = 0; w < waves.size(); ++w)
      parts += int(split[w].mid > waves[w].tile_begin) + int(waves[w].tile_end > split[w].mid);
    return tm.stop(st, parts);
  }
  for (size_t w = w0; w < nw; ++w) {
    const WaveRange &wr = waves[w];
    const int nt = wr.tile_end - wr.tile_begin;
    const int nb = wr.big_end - wr.big_begin;
    const bool list = dir == kBwd && wr.list;
    if (wrap && dir == kBwd && w + 1 == nw) {
      // same tiles as the first forward wave (the plan checked it), launched in forward numbering
      const WaveRange &f = P.fwd_waves.front();
      if (int32_t rc = launched(launch_wave(kFwd, kWrap, true, false, nt, f.tile_begin, S.D, st, wr.tile_begin),
                                "wave kernel (wrap-around)"))
        return rc;
      continue;
    }
    const int m = (turn && dir == kBwd && w == 0) ? kTurn : mode;
    if (nt > 0)
      if (int32_t rc = launched(launch_wave(dir, m, wr.narrow_only, list, nt, wr.tile_begin, S.D, st), "wave kernel"))
        return rc;
    if (nb > 0)
      if (int32_t rc = launched(launch_wave_big(dir, mode, list, nb, wr.big_begin, S.D, st), "wave kernel (big)"))
        return rc;
  }
  return tm.stop(st, int(nw - w0));
}

// the bound of the backward sweep just run, from its per-tile partials, into the history slot the
// device counter names (the caller advances the host count S.n_hist)
int32_t enqueue_lb(Solver &S, std::vector<EventPair> *ev, hipStream_t st, int which = 0) {
  const Plan &P = *S.plan;
  Timer tm{ev};
  if (int32_t rc = tm.start(st, 2)) return rc;
  if (int32_t rc = launched(launch_lb(S.D, int(P.n_lbpart + P.n_cut_parts), which, st), "bound reduction")) return rc;
  return tm.stop(st, 1);
}

// the cut roots' forward messages and the bound partials of the sub-BDDs they start (Sec. 6),
// with (update) or without the backward copy-arc update
int32_t enqueue_copy_bwd(Solver &S, int update, hipStream_t st) {
  const Plan &P = *S.plan;
  return launched(launch_copy_bwd(S.D, int(P.n_cuts), int(P.n_cut_narrow), update, int(P.n_lbpart), st),
                  "copy-arc update");
}

int32_t initial_sweep(Solver &S) {
  if (int32_t rc = run_pass(S, kBwd, kNoUpdate, nullptr, S.stream)) return rc;
  if (int32_t rc = enqueue_copy_bwd(S, 0, S.stream)) return rc;
  if (int32_t rc = enqueue_lb(S, nullptr, S.stream)) return rc;
  S.n_hist++;
  return BDDMP_OK;
}

// enqueue one iteration (forward pass, backward pass, bound) on st; with a split each pass is
// followed by its copy-arc update (Alg. "Parallel min-marginal averaging"). form 0: a whole
// iteration; with a wrap-around plan, form 1 starts at the second forward wave and ends with the
// wrap-around launch, form 2 starts at the second forward wave and ends with the plain last wave.
int32_t enqueue_iteration(Solver &S, std::vector<EventPair> *ev, hipStream_t st, int form = 0) {
  const Plan &P = *S.plan;
  if (int32_t rc = run_pass(S, kFwd, kUpdate, ev, st, use_turn(S), form != 0)) return rc;
  if (int32_t rc = launched(launch_copy_fwd(S.D, int(P.n_cuts), int(P.n_cut_narrow), st), "copy-arc update")) return rc;
  if (int32_t rc = run_pass(S, kBwd, kUpdate, ev, st, use_turn(S), false, form == 1)) return rc;
  if (int32_t rc = enqueue_copy_bwd(S, 1, st)) return rc;
  return enqueue_lb(S, ev, st);
}

int32_t one_iteration(Solver &S, std::vector<EventPair> *ev) {
  if (int32_t rc = enqueue_iteration(S, ev, S.stream)) return rc;
  S.n_hist++;
  S.iters++;
  return BDDMP_OK;
}

void drop_graph(Solver &S) {
  if (S.gexec) (void)hipGraphExecDestroy(S.gexec);
  if (S.gexec_wrap) (void)hipGraphExecDestroy(S.gexec_wrap);
  S.gexec = nullptr;
  S.gexec_wrap = nullptr;
}

// Captures one iteration's launches (in the given form) on a private stream into an executable graph.
int32_t capture_form(Solver &S, int form, hipGraphExec_t &out) {
  if (!S.cap) HIP_TRY(hipStreamCreateWithFlags(&S.cap, hipStreamNonBlocking), "hipStreamCreateWithFlags");
  HIP_TRY(hipStreamBeginCapture(S.cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  const int32_t rc = enqueue_iteration(S, nullptr, S.cap, form);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(S.cap, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
  const hipError_t ei = hipGraphInstantiate(&out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    out = nullptr;
    return hip_fail(ei, "hipGraphInstantiate");
  }
  return BDDMP_OK;
}

// The graphs iterate replays: one whole iteration, or with a wrap-around plan the two forms of
// enqueue_iteration that runs of iterations are made of.
int32_t capture_iteration(Solver &S) {
  drop_graph(S);
  const bool wrap = use_wrap(S);
  if (int32_t rc = capture_form(S, wrap ? 2 : 0, S.gexec)) return rc;
  if (wrap)
    if (int32_t rc = capture_form(S, 1, S.gexec_wrap)) {
      drop_graph(S);
      return rc;
    }
  S.graph_gsel = S.D.gsel;
  return BDDMP_OK;
}

}  // namespace

int32_t solver_bind(const Plan &P, void *arena, size_t bytes, void *stream, Solver *&out) {
  out = nullptr;
  if (P.lay.total && !arena) return set_error(BDDMP_INVALID_ARG, "null device arena");
  if (bytes < P.lay.total)
    return set_error(BDDMP_INVALID_ARG, "arena too small: need " + std::to_string(P.lay.total) + " bytes");
  if (reinterpret_cast<uintptr_t>(arena) % 256) return set_error(BDDMP_INVALID_ARG, "arena not 256-byte aligned");
  auto *S = new Solver();
  S->plan = &P;
  S->arena = static_cast<char *>(arena);
  S->stream = static_cast<hipStream_t>(stream);
  const ArenaLayout &A = P.lay;
  char *b = S->arena;
  Dev &D = S->D;
  D.meta = reinterpret_cast<const uint32_t *>(b + A.meta);
  D.child = reinterpret_cast<const int32_t *>(b + A.child);
  D.parent = reinterpret_cast<const int32_t *>(b + A.parent);
  D.lam = reinterpret_cast<float *>(b + A.lam);
  D.mf = reinterpret_cast<float *>(b + A.mf);
  D.mbc = reinterpret_cast<float *>(b + A.mbc);
  D.garcs = reinterpret_cast<const uint32_t *>(b + A.garcs);
  D.grec = P.grec.empty() ? nullptr : reinterpret_cast<const int4 *>(b + A.grec);
  D.gnb = reinterpret_cast<const int2 *>(b + A.gnb);
  D.rbeg = reinterpret_cast<const int32_t *>(b + A.rbeg);
  D.rin = reinterpret_cast<const uint32_t *>(b + A.rin);
  D.rarc = reinterpret_cast<const uint16_t *>(b + A.rarc);
  D.gsel = P.gsel;
  D.canon_of = reinterpret_cast<const int32_t *>(b + A.canon_of);
  D.layer_of = reinterpret_cast<const int32_t *>(b + A.layer_of);
  D.layer_var = reinterpret_cast<const int32_t *>(b + A.layer_var);
  D.root_slot = reinterpret_cast<const int32_t *>(b + A.root_slot);
  D.fwd_tiles = reinterpret_cast<const int32_t *>(b + A.fwd_tiles);
  D.bwd_tiles = reinterpret_cast<const int32_t *>(b + A.bwd_tiles);
  D.bwd_list = reinterpret_cast<const int32_t *>(b + A.bwd_list);
  D.fwd_big = reinterpret_cast<const int32_t *>(b + A.fwd_big);
  D.bwd_big = reinterpret_cast<const int32_t *>(b + A.bwd_big);
  D.bdd_canon_off = reinterpret_cast<const int32_t *>(b + A.bdd_canon_off);
  D.cost = reinterpret_cast<const double *>(b + A.cost);
  D.var_first = reinterpret_cast<const int32_t *>(b + A.var_first);
  D.var_nj = reinterpret_cast<const int32_t *>(b + A.var_nj);
  D.d_fresh = reinterpret_cast<float *>(b + A.d_fresh);
  D.mbuf = reinterpret_cast<float *>(b + A.mbuf);
  D.xbuf = reinterpret_cast<int8_t *>(b + A.xbuf);
  D.part = reinterpret_cast<double *>(b + A.part);
  D.lbpart = reinterpret_cast<double *>(b + A.lbpart);
  D.lb_hist = reinterpret_cast<double *>(b + A.lb_hist);
  D.scal = reinterpret_cast<double *>(b + A.scal);
  D.out0 = D.out1 = nullptr;
  D.n_bwd_tiles = int32_t(P.bwd_tiles.size() / 2);
  D.hist_n = reinterpret_cast<long long *>(b + A.scal + 64);
  D.flag = reinterpret_cast<unsigned *>(b + A.scal + 128);
  D.lbc = reinterpret_cast<double *>(b + A.scal + 80);
  D.hist_cap = P.hist_cap;
  D.inst_row = reinterpret_cast<const int32_t *>(b + A.inst_row);
  D.inst_lb = reinterpret_cast<double *>(b + A.inst_lb);
  D.cuts = reinterpret_cast<const int4 *>(b + A.cuts);
  D.cut_slots = reinterpret_cast<const int4 *>(b + A.cut_slots);
  D.cut_live = reinterpret_cast<const int32_t *>(b + A.cut_live);
  D.cut_rb = reinterpret_cast<const int32_t *>(b + A.cut_rb);
  D.cut_arc = reinterpret_cast<const uint16_t *>(b + A.cut_arc);
  D.mu_in = reinterpret_cast<float *>(b + A.mu_in);
  D.dfw = reinterpret_cast<float *>(b + A.dfw);
  D.dbw = reinterpret_cast<float *>(b + A.dbw);
  D.cut_e = reinterpret_cast<float *>(b + A.cut_e);
  D.inst_cut = reinterpret_cast<const int32_t *>(b + A.inst_cut);
  D.inst_cut_idx = reinterpret_cast<const int32_t *>(b + A.inst_cut_idx);
  D.exit_rec = P.exit_rec.empty() ? nullptr : reinterpret_cast<const int32_t *>(b + A.exit_rec);
  D.fgt = reinterpret_cast<const int2 *>(b + A.fgt);
  D.bgt = reinterpret_cast<const int2 *>(b + A.bgt);
  D.fgm = reinterpret_cast<const uint8_t *>(b + A.fgm);
  D.bgm = reinterpret_cast<const uint8_t *>(b + A.bgm);
  D.gamma = P.split_gamma;
  for (int p = 0; p < 2; ++p) {
    PassArgs &pa = S->pass[p];
    pa.trec = reinterpret_cast<const int4 *>(b + (p ? A.btrec : A.ftrec));
    pa.dep_list = reinterpret_cast<const int32_t *>(b + (p ? A.bdep_list : A.fdep_list));
    pa.qptr = reinterpret_cast<const int32_t *>(b + (p ? A.bqptr : A.fqptr));
    pa.qtile = reinterpret_cast<const int32_t *>(b + (p ? A.bqtile : A.fqtile));
    pa.n_queues = P.n_groups;
    pa.flags = reinterpret_cast<uint32_t *>(b + (p ? A.bflag : A.fflag));
    pa.ctl = reinterpret_cast<uint32_t *>(b + A.pctl) + kPassCtlWords * p;
    pa.n_tiles = int32_t((p ? P.btinfo : P.ftinfo).size());
    pa.chunk = 1;
    pa.spin_limit = kPassSpinLimit;
  }

  auto up = [&](size_t off, const void *src, size_t nbytes) -> hipError_t {
    if (!nbytes) return hipSuccess;
    return hipMemcpyAsync(b + off, src, nbytes, hipMemcpyHostToDevice, S->stream);
  };
  const hipError_t errs[] = {
      up(A.meta, P.meta.data(), 4 * P.meta.size()),
      up(A.child, P.child.data(), 4 * P.child.size()),
      up(A.parent, P.parent.data(), 4 * P.parent.size()),
      up(A.garcs, P.garcs.data(), 4 * P.garcs.size()),
      up(A.grec, P.grec.data(), 4 * P.grec.size()),
      up(A.gnb, P.gnb.data(), 4 * P.gnb.size()),
      up(A.rbeg, P.rbeg.data(), 4 * P.rbeg.size()),
      up(A.rin, P.rin.data(), 4 * P.rin.size()),
      up(A.rarc, P.rarc.data(), 2 * P.rarc.size()),
      up(A.canon_of, P.canon_of.data(), 4 * P.canon_of.size()),
      up(A.layer_of, P.layer_of.data(), 4 * P.layer_of.size()),
      up(A.layer_var, P.layer_var.data(), 4 * P.layer_var.size()),
      up(A.root_slot, P.root_slot.data(), 4 * P.root_slot.size()),
      up(A.fwd_tiles, P.fwd_tiles.data(), 4 * P.fwd_tiles.size()),
      up(A.bwd_tiles, P.bwd_tiles.data(), 4 * P.bwd_tiles.size()),
      up(A.bwd_list, P.bwd_list.data(), 4 * P.bwd_list.size()),
      up(A.fwd_big, P.fwd_big.data(), 4 * P.fwd_big.size()),
      up(A.bwd_big, P.bwd_big.data(), 4 * P.bwd_big.size()),
      up(A.bdd_canon_off, P.bdd_canon_off.data(), 4 * P.bdd_canon_off.size()),
      up(A.cost, P.cost.data(), 8 * P.cost.size()),
      up(A.var_first, P.var_first.data(), 4 * P.var_first.size()),
      up(A.var_nj, P.var_nj.data(), 4 * P.var_nj.size()),
      up(A.inst_row, P.inst_row32.data(), 4 * P.inst_row32.size()),
      up(A.cuts, P.cuts.data(), 4 * P.cuts.size()),
      up(A.cut_slots, P.cut_slots.data(), 4 * P.cut_slots.size()),
      up(A.cut_live, P.cut_live.data(), 4 * P.cut_live.size()),
      up(A.cut_rb, P.cut_rb.data(), 4 * P.cut_rb.size()),
      up(A.inst_cut, P.inst_cut.data(), 4 * P.inst_cut.size()),
      up(A.inst_cut_idx, P.inst_cut_idx.data(), 4 * P.inst_cut_idx.size()),
      up(A.exit_rec, P.exit_rec.data(), 4 * P.exit_rec.size()),
      up(A.cut_arc, P.cut_arc.data(), 2 * P.cut_arc.size()),
      up(A.fdep_list, P.fdep_list.data(), 4 * P.fdep_list.size()),
      up(A.bdep_list, P.bdep_list.data(), 4 * P.bdep_list.size()),
      up(A.ftrec, P.ftrec.data(), 4 * P.ftrec.size()),
      up(A.btrec, P.btrec.data(), 4 * P.btrec.size()),
      up(A.fqptr, P.fqptr.data(), 4 * P.fqptr.size()),
      up(A.fqtile, P.fqtile.data(), 4 * P.fqtile.size()),
      up(A.bqptr, P.bqptr.data(), 4 * P.bqptr.size()),
      up(A.bqtile, P.bqtile.data(), 4 * P.bqtile.size()),
      up(A.fgt, P.fgt.data(), 4 * P.fgt.size()),
      up(A.bgt, P.bgt.data(), 4 * P.bgt.size()),
      up(A.fgm, P.fgm.data(), P.fgm.size()),
      up(A.bgm, P.bgm.data(), P.bgm.size()),
  };
  for (hipError_t e : errs)
    if (e != hipSuccess) {
      delete S;
      return hip_fail(e, "hipMemcpyAsync (upload)");
    }
  // dataflow launch state: flags and control words start at zero (generation 0, no launch yet)
  for (const auto &z : {std::make_pair(A.fflag, P.ftinfo.size()), std::make_pair(A.bflag, P.btinfo.size()),
                        std::make_pair(A.pctl, 2 * size_t(kPassCtlWords))})
    if (int32_t rc = launched(launch_fill(reinterpret_cast<float *>(b + z.first), 0.0f, int(z.second), S->stream), "fill")) {
      delete S;
      return rc;
    }
  if (const int32_t rc = solver_reset(*S)) {
    delete S;
    return rc;
  }
  out = S;
  return BDDMP_OK;
}

// Initialisation of Alg. "Min-marginal averaging": lambda^j_i = c_i / |J_i|, forward messages
// +inf except the roots (0; padding slots stay +inf), and the initial backward sweep that fills
// every backward message.
int32_t solver_reset(Solver &S) {
  const Plan &P = *S.plan;
  const int nslots = int(P.S + 4);
  if (int32_t rc = launched(launch_fill(S.D.mf, INFINITY, nslots, S.stream), "fill")) return rc;
  const int ncslots = int(P.Sc + 4);
  if (int32_t rc = launched(launch_fill(S.D.mbc, INFINITY, ncslots, S.stream), "fill")) return rc;
  if (int32_t rc = launched(launch_init_lambda(S.D, int(P.I), S.stream), "init_lambda")) return rc;
  if (int32_t rc = launched(launch_root_zero(S.D, P.m, S.stream), "root_zero")) return rc;
  if (int32_t rc = launched(launch_copy_init(S.D, int(P.n_cuts), S.stream), "copy_init")) return rc;
  // bound partials: tiles without a root level never write theirs, which stay zero
  const int nlb = int(2 * (P.n_lbpart + P.n_cut_parts + 1));
  if (int32_t rc = launched(launch_fill(reinterpret_cast<float *>(S.D.lbpart), 0.0f, nlb, S.stream), "fill")) return rc;
  if (int32_t rc = launched(launch_set_counter(S.D, S.n_hist, S.stream), "set_counter")) return rc;
  // the dataflow launches' error words (generations and tickets stay as they are)
  for (int p = 0; p < 2; ++p)
    if (int32_t rc = launched(launch_fill(reinterpret_cast<float *>(S.pass[p].ctl + kPassErr), 0.0f, 1, S.stream), "fill"))
      return rc;
  if (int32_t rc = launched(launch_free_const(S.D, P.n, 1.0f, S.stream), "free_const")) return rc;
  S.iters = 0;
  return initial_sweep(S);
}

int32_t solver_iterate(Solver &S, int32_t n) {
  if (n < 0) return set_error(BDDMP_INVALID_ARG, "negative iteration count");
  if (S.use_graph && n > 0) {
    const Plan &P = *S.plan;
    const bool wrap = use_wrap(S);
    if (!S.gexec || (wrap && !S.gexec_wrap) || S.graph_gsel != S.D.gsel)
      if (int32_t rc = capture_iteration(S)) return rc;
    if (wrap) {
      // the first forward wave, then n - 1 iterations that end one wave into the next, then one
      // that ends with the plain last backward wave
      const WaveRange &f = P.fwd_waves.front();
      if (int32_t rc = launched(launch_wave(kFwd, kUpdate, true, false, f.tile_end - f.tile_begin, f.tile_begin, S.D,
                                            S.stream),
                                "wave kernel"))
        return rc;
    }
    for (int32_t t = 0; t < n; ++t) {
      HIP_TRY(hipGraphLaunch((wrap && t + 1 < n) ? S.gexec_wrap : S.gexec, S.stream), "hipGraphLaunch");
      S.n_hist++;
      S.iters++;
    }
    return BDDMP_OK;
  }
  for (int32_t t = 0; t < n; ++t)
    if (int32_t rc = one_iteration(S, nullptr)) return rc;
  return BDDMP_OK;
}

int32_t solver_iterate_until(Solver &S, int32_t max_iters, double rel, int32_t every, int32_t *done, int32_t *at,
                             double *lb) {
  const Plan &P = *S.plan;
  if (max_iters < 0 || !(rel >= 0.0) || every < 1 || every >= P.hist_cap || !done || !at || !lb)
    return set_error(BDDMP_INVALID_ARG, "max_iters >= 0, min_rel_impr >= 0, 1 <= check_every < hist_cap, non-null outputs");
  std::vector<double> b(size_t(every) + 1);
  int32_t got = 0;
  if (int32_t rc = solver_lb_history(S, b.data(), 1, &got)) return rc;
  double prev = got ? b[0] : 0.0;
  int32_t n = 0;
  *at = -1;
  while (n < max_iters && *at < 0) {
    const int32_t k = std::min(every, max_iters - n);
    if (int32_t rc = solver_iterate(S, k)) return rc;
    if (int32_t rc = solver_lb_history(S, b.data(), k, &got)) return rc;
    for (int32_t q = 0; q < got && *at < 0; ++q) {
      if (b[size_t(q)] - prev < rel * std::max(std::fabs(b[size_t(q)]), 1.0)) *at = n + q + 1;
      prev = b[size_t(q)];
    }
    prev = b[size_t(got - 1)];
    n += k;
  }
  *done = n;
  *lb = prev;
  return BDDMP_OK;
}

int32_t solver_set_graphs(Solver &S, int32_t enable) {
  S.use_graph = enable != 0;
  if (!S.use_graph) drop_graph(S);
  return BDDMP_OK;
}

int32_t solver_lower_bound(Solver &S, double *lb, double *residual, double *any_lambda_bound) {
  const Plan &P = *S.plan;
  double h = 0.0, sc[2] = {0.0, 0.0};
  const int slot = int((S.n_hist - 1) % P.hist_cap);
  HIP_TRY(hipMemcpyAsync(&h, S.D.lb_hist + slot, 8, hipMemcpyDeviceToHost, S.stream), "hipMemcpyAsync");
  uint32_t err[2] = {0u, 0u};
  for (int p = 0; p < 2; ++p)
    HIP_TRY(hipMemcpyAsync(err + p, S.pass[p].ctl + kPassErr, 4, hipMemcpyDeviceToHost, S.stream), "hipMemcpyAsync");
  if ((residual || any_lambda_bound) && P.n > 0) {
    if (int32_t rc = launched(launch_residual(S.D, P.n, S.stream), "residual")) return rc;
    HIP_TRY(hipMemcpyAsync(sc, S.D.scal, 16, hipMemcpyDeviceToHost, S.stream), "hipMemcpyAsync");
  }
  HIP_TRY(hipStreamSynchronize(S.stream), "hipStreamSynchronize");
  if (int32_t rc = pass_error(err[0] | err[1])) return rc;
  if (lb) *lb = h;
  if (residual) *residual = sc[0];
  if (any_lambda_bound) *any_lambda_bound = h + sc[1];
  if (!std::isfinite(h)) return set_error(BDDMP_NONFINITE, std::isnan(h) ? "lower bound is NaN" : "lower bound is infinite");
  return BDDMP_OK;
}

int32_t solver_instance_bounds(Solver &S, double *lb_host, int32_t n) {
  const Plan &P = *S.plan;
  const int32_t n_inst = int32_t(P.inst_lb_const.size());
  if (S.costs_replaced) return set_error(BDDMP_BAD_STATE, "instance bounds use the plan's costs; costs were replaced");
  if (!lb_host || n != n_inst)
    return set_error(BDDMP_INVALID_ARG, "lb array must hold n_instances = " + std::to_string(n_inst) + " values");
  if (int32_t rc = launched(launch_instance_bounds(S.D, n_inst, S.stream), "instance_bounds")) return rc;
  HIP_TRY(hipMemcpyAsync(lb_host, S.D.inst_lb, 8 * size_t(n_inst), hipMemcpyDeviceToHost, S.stream), "hipMemcpyAsync");
  HIP_TRY(hipStreamSynchronize(S.stream), "hipStreamSynchronize");
  for (int32_t k = 0; k < n_inst; ++k) lb_host[k] += P.inst_lb_const[size_t(k)];
  return BDDMP_OK;
}

int32_t solver_lb_history(Solver &S, double *out, int32_t cap, int32_t *n_out) {
  const Plan &P = *S.plan;
  const int64_t have = std::min<int64_t>(S.n_hist, P.hist_cap);
  const int64_t cnt = std::min<int64_t>(have, cap);
  std::vector<double> ring(size_t(P.hist_cap));
  HIP_TRY(hipMemcpyAsync(ring.data(), S.D.lb_hist, 8 * size_t(P.hist_cap), hipMemcpyDeviceToHost, S.stream),
          "hipMemcpyAsync");
  uint32_t err[2] = {0u, 0u};
  for (int p = 0; p < 2; ++p)
    HIP_TRY(hipMemcpyAsync(err + p, S.pass[p].ctl + kPassErr, 4, hipMemcpyDeviceToHost, S.stream), "hipMemcpyAsync");
  HIP_TRY(hipStreamSynchronize(S.stream), "hipStreamSynchronize");
  if (int32_t rc = pass_error(err[0] | err[1])) return rc;
  for (int64_t q = 0; q < cnt; ++q) {
    const int64_t idx = S.n_hist - cnt + q;
    out[q] = ring[size_t(idx % P.hist_cap)];
  }
  if (n_out) *n_out = int32_t(cnt);
  return BDDMP_OK;
}

int32_t solver_min_marginals(Solver &S, float *m0, float *m1) {
  S.D.out0 = m0;
  S.D.out1 = m1;
  const int32_t rc = run_pass(S, kFwd, kExtract, nullptr, S.stream);
  S.D.out0 = S.D.out1 = nullptr;
  return rc;
}

int32_t solver_get_lambda(Solver &S, float *lam) {
  const Plan &P = *S.plan;
  return launched(launch_lambda_out(S.D, lam, int(P.I), S.stream), "lambda_out");
}

int32_t solver_set_lambda(Solver &S, const float *lam) {
  const Plan &P = *S.plan;
  if (int32_t rc = check_finite<float>(S, {lam}, P.I, "the multipliers")) return rc;
  if (int32_t rc = launched(launch_lambda_in(S.D, lam, int(P.I), S.stream), "lambda_in")) return rc;
  return initial_sweep(S);
}

int32_t solver_copy_duals(Solver &S, bool out, float *mu_bar, float *mu, float *dfw, float *dbw) {
  const Plan &P = *S.plan;
  if (!out && (!mu_bar || !mu || !dfw || !dbw) && P.n_copy)
    return set_error(BDDMP_INVALID_ARG, "setting the copy state needs all four arrays");
  if (!out)
    if (int32_t rc = check_finite<float>(S, {mu_bar, mu, dfw, dbw}, P.n_copy, "the copy-arc state")) return rc;
  if (int32_t rc = launched(launch_copy_io(S.D, int(P.n_cuts), out, mu_bar, mu, dfw, dbw, S.stream), "copy state"))
    return rc;
  return out ? BDDMP_OK : initial_sweep(S);
}

int32_t solver_round_primal(Solver &S, float *M_dev, int8_t *x_host, double *obj, int64_t *nviol) {
  const Plan &P = *S.plan;
  if (int32_t rc = solver_min_marginals(S, nullptr, nullptr)) return rc;
  double sc[2] = {0.0, 0.0};
  if (int32_t rc = launched(launch_round(S.D, P.n, P.m, S.stream), "rounding")) return rc;
  if (M_dev && P.n)
    HIP_TRY(hipMemcpyAsync(M_dev, S.D.mbuf, 4 * size_t(P.n), hipMemcpyDeviceToDevice, S.stream), "hipMemcpyAsync");
  if (x_host && P.n)
    HIP_TRY(hipMemcpyAsync(x_host, S.D.xbuf, size_t(P.n), hipMemcpyDeviceToHost, S.stream), "hipMemcpyAsync");
  HIP_TRY(hipMemcpyAsync(sc, S.D.scal + 2, 16, hipMemcpyDeviceToHost, S.stream), "hipMemcpyAsync");
  HIP_TRY(hipStreamSynchronize(S.stream), "hipStreamSynchronize");
  if (obj) *obj = sc[0];
  if (nviol) *nviol = int64_t(sc[1]);
  return BDDMP_OK;
}

int32_t solver_set_launch(Solver &S, int32_t mode, int32_t chunk) {
  const Plan &P = *S.plan;
  if (mode < 0 || mode > 4)
    return set_error(BDDMP_INVALID_ARG, "launch mode must be 0 (wave launches), 1 (dataflow), 2 (two-branch waves), "
                                        "3 (wave groups) or 4 (wave groups, two tiles per workgroup)");
  if (chunk < 0 || chunk > 4096) return set_error(BDDMP_INVALID_ARG, "chunk must be 0 (default) .. 4096");
  if (mode != 0 && !P.pers_ok)
    return set_error(BDDMP_INVALID_ARG, "the plan has a variable in more than 256 rows: no dataflow or two-branch launch");
  if (mode == 4 && P.n_general != 0)
    return set_error(BDDMP_INVALID_ARG, "two tiles per workgroup (launch mode 4) need a plan whose layers are all narrow");
  if (mode == 2) {
    if (!S.side) HIP_TRY(hipStreamCreateWithFlags(&S.side, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    if (!S.cap_side) HIP_TRY(hipStreamCreateWithFlags(&S.cap_side, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    const size_t n_ev = 4 + P.fwd_waves.size() + P.bwd_waves.size();
    while (S.pipe_ev.size() < n_ev) {
      hipEvent_t e = nullptr;
      HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreateWithFlags");
      S.pipe_ev.push_back(e);
    }
  }
  if (mode == 1) {
    int dev = 0, ncu = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
    for (int p = 0; p < 2; ++p) {
      int per_cu = 0;
      HIP_TRY(pass_blocks_per_cu(p ? kBwd : kFwd, P.n_general == 0, &per_cu), "hipOccupancyMaxActiveBlocksPerMultiprocessor");
      PassArgs &pa = S.pass[p];
      pa.chunk = chunk ? chunk : 1;
      pa.spin_limit = kPassSpinLimit;
      if (const char *e = std::getenv("BDDMP_PASS_SPIN_LIMIT")) pa.spin_limit = uint32_t(std::strtoul(e, nullptr, 10));
      const auto &qptr = p ? P.bqptr : P.fqptr;
      int64_t n_chunks = 0;
      for (size_t g = 0; g + 1 < qptr.size(); ++g) n_chunks += (int64_t(qptr[g + 1] - qptr[g]) + pa.chunk - 1) / pa.chunk;
      S.pass_grid[p] = int(std::min<int64_t>(n_chunks, int64_t(std::max(per_cu, 1)) * std::max(ncu, 1)));
    }
  }
  S.dataflow = mode == 1;
  S.pipe = mode == 2;
  S.group_waves = mode == 3 || mode == 4 ? (chunk ? chunk : kGroupDefaultWaves) : 0;
  S.group_pairs = mode == 4;
  S.group_spin = kGroupSpinLimit;
  if (const char *e = std::getenv("BDDMP_PASS_SPIN_LIMIT")) S.group_spin = uint32_t(std::strtoul(e, nullptr, 10));
  drop_graph(S);
  return BDDMP_OK;
}

int32_t solver_get_launch(const Solver &S, int32_t *mode, int32_t *chunk) {
  if (mode) *mode = S.dataflow ? 1 : (S.pipe ? 2 : (S.group_waves ? (S.group_pairs ? 4 : 3) : 0));
  if (chunk) *chunk = S.group_waves ? S.group_waves : S.pass[0].chunk;
  return BDDMP_OK;
}

int32_t solver_set_groups(Solver &S, const int32_t *lanes) {
  if (!lanes) return set_error(BDDMP_INVALID_ARG, "null lanes");
  uint32_t g = 0;
  for (int c = 0; c < kWidthClasses; ++c) {
    uint32_t code = 0;
    if (!gsel_code(lanes[c], code)) return set_error(BDDMP_INVALID_ARG, "lanes must be 0 or powers of two up to 64");
    g |= code << (4 * c);
  }
  S.D.gsel = g;
  return BDDMP_OK;
}

int32_t solver_get_groups(const Solver &S, int32_t *lanes) {
  if (!lanes) return set_error(BDDMP_INVALID_ARG, "null lanes");
  for (int c = 0; c < kWidthClasses; ++c) {
    const uint32_t code = (S.D.gsel >> (4 * c)) & 0xFu;
    lanes[c] = code == kGselFlat ? 0 : 1 << code;
  }
  return BDDMP_OK;
}

// Coordinate search over the general-layer path: for each width class that has tiles, time iters
// iterations with the node-parallel path and with groups of every power of two from 1 to 64 lanes
// (the other classes at their current choice) and keep the fastest. Every choice computes the same values (min is exact), so only
// time differs; the solver advances by the iterations run.
int32_t solver_autotune(Solver &S, int32_t iters, int32_t *lanes) {
  const Plan &P = *S.plan;
  if (iters < 1) return set_error(BDDMP_INVALID_ARG, "iters must be positive");
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a), "hipEventCreate");
  HIP_TRY(hipEventCreate(&b), "hipEventCreate");
  int32_t rc = BDDMP_OK;
  for (int c = 0; c < kWidthClasses && !rc; ++c) {
    if (!P.class_tiles[c]) continue;
    uint32_t best_lg = (S.D.gsel >> (4 * c)) & 0xFu;
    float best = INFINITY;
    for (uint32_t lg : {kGselFlat, 0u, 1u, 2u, 3u, 4u, 5u, 6u}) {
      if (rc) break;
      S.D.gsel = (S.D.gsel & ~(0xFu << (4 * c))) | (lg << (4 * c));
      hipError_t e = hipEventRecord(a, S.stream);
      if (e == hipSuccess) rc = solver_iterate(S, iters);
      if (e == hipSuccess) e = hipEventRecord(b, S.stream);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (e != hipSuccess && !rc) rc = hip_fail(e, "autotune timing");
      if (!rc && ms < best) {
        best = ms;
        best_lg = lg;
      }
    }
    S.D.gsel = (S.D.gsel & ~(0xFu << (4 * c))) | (best_lg << (4 * c));
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc) return rc;
  return lanes ? solver_get_groups(S, lanes) : BDDMP_OK;
}

int32_t solver_time_kernels(Solver &S, int32_t n, bddmp_kernel_times *out) {
  const Plan &P = *S.plan;
  std::vector<EventPair> ev;
  ev.reserve(size_t(n) * 3);
  int32_t rc = BDDMP_OK;
  for (int32_t t = 0; t < n && !rc; ++t) rc = one_iteration(S, &ev);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (!rc) {
    HIP_TRY(hipEventCreate(&t0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&t1), "hipEventCreate");
    HIP_TRY(hipEventRecord(t0, S.stream), "hipEventRecord");
    rc = solver_iterate(S, n);
    HIP_TRY(hipEventRecord(t1, S.stream), "hipEventRecord");
  }
  const hipError_t se = hipStreamSynchronize(S.stream);
  bddmp_kernel_times r{};
  for (const EventPair &e : ev) {
    float ms = 0.0f;
    if (!rc && se == hipSuccess) (void)hipEventElapsedTime(&ms, e.a, e.b);
    if (e.cls == 0) {
      r.fwd_ms += ms;
      r.fwd_launches += e.launches;
    } else if (e.cls == 1) {
      r.bwd_ms += ms;
      r.bwd_launches += e.launches;
    } else {
      r.lb_ms += ms;
      r.lb_launches += e.launches;
    }
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  if (!rc && se == hipSuccess && t0) {
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    r.iter_ms = n ? ms / n : 0.0;
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (rc) return rc;
  if (se != hipSuccess) return hip_fail(se, "hipStreamSynchronize");
  // model bytes per pass; with a fused turnaround the last forward wave's share is timed with the
  // backward pass
  const double pass_bytes = 20.0 * double(P.N) + 8.0 * double(P.I);
  const double turn_bytes =
      use_turn(S) ? 20.0 * double(P.fwd_waves.back().nodes) + 8.0 * double(P.fwd_waves.back().layers) : 0.0;
  r.fwd_bytes = (pass_bytes - turn_bytes) * n;
  r.bwd_bytes = (pass_bytes + turn_bytes) * n;
  *out = r;
  return BDDMP_OK;
}

// ---------------------------------------------------------------------------------------------
// smoothed variant and its derivative
// ---------------------------------------------------------------------------------------------

namespace {

struct SmoothWs {
  float *ckpt, *lam_mid, *mbt, *glam, *gmf, *gmb;
  size_t total;
};

SmoothWs smooth_layout(const Plan &P, int32_t T, char *base) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t I = size_t(std::max<int64_t>(P.I, 1)), S = size_t(P.S + 4), Sc = size_t(P.Sc + 4);
  SmoothWs w{};
  size_t off = 0;
  auto take = [&](size_t floats) {
    float *p = reinterpret_cast<float *>(base + off);
    off = al(off + 4 * floats);
    return p;
  };
  w.ckpt = take(I * size_t(T + 1));
  w.lam_mid = take(I);
  w.mbt = take(Sc);
  w.glam = take(I);
  w.gmf = take(S);
  w.gmb = take(Sc);
  w.total = off;
  return w;
}

int32_t smooth_pass(Solver &S, int dir, int mode, bool adjoint, const SmoothArgs &A) {
  const Plan &P = *S.plan;
  const auto &waves = dir == kFwd ? P.fwd_waves : P.bwd_waves;
  const int nw = int(waves.size());
  for (int q = 0; q < nw; ++q) {
    const WaveRange &wr = waves[size_t(adjoint ? nw - 1 - q : q)];
    const int nt = wr.tile_end - wr.tile_begin;
    const bool list = dir == kBwd && wr.list;
    if (int32_t rc = launched(launch_smooth_wave(dir, mode, adjoint, list, nt, wr.tile_begin, S.D, A, S.stream),
                              adjoint ? "smoothed adjoint wave" : "smoothed wave"))
      return rc;
  }
  return BDDMP_OK;
}

int32_t smooth_check(Solver &S, float alpha, int32_t T, void *ws, size_t bytes, SmoothWs &w) {
  const Plan &P = *S.plan;
  if (!(alpha > 0.0f) || !std::isfinite(alpha)) return set_error(BDDMP_INVALID_ARG, "alpha must be positive");
  if (T < 0) return set_error(BDDMP_INVALID_ARG, "negative iteration count");
  if (!P.fwd_big.empty() || !P.bwd_big.empty())
    return set_error(BDDMP_INVALID_ARG, "the smoothed passes take variables in at most 256 rows");
  if (P.n_cuts) return set_error(BDDMP_INVALID_ARG, "the smoothed passes run on unsplit plans");
  w = smooth_layout(P, T, static_cast<char *>(ws));
  if (!ws || bytes < w.total) return set_error(BDDMP_INVALID_ARG, "workspace too small: need " + std::to_string(w.total));
  if (reinterpret_cast<uintptr_t>(ws) % 256) return set_error(BDDMP_INVALID_ARG, "workspace not 256-byte aligned");
  return BDDMP_OK;
}

hipError_t copy_f(float *dst, const float *src, int64_t n, hipStream_t s) {
  return n > 0 ? hipMemcpyAsync(dst, src, 4 * size_t(n), hipMemcpyDeviceToDevice, s) : hipSuccess;
}

}  // namespace

int32_t solver_smooth_workspace(const Plan &P, int32_t T, size_t *bytes) {
  if (T < 0 || !bytes) return set_error(BDDMP_INVALID_ARG, "negative iteration count or null out");
  *bytes = smooth_layout(P, T, nullptr).total;
  return BDDMP_OK;
}

// Smoothed Alg. "Min-marginal averaging" from lambda = c / |J_i|: the smoothed initial sweep and T
// smoothed iterations, each bound LB_alpha appended to the history; lambda after each iteration
// kept in the workspace (checkpoint t = lambda after t iterations, in storage order).
int32_t solver_smooth_run(Solver &S, float alpha, int32_t T, void *ws, size_t bytes) {
  const Plan &P = *S.plan;
  SmoothWs w{};
  if (int32_t rc = smooth_check(S, alpha, T, ws, bytes, w)) return rc;
  SmoothArgs A{alpha, 0.0f, nullptr, nullptr, nullptr, w.glam, w.gmf, w.gmb};
  const int nslots = int(P.S + 4), ncslots = int(P.Sc + 4);
  if (int32_t rc = launched(launch_fill(S.D.mf, INFINITY, nslots, S.stream), "fill")) return rc;
  if (int32_t rc = launched(launch_fill(S.D.mbc, INFINITY, ncslots, S.stream), "fill")) return rc;
  if (int32_t rc = launched(launch_init_lambda(S.D, int(P.I), S.stream), "init_lambda")) return rc;
  if (int32_t rc = launched(launch_root_zero(S.D, P.m, S.stream), "root_zero")) return rc;
  if (int32_t rc = launched(launch_free_const(S.D, P.n, alpha, S.stream), "free_const")) return rc;
  if (int32_t rc = smooth_pass(S, kBwd, kNoUpdate, false, A)) return rc;
  if (int32_t rc = enqueue_lb(S, nullptr, S.stream, 1)) return rc;
  S.n_hist++;
  S.iters = 0;
  HIP_TRY(copy_f(w.ckpt, S.D.lam, P.I, S.stream), "hipMemcpyAsync");
  for (int32_t t = 0; t < T; ++t) {
    if (int32_t rc = smooth_pass(S, kFwd, kUpdate, false, A)) return rc;
    if (int32_t rc = smooth_pass(S, kBwd, kUpdate, false, A)) return rc;
    if (int32_t rc = enqueue_lb(S, nullptr, S.stream, 1)) return rc;
    S.n_hist++;
    S.iters++;
    HIP_TRY(copy_f(w.ckpt + size_t(std::max<int64_t>(P.I, 1)) * size_t(t + 1), S.D.lam, P.I, S.stream), "hipMemcpyAsync");
  }
  return BDDMP_OK;
}

// d LB_alpha(T) / d c times dlb into grad (device float [n], variable order), by reverse
// accumulation over the checkpoints of solver_smooth_run (same alpha, T and workspace). Each
// iteration is recomputed from its checkpoint (the initial sweep of lambda_t gives the backward
// messages it started from), then its backward and forward passes are undone wave by wave in
// reverse order. Leaves the solver at lambda_T with its backward messages.
int32_t solver_smooth_grad(Solver &S, float alpha, int32_t T, void *ws, size_t bytes, double dlb, float *grad) {
  const Plan &P = *S.plan;
  SmoothWs w{};
  if (int32_t rc = smooth_check(S, alpha, T, ws, bytes, w)) return rc;
  if (!grad && P.n > 0) return set_error(BDDMP_INVALID_ARG, "null gradient output");
  const size_t I1 = size_t(std::max<int64_t>(P.I, 1));
  const int nslots = int(P.S + 4), ncslots = int(P.Sc + 4);
  if (int32_t rc = launched(launch_fill(w.glam, 0.0f, int(I1), S.stream), "fill")) return rc;
  if (int32_t rc = launched(launch_fill(w.gmf, 0.0f, nslots, S.stream), "fill")) return rc;
  if (int32_t rc = launched(launch_fill(w.gmb, 0.0f, ncslots, S.stream), "fill")) return rc;
  SmoothArgs A{alpha, 0.0f, nullptr, nullptr, w.mbt, w.glam, w.gmf, w.gmb};
  for (int32_t t = T - 1; t >= 0; --t) {
    const float *ck = w.ckpt + I1 * size_t(t);
    HIP_TRY(copy_f(S.D.lam, ck, P.I, S.stream), "hipMemcpyAsync");
    if (int32_t rc = smooth_pass(S, kBwd, kNoUpdate, false, A)) return rc;
    HIP_TRY(copy_f(w.mbt, S.D.mbc, ncslots, S.stream), "hipMemcpyAsync");
    if (int32_t rc = smooth_pass(S, kFwd, kUpdate, false, A)) return rc;
    HIP_TRY(copy_f(w.lam_mid, S.D.lam, P.I, S.stream), "hipMemcpyAsync");
    if (int32_t rc = smooth_pass(S, kBwd, kUpdate, false, A)) return rc;
    SmoothArgs AB = A;
    AB.root_seed = t == T - 1 ? float(dlb) : 0.0f;
    AB.lam_prev = w.lam_mid;
    if (int32_t rc = smooth_pass(S, kBwd, kUpdate, true, AB)) return rc;
    SmoothArgs AF = A;
    AF.lam_prev = ck;
    AF.lam_upd = w.lam_mid;
    if (int32_t rc = smooth_pass(S, kFwd, kUpdate, true, AF)) return rc;
  }
  HIP_TRY(copy_f(S.D.lam, w.ckpt, P.I, S.stream), "hipMemcpyAsync");
  if (int32_t rc = smooth_pass(S, kBwd, kNoUpdate, false, A)) return rc;
  SmoothArgs A0 = A;
  A0.root_seed = T == 0 ? float(dlb) : 0.0f;
  if (int32_t rc = smooth_pass(S, kBwd, kNoUpdate, true, A0)) return rc;
  if (int32_t rc = launched(launch_smooth_grad(S.D, A, P.n, float(dlb), grad, S.stream), "smooth_grad")) return rc;
  HIP_TRY(copy_f(S.D.lam, w.ckpt + I1 * size_t(T), P.I, S.stream), "hipMemcpyAsync");
  return smooth_pass(S, kBwd, kNoUpdate, false, A);
}

// ---------------------------------------------------------------------------------------------
// smoothed gradient without a caller workspace (for callers that cannot allocate device memory)
// ---------------------------------------------------------------------------------------------

namespace {

// The workspace of solver_smooth_grad_noalloc: a fixed array in the code object, one copy per GPU,
// allocated when the library's code is loaded on that GPU and held until the process ends. Calls on
// one GPU share it. In host code `scratch` names a host-side stand-in, never the device memory:
// only the address hipGetSymbolAddress returns for a device is passed on.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // per device ordinal: the array's address on that device

// The array's address on the GPU that holds the solver's arena, looked up once per device with that
// device current.
int32_t scratch_of(const Solver &S, void *&out) {
  hipPointerAttribute_t attr{};
  HIP_TRY(hipPointerGetAttributes(&attr, S.arena), "hipPointerGetAttributes");
  const int dev = attr.device;
  if (dev < 0) return set_error(BDDMP_DEVICE, "the solver's arena is not device memory");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (size_t(dev) >= g_scratch_ptr.size()) g_scratch_ptr.resize(size_t(dev) + 1, nullptr);
  if (!g_scratch_ptr[size_t(dev)]) {
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur), "hipGetDevice");
    if (cur != dev) HIP_TRY(hipSetDevice(dev), "hipSetDevice");
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) HIP_TRY(hipSetDevice(cur), "hipSetDevice");
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress (static scratch)");
    if (!p || reinterpret_cast<uintptr_t>(p) % 256) return set_error(BDDMP_DEVICE, "static scratch misplaced");
    g_scratch_ptr[size_t(dev)] = p;
  }
  out = g_scratch_ptr[size_t(dev)];
  return BDDMP_OK;
}

}  // namespace

int32_t solver_smooth_grad_noalloc(Solver &S, float alpha, int32_t T, double dlb, float *grad) {
  const Plan &P = *S.plan;
  if (T < 0) return set_error(BDDMP_INVALID_ARG, "negative iteration count");
  size_t need = 0;
  if (int32_t rc = solver_smooth_workspace(P, T, &need)) return rc;
  if (need > kNoAllocScratchBytes)
    return set_error(BDDMP_INVALID_ARG, "workspace of " + std::to_string(need) + " bytes exceeds the static scratch of " +
                                            std::to_string(kNoAllocScratchBytes) + " bytes");
  void *ws = nullptr;
  if (int32_t rc = scratch_of(S, ws)) return rc;
  // the run writes every checkpoint before the gradient reads it, and the gradient clears its
  // adjoint arrays itself: nothing left by an earlier call is read
  if (int32_t rc = solver_smooth_run(S, alpha, T, ws, kNoAllocScratchBytes)) return rc;
  return solver_smooth_grad(S, alpha, T, ws, kNoAllocScratchBytes, dlb, grad);
}

int32_t solver_set_costs(Solver &S, const double *cost_dev) {
  const Plan &P = *S.plan;
  if (!cost_dev && P.n > 0) return set_error(BDDMP_INVALID_ARG, "null costs");
  if (int32_t rc = check_finite<double>(S, {cost_dev}, P.n, "the costs")) return rc;
  if (int32_t rc = launched(launch_cost_in(S.D, cost_dev, P.n, S.stream), "cost_in")) return rc;
  S.costs_replaced = true;
  return BDDMP_OK;
}

void solver_destroy(Solver *S) { delete S; }

}  // namespace bddmp
