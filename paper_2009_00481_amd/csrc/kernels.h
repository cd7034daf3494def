// Device state and launch entry points of the bddmp kernels (kernels.hip). The host orchestration
// in solver.hip only calls these functions; each returns the launch's hipError_t.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace bddmp {

constexpr int kFwd = 0, kBwd = 1;
constexpr int kUpdate = 0;    // min-marginals, J_i sum, multiplier update, then step
constexpr int kNoUpdate = 1;  // step only (initial backward sweep)
constexpr int kExtract = 2;   // min-marginals to the outputs, then step with unchanged multipliers
constexpr int kTurn = 3;      // backward launch over the last forward wave's levels: the forward update,
                              // then the backward update and step (narrow-only, storage-order tiles)
constexpr int kWrap = 4;      // forward launch over the first forward wave's levels (the rows' roots): the
                              // last backward wave's update and bound partials, then the next
                              // iteration's forward update and step
constexpr int kLbStage = 256; // fixed chunk count of the bound reduction
constexpr uint32_t kFlat = 7; // gsel code of the node-parallel path for general layers

// Pointers into the caller's arena (see ArenaLayout) and the per-call outputs.
struct Dev {
  const uint32_t *meta;
  const int32_t *child, *parent;
  float *lam;
  float *mf;   // forward messages of each layer's own level (own slots)
  float *mbc;  // backward messages of each layer's child level (child slots)
  const uint32_t *garcs;
  const int4 *grec;
  const int2 *gnb;        // child layer's own slot, parent layer's child slot (-1 at row ends)
  const int32_t *rbeg;    // in-arc offsets of general layers' child levels
  const uint32_t *rin;    // the same nodes' in-arcs packed when at most two (kManyInArcs otherwise)
  const uint16_t *rarc;   // in-arcs (source node | kInArcHi for a 1-arc)
  const int32_t *canon_of, *layer_of, *layer_var, *root_slot;
  const int32_t *fwd_tiles, *bwd_tiles, *bwd_list, *fwd_big, *bwd_big;
  const int32_t *bdd_canon_off;
  const double *cost;
  const int32_t *var_first, *var_nj;
  float *d_fresh, *mbuf;
  int8_t *xbuf;
  double *part, *lbpart;
  double *lb_hist, *scal;
  float *out0, *out1;
  int32_t n_bwd_tiles;  // bound partials of big backward tiles start here
  const int32_t *inst_row;  // [n_inst + 1] first row of each instance
  double *inst_lb;          // [n_inst] per-instance bounds
  double *lbc;              // [2] bound constants of the variables in no row: min-plus, smoothed
  long long *hist_n;        // bounds recorded so far (device counter; slot = count % hist_cap)
  unsigned *flag;           // set to 1 by the finiteness checks of device inputs
  int32_t hist_cap;
  uint32_t gsel;            // per tile width class, 4 bits: log2 of the lanes per general layer
                            // (0..6), or kFlat for the node-parallel tile path
  // sub-BDD split (Sec. 6): cut tables (see Plan) and the copy-arc state per arc index; mu_bar of
  // an arc sits in its exit layer's virtual child slot of mbc
  const int4 *cuts, *cut_slots;
  const int32_t *cut_live, *cut_rb;
  const uint16_t *cut_arc;
  float *mu_in, *dfw, *dbw;
  float *cut_e;               // E of the sub-BDD after each cut (written by the backward copy update)
  const int32_t *inst_cut, *inst_cut_idx;  // each instance's cut records (offsets, record indices)
  const int32_t *exit_rec;    // per layer: the cut record it is the exit layer of, or -1 (null: no split)
  float gamma;
  // node maps of the flat path per pass (see Plan): per tile {byte offset of its maps or -1, own |
  // child nodes << 16}, and the maps (layer rank of each staged node, 16-byte aligned per tile)
  const int2 *fgt, *bgt;
  const uint8_t *fgm, *bgm;
};

// One wave: nt normal tiles from tile0 of the pass's tile list (dir kFwd / kBwd, mode as above).
// narrow_only selects the variant without wide levels, list the backward index-list variant.
// kWrap (dir kFwd, narrow-only, no list): bwd_tile0 is the first backward tile of the same levels.
hipError_t launch_wave(int dir, int mode, bool narrow_only, bool list, int nt, int tile0, const Dev &D,
                       hipStream_t s, int bwd_tile0 = 0);
// Dataflow launch of one pass (update mode; plans without big tiles): the pass's tiles in ticket
// order, each after the tiles it depends on (see pass_kernel in kernels.hip).
struct PassArgs {
  const int4 *trec;                   // per tile, 2 int4: start, end, info | deps << 8, list offset; deps
  const int32_t *dep_list;            // dependencies of tiles with more than four
  const int32_t *qptr, *qtile;        // each group's tiles in pass order (CSR over n_queues groups)
  uint32_t *flags;                    // per tile: generation of the launch that finished it
  uint32_t *ctl;                      // kPassCtlWords control words (internal.h)
  int32_t n_tiles;
  int32_t n_queues;                   // groups of instances, one ticket counter each (<= kPassQueues)
  int32_t chunk;                      // consecutive tiles of a queue per ticket (>= 1)
  uint32_t spin_limit;                // polls of one flag before the wait gives up (error word)
};
hipError_t launch_pass(int dir, bool narrow_plan, int grid, const Dev &D, const PassArgs &A, hipStream_t s);
// Resident workgroups per CU of the pass kernel (the launch's grid is this times the CU count).
hipError_t pass_blocks_per_cu(int dir, bool narrow_plan, int *blocks);

// Several consecutive waves of one update pass in one launch (launch mode 3): the pass's tiles
// [t0, t_end), workgroup b running tile t0 + b; [t0, t_first) is the launch's first wave and
// [t_last, t_end) its last. A tile past the first wave waits for the flags of the tiles it reads
// from; every tile stores its flag. The flag value is the bound counter with bit 31 set, the same
// for both passes of an iteration and new in the next.
struct GroupArgs {
  const int4 *trec;      // as PassArgs
  const int32_t *dep_list;
  uint32_t *flags;
  uint32_t *ctl;         // the pass's control words (error word)
  uint32_t spin_limit;
  int32_t t0, t_first, t_last, t_end;
};
// pairs: two tiles per workgroup (group_pair_kernel; plans whose layers are all narrow)
hipError_t launch_group(int dir, bool narrow_plan, bool pairs, const Dev &D, const GroupArgs &A, hipStream_t s);

// Big tiles (one variable with more than kTile rows each) of one wave.
hipError_t launch_wave_big(int dir, int mode, bool list, int nb, int big0, const Dev &D, hipStream_t s);

hipError_t launch_fill(float *p, float v, int n, hipStream_t s);
hipError_t launch_init_lambda(const Dev &D, int I, hipStream_t s);
hipError_t launch_root_zero(const Dev &D, int m, hipStream_t s);
hipError_t launch_lambda_out(const Dev &D, float *out, int I, hipStream_t s);
hipError_t launch_lambda_in(const Dev &D, const float *in, int I, hipStream_t s);
// D.flag = 0 (clear), then D.flag = 1 if any of the n values is NaN or infinite (the check may run
// several times between one clear and the read of the flag).
hipError_t launch_flag_clear(const Dev &D, hipStream_t s);
hipError_t launch_nonfinite(const Dev &D, const float *p, int64_t n, hipStream_t s);
hipError_t launch_nonfinite(const Dev &D, const double *p, int64_t n, hipStream_t s);
// Bound of the backward sweep just run into the history ring at the device counter's slot, then
// the counter advances (no host-side argument changes between iterations, so graphs can replay it).
// which: 0 adds the min-plus constant D.lbc[0], 1 the smoothed one D.lbc[1].
hipError_t launch_lb(const Dev &D, int nparts, int which, hipStream_t s);
hipError_t launch_set_counter(const Dev &D, long long value, hipStream_t s);
// Per-instance bound of the last backward sweep (sum over the instance's rows of E^j, recomputed
// from the messages and multipliers; instance k's constant term is added by the host).
hipError_t launch_instance_bounds(const Dev &D, int n_inst, hipStream_t s);
hipError_t launch_residual(const Dev &D, int n, hipStream_t s);
hipError_t launch_round(const Dev &D, int n, int m, hipStream_t s);

// Sub-BDD split (split.hip): copy duals to zero; the forward and backward copy-arc updates of
// Alg. "Parallel min-marginal averaging" (update = 0: only the cut roots' forward messages and the
// bound partials, written at lbpart[part0 + block]); export / import of the copy state per live pair.
hipError_t launch_copy_init(const Dev &D, int n_cuts, hipStream_t s);
// n_narrow: the leading narrow cuts (one lane each); the others run one wavefront each.
hipError_t launch_copy_fwd(const Dev &D, int n_cuts, int n_narrow, hipStream_t s);
hipError_t launch_copy_bwd(const Dev &D, int n_cuts, int n_narrow, int update, int part0, hipStream_t s);
hipError_t launch_copy_io(const Dev &D, int n_cuts, bool out, float *mu_bar, float *mu, float *dfw, float *dbw,
                          hipStream_t s);

// Smoothed variant (smooth.hip).
struct SmoothArgs {
  float alpha;
  float root_seed;        // adjoint of each root's new backward message in this pass
  const float *lam_prev;  // multipliers before the pass's updates
  const float *lam_upd;   // multipliers after the forward pass's updates
  const float *mbt;       // backward messages the forward pass read
  float *glam, *gmf, *gmb;
};
// One wave of a smoothed pass (adjoint = false) or of its adjoint (true).
hipError_t launch_smooth_wave(int dir, int mode, bool adjoint, bool list, int nt, int tile0, const Dev &D,
                              const SmoothArgs &A, hipStream_t s);
// D.lbc[0] = sum of min(0, c_i), D.lbc[1] = sum of smin_alpha(0, c_i) over variables in no row.
hipError_t launch_free_const(const Dev &D, int n, float alpha, hipStream_t s);
hipError_t launch_smooth_grad(const Dev &D, const SmoothArgs &A, int n, float scale, float *grad, hipStream_t s);
hipError_t launch_cost_in(const Dev &D, const double *c, int n, hipStream_t s);

}  // namespace bddmp
