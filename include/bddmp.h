/*
 * bddmp: BDD-based min-marginal averaging for 0-1 ILP relaxations on one
 * MI355X (gfx950) GPU.
 *
 * The method is dual block coordinate ascent on the Lagrangean decomposition
 * of a 0-1 ILP into one binary decision diagram (BDD) per linear row
 * (J.-H. Lange and P. Swoboda, "Efficient Message Passing for 0-1 ILPs with
 * Binary Decision Diagrams", ICML 2021):
 *   - problem: min c^T x s.t. each row sum_i a_ji x_i (=, <=, >=) b_j,
 *     x in {0,1}^n (Sec. 3, Def. "Binary program", Example "ILP");
 *   - dual (D): max sum_j E^j(lambda^j), E^j = min over the row's feasible set
 *     of x^T lambda^j, s.t. sum_{j in J_i} lambda^j_i = c_i (Sec. 3.1);
 *   - one iteration = a forward and a backward pass of Alg. "Min-marginal
 *     averaging" (Sec. 3.2) with the incremental BDD updates of Sec. 5.3-5.4;
 *   - outputs: the bound, multipliers, min-marginals (eq. "min-marginals")
 *     and the rounded primal of eq. "preferred-variable-value" (Sec. 4).
 *
 * Conventions for every entry point:
 *   - Return value: BDDMP_OK (0) or a negative status below; after a failure
 *     bddmp_last_error() returns a message (thread-local).
 *   - Host input arrays are copied; the caller keeps ownership.
 *   - Handles are created and destroyed only through this API. A plan must
 *     outlive every solver bound from it.
 *   - Device memory belongs to the caller. bddmp_solver_bind receives one
 *     arena (at least bddmp_stats.device_bytes bytes, 256-byte aligned) and
 *     the library keeps all of its device state there; it allocates no other
 *     device memory and never frees the arena.
 *   - Device work is enqueued on the caller's HIP stream. Only the calls that
 *     hand back host values (lower_bound, lb_history, round_primal,
 *     time_kernels) and the calls that check device inputs for NaN and
 *     infinities (set_lambda, set_copy_duals, set_costs) synchronise it.
 *   - One handle is used by one host thread at a time.
 *   - Per-incidence arrays use the canonical incidence order: rows in input
 *     order, and within a row its variables in processing order (the levels
 *     of its BDD). Per-node arrays use rows, then levels, then the in-level
 *     node order (breadth-first from the root, 0-arc child first).
 */
#ifndef BDDMP_H
#define BDDMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define BDDMP_OK 0
#define BDDMP_INVALID_ARG (-1)    /* bad pointer, size, index, sense or permutation          */
#define BDDMP_ROW_INFEASIBLE (-2) /* a row has no 0/1 solution (its BDD would be empty)      */
#define BDDMP_BDD_TOO_LARGE (-3)  /* node budget exceeded, or a level wider than 32767       */
#define BDDMP_NOT_INTEGER (-4)    /* a real coefficient or right-hand side is not an integer  */
#define BDDMP_CONFLICT (-5)       /* rows force one variable to both 0 and 1                 */
#define BDDMP_DEVICE (-6)         /* a HIP call failed; the message holds HIP's error string */
#define BDDMP_BAD_STATE (-7)      /* call out of order                                       */
#define BDDMP_NONFINITE (-8)      /* NaN or infinite cost, multiplier, copy dual or bound    */

/* row senses */
#define BDDMP_EQ 0
#define BDDMP_LE 1
#define BDDMP_GE 2

typedef struct bddmp_problem bddmp_problem; /* host: costs, rows, order              */
typedef struct bddmp_plan bddmp_plan;       /* host: BDDs, wave schedule, HBM layout */
typedef struct bddmp_solver bddmp_solver;   /* device state in the caller's arena    */

typedef struct {
  int32_t order_mode;     /* 0: the problem's order (identity if none set); 1: greedy colouring */
  int32_t hist_cap;       /* bound history ring length on the device (default 4096)           */
  int64_t node_budget;    /* max total BDD nodes, 0 = unlimited                                */
  int32_t tile_work;      /* a tile closes once its general levels hold this many own plus next-
                             level nodes (0: 2048; the node-parallel path stages up to 2048 of each) */
  const char *tiling;     /* general-layer path by width class, "g0,g1,g2,g3" (NULL: default
                             "0,0,0,0"); see bddmp_solver_set_groups                             */
  int32_t n_intervals;    /* Sec. 6 split: variable intervals per instance (0 or 1: no split)   */
  float split_gamma;      /* copy-arc step size gamma in (0, 1] (0: default 0.5)                 */
  int32_t wave_align;     /* 0: each variable in its earliest wave (the longest chain of row
                             predecessors before it); 1: in its latest (the longest chain after it
                             ends with the last wave), so shorter instances of a batch start late.
                             Both order every variable after its predecessors in each pass, so
                             results are the same; only the schedule differs                     */
} bddmp_options;

typedef struct {
  int64_t n_vars, n_bdds, n_nodes, n_arcs_live, n_arcs_bot, n_incidences;
  int32_t waves_fwd, waves_bwd; /* dependency waves per forward / backward pass            */
  int64_t device_bytes;         /* arena size bddmp_solver_bind needs                      */
  int32_t max_width;            /* widest BDD level                                        */
  int32_t n_shapes;             /* distinct BDD shapes built (rows sharing coefficients)   */
  int32_t max_rows_per_var;     /* max |J_i|                                               */
  int32_t bwd_contiguous;       /* 1 if every backward wave is a contiguous layer range    */
  int64_t fwd_tiles, bwd_tiles; /* workgroups per forward / backward pass                  */
  int32_t n_instances;          /* independent instances in the plan (1 unless batched)   */
  int32_t n_intervals;          /* Sec. 6 variable intervals per instance (0: no split)    */
  int64_t n_cuts;               /* cut levels (one per sub-BDD boundary)                   */
  int64_t n_copy_pairs;         /* copy-arc pairs (live arcs leaving the cut levels)       */
  int32_t fused_turn;           /* 1 if the last forward wave and the first backward wave run
                                   as one launch (their levels are the rows' last levels)  */
  int32_t fused_wrap;           /* 1 if, inside a run of iterations, the last backward wave
                                   and the next iteration's first forward wave run as one
                                   launch (their levels are the rows' roots)                */
  int32_t dataflow;             /* 1 if the plan supports the dataflow launch of a pass
                                   (bddmp_solver_set_launch; no variable in > 256 rows)     */
  int32_t max_tile_deps;        /* most tiles one tile waits for in the dataflow launch    */
  int32_t n_groups;             /* groups of instances, one ticket queue each (dataflow)    */
  int64_t tile_deps_fwd, tile_deps_bwd; /* tile-to-tile dependencies per pass              */
} bddmp_stats;

typedef struct {
  double fwd_ms, bwd_ms, lb_ms;          /* summed pass time per class over the timed iterations   */
  int64_t fwd_launches, bwd_launches, lb_launches;
  double fwd_bytes, bwd_bytes;           /* algorithmic bytes moved by all launches of the class   */
  double iter_ms;                        /* event time per iteration without inner events          */
} bddmp_kernel_times;

/* Library version (major*10000 + minor*100 + patch). */
int32_t bddmp_version(void);

/* Message of the calling thread's last failure ("" if none). Valid until the next call. */
const char *bddmp_last_error(void);

/* Fills *opt with defaults (order_mode 0, hist_cap 4096, no budget). */
int32_t bddmp_options_default(bddmp_options *opt);

/*
 * A problem with n_vars binary variables and objective c (Sec. 3, eq. "binary-program").
 * cost: host array [n_vars], copied. n_vars >= 0. NONFINITE if a cost is NaN or infinite.
 */
int32_t bddmp_problem_create(int32_t n_vars, const double *cost, bddmp_problem **out);

/*
 * Appends n_rows linear rows sum_q coef[q] x_{col[q]} (sense) rhs for q in
 * [row_ptr[r], row_ptr[r+1]) (CSR; row_ptr has n_rows+1 entries, row_ptr[0] may be nonzero).
 * Each row becomes one subproblem X_j with I_j = {i : a_ji != 0} (Sec. 3, Example "ILP");
 * zero coefficients are dropped. A column repeated inside a row is INVALID_ARG.
 * sense: BDDMP_EQ, BDDMP_LE or BDDMP_GE. All arrays are host memory and copied.
 * The diagrams are built from partial sums of the coefficients in int64: a row whose
 * sum_q |coef[q]| + |rhs| reaches 2^62 is INVALID_ARG (nothing of the call is kept).
 */
int32_t bddmp_problem_add_rows(bddmp_problem *p, int32_t n_rows, const int64_t *row_ptr, const int32_t *col,
                               const int64_t *coef, const int8_t *sense, const int64_t *rhs);

/*
 * bddmp_problem_add_rows for coefficients and right-hand sides held as doubles (as LP and MPS
 * readers deliver them). The method takes integer rows (Sec. 3, Example "ILP"; the threshold
 * construction of Sec. 5.2 works on integer partial sums): every coef[q] and rhs[r] must be a
 * finite integral value of magnitude below 2^53, else NOT_INTEGER and nothing of the call is kept.
 * Other arguments and errors as bddmp_problem_add_rows.
 */
int32_t bddmp_problem_add_rows_real(bddmp_problem *p, int32_t n_rows, const int64_t *row_ptr, const int32_t *col,
                                    const double *coef, const int8_t *sense, const double *rhs);

/*
 * Processing order of Alg. "Min-marginal averaging": perm[r] is the variable processed r-th by
 * the forward pass (the backward pass uses the reverse). perm: host [n_vars], a permutation;
 * NULL restores the identity.
 */
int32_t bddmp_problem_set_order(bddmp_problem *p, const int32_t *perm);

/*
 * Host build: one canonical quasi-reduced BDD per row (Sec. 5.1 Def. "Binary decision diagram",
 * Prop. "Canonicity"; threshold construction of Sec. 5.2 in O(N log W)), the variable->row
 * incidence J_i (Sec. 3.1), the dependency waves that run Alg. "Min-marginal averaging" exactly
 * (a variable's wave is one more than the latest wave of its predecessor in any of its rows), and
 * the level-sorted structure-of-arrays layout for HBM. opt may be NULL (defaults).
 * Errors: ROW_INFEASIBLE, BDD_TOO_LARGE, CONFLICT (a variable forced to 0 by one row and to 1
 * by another), INVALID_ARG.
 */
int32_t bddmp_plan_create(const bddmp_problem *p, const bddmp_options *opt, bddmp_plan **out);

/*
 * Batched host build: n_inst independent problems solved as one. The plan is that of their
 * block-diagonal union (variables, rows and orders concatenated in instance order), so one wave
 * schedule holds every instance: its depth is the largest instance depth, not the sum. The
 * decomposition (problem (D), Sec. 3.1) splits along instances, so each instance's multipliers,
 * min-marginals and rounded primal are computed with exactly the operations of its own plan
 * (bitwise equal results), and its bound is the sum of its rows' terms. Per-incidence and
 * per-variable outputs are the concatenation of the instances' canonical arrays
 * (bddmp_plan_instances gives the offsets). probs: host array of n_inst >= 1 problem handles,
 * copied. Errors as bddmp_plan_create.
 */
int32_t bddmp_plan_create_batch(const bddmp_problem *const *probs, int32_t n_inst, const bddmp_options *opt,
                                bddmp_plan **out);

/*
 * Offsets of each instance's variables, rows and canonical incidences in the plan's outputs:
 * host arrays of n_instances + 1 (any may be NULL). A plan from bddmp_plan_create has one
 * instance.
 */
int32_t bddmp_plan_instances(const bddmp_plan *plan, int64_t *var_off, int64_t *row_off, int64_t *inc_off);

/*
 * Primal heuristic (Sec. 4; App. "Primal heuristic", Alg. "Primal-Heuristic" with Alg.
 * "Restriction-Propagation" and the BDD manipulations of App. "Variable fixations"): variables are
 * fixed to their preferred values beta_i = [M_i <= 0] (eq. "preferred-variable-value") in
 * descending order of the score (score_mode 0: |M_i|; 1: -M_i; 2: sign(R_i) M_i with R_i the
 * search space reduction coefficient, eq. "search-space-reduction-coeff"; ties by index). Each
 * fixation restricts every diagram of the variable and propagates the values the restricted
 * diagrams imply; when that empties a feasible set the other value is tried; when both fail the
 * search returns to the latest fixation whose other value is untried (depth-first search, Sec. 4).
 * It stops with a solution or after max_dead_ends dead ends (*feasible = 0; undecided variables
 * are -1 in x). Variables in no row take [c_i < 0]. M: host float [n_vars] total min-marginal
 * differences (e.g. from bddmp_solver_round_primal); x: host int8 [n_vars]; *obj = c^T x over the
 * variables set to 1; *n_implied: variables fixed by propagation rather than chosen. Host only.
 */
int32_t bddmp_plan_primal_search(const bddmp_plan *plan, const float *M, int32_t score_mode, int64_t max_dead_ends,
                                 int8_t *x, double *obj, int32_t *feasible, int64_t *n_implied);

/*
 * One row's diagram after fixing variables (App. "Variable fixations": (1-beta)-arcs of the
 * variable's level to FALSE, nodes cut off from the root removed forward, nodes without a path to
 * TRUE removed backward with their in-arcs sent to FALSE). vars/vals: host [n_fix], fixations of
 * variables outside the row are ignored. alive (uint8), lo, hi: host [nodes of the row] in
 * canonical node order, children as in-level indices, -1 FALSE, -2 TRUE; *feasible = 0 when the
 * restricted feasible set is empty. Host only.
 */
int32_t bddmp_plan_restrict_row(const bddmp_plan *plan, int32_t row, int32_t n_fix, const int32_t *vars,
                                const int8_t *vals, uint8_t *alive, int32_t *lo, int32_t *hi, int32_t *feasible);

/* Sizes of the plan (host). */
int32_t bddmp_plan_stats(const bddmp_plan *plan, bddmp_stats *out);

/* The processing order the plan uses: perm_out host [n_vars]. */
int32_t bddmp_plan_export_order(const bddmp_plan *plan, int32_t *perm_out);

/*
 * Canonical structure for exact comparisons: level_width and level_var host [n_incidences],
 * lo and hi host [n_nodes] holding in-level child indices of the next level, -1 for the false
 * terminal and -2 for the true terminal. Any pointer may be NULL.
 */
int32_t bddmp_plan_export_structure(const bddmp_plan *plan, int32_t *level_width, int32_t *level_var,
                                    int32_t *lo, int32_t *hi);

/*
 * Tile schedule of one pass of the dataflow launch (bddmp_solver_set_launch), for inspection and
 * host-side checks: pass 0 forward, 1 backward; dep_ptr host [tiles + 1] (tiles: fwd_tiles or
 * bwd_tiles of bddmp_stats), dep_list host [tile_deps_fwd or tile_deps_bwd]: the tiles tile t waits
 * for are dep_list[dep_ptr[t] .. dep_ptr[t+1]), ascending, each smaller than t; tile_group host
 * [tiles]: the group of instances (ticket queue) of each tile, 0 .. n_groups - 1, the same for a
 * tile and every tile it waits for. Any pointer may be NULL. INVALID_ARG for a plan without
 * dataflow support.
 */
int32_t bddmp_plan_export_tile_deps(const bddmp_plan *plan, int32_t pass, int32_t *dep_ptr, int32_t *dep_list,
                                    int32_t *tile_group);

/*
 * Two-branch split of each wave of one pass (launch mode 2 of bddmp_solver_set_launch), for
 * inspection and host-side checks: pass 0 forward, 1 backward; W = waves_fwd or waves_bwd of
 * bddmp_stats. tile_begin host [W + 1]: wave w holds the pass's tiles [tile_begin[w],
 * tile_begin[w+1]) (the numbering of bddmp_plan_export_tile_deps); mid host [W]: part A of wave w
 * is [tile_begin[w], mid[w]), part B the rest; b_wait host [W]: part B of wave w runs after part A
 * of wave b_wait[w] (-1: it reads no A tile). Every tile of an A part depends only on A tiles of
 * earlier waves, every tile of a B part on B tiles of earlier waves or A tiles of waves up to
 * b_wait. Any pointer may be NULL. INVALID_ARG for a plan without tile dependency lists.
 */
int32_t bddmp_plan_export_wave_split(const bddmp_plan *plan, int32_t pass, int32_t *tile_begin, int32_t *mid,
                                     int32_t *b_wait);

/*
 * A 64-bit digest (FNV-1a) of every array the plan holds for the device and of its layout sizes,
 * for reproducibility checks: plans that upload the same bytes have the same digest, and the same
 * problem and options give the same plan whatever the number of host threads that built it.
 * digest: host uint64 out. INVALID_ARG for a null plan or digest.
 */
int32_t bddmp_plan_digest(const bddmp_plan *plan, uint64_t *digest);

/* Forward and backward wave of every variable (1-based, 0 for variables in no row); host [n_vars]. */
int32_t bddmp_plan_export_waves(const bddmp_plan *plan, int32_t *wave_fwd, int32_t *wave_bwd);

/*
 * Binds a plan to caller device memory and a stream: uploads the layout into dev_arena
 * (device pointer, >= device_bytes, 256-byte aligned), sets lambda^j_i = c_i/|J_i| and runs the
 * initial backward sweep that fills every backward message (Alg. "Min-marginal averaging"
 * initialisation; Prop. "correctness"), then records LB_0. hip_stream is a hipStream_t (NULL =
 * the null stream). Asynchronous on that stream.
 */
int32_t bddmp_solver_bind(const bddmp_plan *plan, void *dev_arena, size_t bytes, void *hip_stream,
                          bddmp_solver **out);

/*
 * Restarts the method on the bound data without uploading again: lambda^j_i = c_i/|J_i|, the
 * initial backward sweep, and LB_0 appended to the bound history. Asynchronous.
 */
int32_t bddmp_solver_reset(bddmp_solver *s);

/*
 * n_iters iterations (forward pass then backward pass, Sec. 3.2 with Sec. 5.4), each followed by
 * the fp64 bound LB_t = sum_j E^j (+ sum of min(0, c_i) over variables in no row), appended to the
 * device bound history. Asynchronous.
 */
int32_t bddmp_solver_iterate(bddmp_solver *s, int32_t n_iters);

/*
 * Iterates until the bound's relative improvement drops below min_rel_impr (Sec. 7: the paper
 * stops at a minimal relative objective improvement of 1e-6): iteration t meets the rule when
 * LB_t - LB_{t-1} < min_rel_impr * max(|LB_t|, 1). The iterations run asynchronously in blocks of
 * check_every; after each block the stream is synchronised and the block's bounds are checked.
 * *iters_done: iterations run (the solver's state is after them; at most max_iters, a multiple of
 * check_every unless max_iters ends the run); *stop_at: the first iteration of this call meeting the
 * rule (1-based), or -1; *lb: the last bound. check_every: 1 .. hist_cap - 1; min_rel_impr >= 0.
 */
int32_t bddmp_solver_iterate_until(bddmp_solver *s, int32_t max_iters, double min_rel_impr, int32_t check_every,
                                   int32_t *iters_done, int32_t *stop_at, double *lb);

/*
 * Latest bound, dual-feasibility residual max_i |c_i - sum_j lambda^j_i| and the bound valid
 * for any lambda, LB + sum_i min(0, c_i - sum_j lambda^j_i) (App. A.1). Synchronises the stream.
 * Any output pointer may be NULL. NONFINITE if the bound is NaN or infinite (the outputs still
 * receive the values); finite multipliers can give an infinite bound when a row's minimum
 * overflows fp32.
 */
int32_t bddmp_solver_lower_bound(bddmp_solver *s, double *lb, double *residual, double *any_lambda_bound);

/*
 * Bound of each instance after the last backward sweep, in fp64: the sum over the instance's rows
 * of E^j (problem (D)) plus the sum of min(0, c_i) over its variables in no row. E^j is recomputed
 * from the root level's messages with the sweep's own operations, and each instance's rows are
 * summed in one fixed shape, so a batched plan gives bitwise the values of each instance's own
 * plan. With a split (Sec. 6) the sub-BDDs after the instance's cuts add their E as the last
 * backward copy-arc update left it, in canonical cut order. lb_host: host [n], n must equal
 * n_instances. Synchronises.
 */
int32_t bddmp_solver_instance_bounds(bddmp_solver *s, double *lb_host, int32_t n);

/* Copies the last min(cap, recorded) bounds (oldest first) to lb_host; *n_out = count. Synchronises. */
int32_t bddmp_solver_lb_history(bddmp_solver *s, double *lb_host, int32_t cap, int32_t *n_out);

/*
 * Fresh min-marginals at the current multipliers (eq. "min-marginals" via eqs. "arc-marginal" and
 * "marginal-aggregation"): a forward sweep without updates, then the level minima.
 * m0_dev, m1_dev: device [n_incidences] in canonical order (either may be NULL). Asynchronous.
 */
int32_t bddmp_solver_min_marginals(bddmp_solver *s, float *m0_dev, float *m1_dev);

/* Multipliers lambda^j_i to lam_dev (device [n_incidences], canonical order). Asynchronous. */
int32_t bddmp_solver_get_lambda(bddmp_solver *s, float *lam_dev);

/* Replaces the multipliers from lam_dev (device, canonical order) and re-runs the initial
 * backward sweep (resume from a checkpoint); appends the new bound. The values are checked on the
 * device first and the stream synchronised: NONFINITE if any is NaN or infinite, and then the
 * solver's state is unchanged. */
int32_t bddmp_solver_set_lambda(bddmp_solver *s, const float *lam_dev);

/*
 * Copy-arc state of a split plan (Sec. 6, Def. "Copy-arc", Alg. "Parallel min-marginal
 * averaging"; bddmp_options.n_intervals > 1). One value per copy-arc pair (n_copy_pairs of
 * bddmp_stats) in canonical order: rows, cut levels ascending, then the arc's tail node (in-level
 * index) and label (0-arc first); only arcs not into BOT. mu_bar: dual of the copy-arc (into TOP)
 * that ends the sub-BDD before the cut; mu: dual of the arc entering the sub-BDD after it; dfw /
 * dbw: the last forward / backward updates delta (the next update of the other dual uses them).
 * get: any pointer may be NULL (device arrays). Asynchronous.
 * set: all four required; then the initial backward sweep re-runs (as bddmp_solver_set_lambda),
 * appending a bound; NONFINITE (state unchanged) if any value is NaN or infinite, checked on the
 * device after which the stream is synchronised. Together with lambda this is a complete
 * checkpoint of a split solver.
 */
int32_t bddmp_solver_get_copy_duals(bddmp_solver *s, float *mu_bar_dev, float *mu_dev, float *dfw_dev, float *dbw_dev);
int32_t bddmp_solver_set_copy_duals(bddmp_solver *s, const float *mu_bar_dev, const float *mu_dev, const float *dfw_dev,
                                    const float *dbw_dev);

/*
 * Rounded primal from fresh min-marginals (Sec. 4): M_i = sum_j (m1_ij - m0_ij) in ascending row
 * order, x_i = [M_i <= 0] (eq. "preferred-variable-value"); variables in no row take [c_i < 0].
 * x_host: host [n_vars]; M_dev: device [n_vars] or NULL; obj: c^T x in fp64; n_violated: rows
 * the point violates (each row's BDD path decides). Synchronises.
 */
int32_t bddmp_solver_round_primal(bddmp_solver *s, float *M_dev, int8_t *x_host, double *obj, int64_t *n_violated);

/*
 * Smoothed variant (App. "Smoothing"): every min of the forward steps, backward steps and
 * min-marginals becomes the soft minimum smin(a, b) = -alpha log(exp(-a/alpha) + exp(-b/alpha))
 * (eq. "marginal-log-sum-exp", the marginal log-sum-exp algebra of Table "algebras" in the log
 * domain), with the update of eq. "mma-update" on those values; the bound is the smoothed dual
 * LB_alpha = sum_j E^j_alpha (eq. "bdd-enery-smoothed") plus smin(0, c_i) for each variable in no
 * row, with E^j >= E^j_alpha >= E^j - alpha log |X_j| (Prop. "Approximation guarantees"). Rows
 * forcing a variable: only the rows whose move raises the smoothed bound hand their difference to
 * the forced rows (d > 0 when a row forces x_i = 1, d < 0 when one forces x_i = 0). Messages and
 * multipliers in fp32, bounds in fp64. Plans with a variable in more than 256 rows: INVALID_ARG.
 *
 * bddmp_smooth_workspace_bytes: device bytes of the workspace for n_iters iterations (multiplier
 * checkpoints after each iteration and the adjoint arrays).
 * bddmp_solver_smooth_run: from lambda = c / |J_i|, the smoothed initial sweep and n_iters smoothed
 * iterations, each LB_alpha appended to the bound history, the multipliers after each iteration
 * kept in ws (device, 256-byte aligned, >= the workspace bytes). Asynchronous.
 * bddmp_solver_smooth_grad: dlb * d LB_alpha(n_iters) / d c into grad_dev (device float [n_vars],
 * variable order), by reverse accumulation over the checkpoints a smooth_run with the same alpha,
 * n_iters and ws left: each iteration is recomputed from its checkpoint, then its backward and
 * forward passes are undone wave by wave in reverse order through the soft-minimum weights. The
 * solver ends at the multipliers after n_iters iterations. Asynchronous.
 */
int32_t bddmp_smooth_workspace_bytes(const bddmp_plan *plan, int32_t n_iters, size_t *bytes);
int32_t bddmp_solver_smooth_run(bddmp_solver *s, float alpha, int32_t n_iters, void *ws, size_t ws_bytes);
int32_t bddmp_solver_smooth_grad(bddmp_solver *s, float alpha, int32_t n_iters, void *ws, size_t ws_bytes,
                                 double dlb, float *grad_dev);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): bddmp_solver_smooth_run followed by
 * bddmp_solver_smooth_grad with the same alpha and n_iters, without a workspace argument. The
 * workspace is a static array in the library's device code, 64 MiB (67108864 bytes) on each GPU
 * the library runs on, allocated when the library's code is loaded on that GPU and held until the
 * process ends; this call itself allocates nothing. Results, bound history and the solver's final
 * state are those of the two calls with a caller workspace. INVALID_ARG, before any device work, if
 * bddmp_smooth_workspace_bytes(plan, n_iters) exceeds 64 MiB. Every call on one GPU uses that GPU's
 * one array: calls that overlap in time on one GPU (from several threads, or on several streams
 * without ordering between them) race and give undefined results. Asynchronous. grad_dev: device
 * float [n_vars].
 */
int32_t bddmp_solver_smooth_grad_noalloc(bddmp_solver *s, float alpha, int32_t n_iters, double dlb, float *grad_dev);

/*
 * Replaces the costs c (device double [n_vars]) used by bddmp_solver_reset and the smoothed run
 * (lambda = c / |J_i| and the terms of variables in no row). The plan keeps its own costs: after
 * this call bddmp_solver_instance_bounds returns BAD_STATE. The values are checked on the device
 * and the stream synchronised: NONFINITE (costs unchanged) if any is NaN or infinite.
 */
int32_t bddmp_solver_set_costs(bddmp_solver *s, const double *cost_dev);

/*
 * Launch mode of bddmp_solver_iterate. enable = 1 (default): one iteration (every wave launch of
 * both passes and the bound reduction) is captured once as a HIP graph on a private stream and
 * replayed on the solver's stream, one graph launch per iteration; the bound's history slot comes
 * from a device counter, so replays need no changed arguments. With bddmp_stats.fused_wrap = 1 a call
 * of n iterations launches the first forward wave, then replays n - 1 times an iteration that ends
 * with the launch that also runs the next iteration's first forward wave, and once an iteration that
 * ends with the plain last backward wave: between calls the state is always that after whole
 * iterations. enable = 0: every wave is launched from the host. Both give bitwise the same results.
 */
int32_t bddmp_solver_set_graphs(bddmp_solver *s, int32_t enable);

/*
 * Launch form of the update passes of bddmp_solver_iterate (and of the timing and autotuning calls).
 * mode 0 (default): one launch per dependency wave, each wave a barrier for the next (with the
 * turnaround and wrap-around fusions of bddmp_stats). mode 1 (dataflow; plans with
 * bddmp_stats.dataflow = 1): one launch per pass whose workgroups stay resident and take tiles
 * (256 layers of whole variables) in the pass's wave order through a device ticket, chunk tiles per
 * ticket (0: 1). A tile starts as soon as the tiles holding the previous levels (forward pass) or
 * the next levels (backward pass) of its rows are done, instead of after the whole previous wave,
 * so independent rows and instances proceed at their own pace; every value computed is the same
 * as with wave launches (the same operations in the same order per layer). Each wait for another
 * tile is bounded; a wait that exceeds its bound (about a second; not expected while the GPU runs
 * only this work) makes the next lower_bound / lb_history return DEVICE until bddmp_solver_reset.
 * mode 2 (two-branch wave launches; plans with bddmp_stats.dataflow = 1): every wave is split in
 * two parts (bddmp_plan_export_wave_split). The A parts are launched in order on the solver's
 * stream and never wait for a B part; the B parts are launched in order on a second stream (created
 * by this call, default priority), each after the A part of the latest wave it reads from. A pass
 * ends when both streams are done. Captured as a graph, the two chains run side by side, so one
 * wave's last workgroups overlap the next wave's first ones. The turnaround and wrap-around fusions
 * are not used; results are bitwise those of mode 0. chunk is ignored by modes 0 and 2.
 * mode 3 (wave groups; plans with bddmp_stats.dataflow = 1): chunk consecutive waves of a pass per
 * launch (0: 4), one workgroup per tile in pass order. A tile of a later wave of the launch first
 * waits for the flags of the tiles it reads from (dependency lists as in mode 1), whose messages
 * are written and read coherently, so the tiles of consecutive waves overlap instead of meeting at
 * a launch boundary. Progress rests on each XCD dispatching its workgroups in block order (every
 * earlier wave's workgroups are dispatched before a later wave's); each wait is bounded all the
 * same, with the error path of mode 1 (about a quarter of a second per wait). The turnaround and
 * wrap-around fusions are not used; results are bitwise those of mode 0. get: chunk is the waves
 * per launch.
 * mode 4 (wave groups, two tiles per workgroup; plans with bddmp_stats.dataflow = 1 whose layers
 * are all narrow, bddmp_stats.max_width <= 2): mode 3 with each workgroup taking two consecutive
 * tiles of the pass order, both tiles' loads and waits issued together, so that twice the loads
 * are in flight per workgroup; a pair whose second tile reads from its first (a pair across a wave
 * boundary) runs them one after the other. It pays on waves of several thousand tiles (halving the
 * workgroups leaves a GPU idle on small waves). Results are bitwise those of mode 0. INVALID_ARG
 * on a plan with general layers.
 * INVALID_ARG for modes 1-4 on a plan without dataflow support.
 * get: either pointer may be NULL.
 * For tests of that failure path, the environment variable BDDMP_PASS_SPIN_LIMIT (read by this
 * call) replaces the bound: the polls of one wait before it gives up.
 */
int32_t bddmp_solver_set_launch(bddmp_solver *s, int32_t mode, int32_t chunk);
int32_t bddmp_solver_get_launch(const bddmp_solver *s, int32_t *mode, int32_t *chunk);

/*
 * Path of the general layers (a level or its next level with more than 2 nodes). Tiles are classed
 * by their widest general level (class 0: <= 8 nodes, 1: <= 32, 2: <= 128, 3: wider); lanes[c]
 * selects the path for class c:
 *   0: node-parallel over the tile: every lane takes nodes of the tile's general levels, the next
 *      levels' messages are staged in LDS, and a layer's min-marginals are integer minima in LDS
 *      (a tile whose general levels exceed the LDS stage falls back to groups of 64);
 *   2^k (1..64): one group of 2^k lanes per layer (one wavefront or a sub-wave group): min-marginals
 *      as per-lane minima and a butterfly minimum over the group.
 * In both, the forward step is a pull over the next level's in-arcs and the backward step takes
 * one node per lane. Results do not depend on the choice (every minimum is exact), only speed.
 * set: host int32[4]; INVALID_ARG unless each is 0 or a power of two up to 64. get: host int32[4].
 */
int32_t bddmp_solver_set_groups(bddmp_solver *s, const int32_t *lanes);
int32_t bddmp_solver_get_groups(const bddmp_solver *s, int32_t *lanes);

/*
 * Autotuner of the general-layer path: for each width class present in the plan, times iters
 * iterations with the node-parallel path and each group size 1, 2, ..., 64 (the other classes at
 * their current choice) and keeps the fastest; lanes (host int32[4], may be NULL) receives the choice. The solver advances by the
 * iterations run (call bddmp_solver_reset to restart). Synchronises.
 */
int32_t bddmp_solver_autotune(bddmp_solver *s, int32_t iters, int32_t *lanes);

/*
 * Diagnostics: runs n_iters iterations launched from the host with a HIP event pair around each
 * forward pass, each backward pass and each bound reduction (not around single launches, so the
 * events add no gap between the waves of a pass) and reports the summed times per class, the
 * launches they cover (one per wave) and the algorithmic bytes of those passes (20 bytes per node
 * and 8 per incidence: arcs 8, messages 12, multiplier 8; with fused_turn the last forward wave's
 * launch and bytes count with the backward pass that runs them); then the same number of iterations as
 * bddmp_solver_iterate runs them (graph replays by default) for iter_ms. The solver advances by
 * 2*n_iters iterations. Synchronises.
 */
int32_t bddmp_solver_time_kernels(bddmp_solver *s, int32_t n_iters, bddmp_kernel_times *out);

void bddmp_solver_destroy(bddmp_solver *s);
void bddmp_plan_destroy(bddmp_plan *plan);
void bddmp_problem_destroy(bddmp_problem *p);

#ifdef __cplusplus
}
#endif
#endif /* BDDMP_H */
