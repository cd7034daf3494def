// C-ABI of bddmp: argument checks, handle ownership, status codes and the last-error message.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include "bddmp.h"
#include "internal.h"
#include "solver.h"

struct bddmp_problem {
  bddmp::Problem p;
};
struct bddmp_plan {
  bddmp::Plan plan;
};
struct bddmp_solver {
  bddmp::Solver *s = nullptr;
};

namespace bddmp {

namespace {
thread_local std::string g_last_error;
}

int32_t set_error(int32_t code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

}  // namespace bddmp

using bddmp::set_error;

namespace {

template <class F>
int32_t guarded(F &&f) {
  try {
    return f();
  } catch (const std::bad_alloc &) {
    return set_error(BDDMP_INVALID_ARG, "host allocation failed");
  } catch (const std::exception &e) {
    return set_error(BDDMP_INVALID_ARG, std::string("exception: ") + e.what());
  }
}

// FNV-1a over the bytes of one array, then its byte count
template <class V>
void digest_add(uint64_t &h, const V &v) {
  const unsigned char *b = reinterpret_cast<const unsigned char *>(v.data());
  const size_t nb = v.size() * sizeof(v[0]);
  for (size_t i = 0; i < nb; ++i) h = (h ^ b[i]) * 1099511628211ull;
  for (int k = 0; k < 8; ++k) h = (h ^ ((uint64_t(nb) >> (8 * k)) & 0xFFu)) * 1099511628211ull;
}

}  // namespace

extern "C" {

int32_t bddmp_version(void) { return 10000; }

const char *bddmp_last_error(void) { return bddmp::g_last_error.c_str(); }

int32_t bddmp_options_default(bddmp_options *opt) {
  if (!opt) return set_error(BDDMP_INVALID_ARG, "null options");
  std::memset(opt, 0, sizeof *opt);
  opt->hist_cap = 4096;
  return BDDMP_OK;
}

int32_t bddmp_problem_create(int32_t n_vars, const double *cost, bddmp_problem **out) {
  return guarded([&] {
    if (!out) return set_error(BDDMP_INVALID_ARG, "null out");
    *out = nullptr;
    if (n_vars < 0 || (n_vars > 0 && !cost)) return set_error(BDDMP_INVALID_ARG, "bad n_vars or null cost");
    for (int32_t i = 0; i < n_vars; ++i)
      if (!std::isfinite(cost[i])) return set_error(BDDMP_NONFINITE, "cost " + std::to_string(i) + " is not finite");
    auto *h = new bddmp_problem();
    h->p.n = n_vars;
    h->p.cost.assign(cost, cost + n_vars);
    *out = h;
    return int32_t(BDDMP_OK);
  });
}

int32_t bddmp_problem_add_rows(bddmp_problem *h, int32_t n_rows, const int64_t *row_ptr, const int32_t *col,
                               const int64_t *coef, const int8_t *sense, const int64_t *rhs) {
  return guarded([&] {
    if (!h || n_rows < 0) return set_error(BDDMP_INVALID_ARG, "null problem or negative row count");
    if (n_rows == 0) return int32_t(BDDMP_OK);
    if (!row_ptr || !sense || !rhs) return set_error(BDDMP_INVALID_ARG, "null row array");
    bddmp::Problem &p = h->p;
    const int64_t base = row_ptr[0];
    for (int32_t r = 0; r < n_rows; ++r)
      if (row_ptr[r + 1] < row_ptr[r]) return set_error(BDDMP_INVALID_ARG, "row_ptr not non-decreasing");
    const int64_t nnz = row_ptr[n_rows] - base;
    if (nnz > 0 && (!col || !coef)) return set_error(BDDMP_INVALID_ARG, "null col or coef");
    for (int64_t q = 0; q < nnz; ++q)
      if (col[base + q] < 0 || col[base + q] >= p.n) return set_error(BDDMP_INVALID_ARG, "column out of range");
    for (int32_t r = 0; r < n_rows; ++r)
      if (sense[r] < 0 || sense[r] > 2) return set_error(BDDMP_INVALID_ARG, "sense must be 0, 1 or 2");
    // the builders add coefficients to partial sums and compare them with the right-hand side in
    // int64: keep every such sum below 2^62
    constexpr int64_t kMag = int64_t(1) << 62;
    for (int32_t r = 0; r < n_rows; ++r) {
      if (rhs[r] <= -kMag || rhs[r] >= kMag) return set_error(BDDMP_INVALID_ARG, "row " + std::to_string(r) + ": |rhs| >= 2^62");
      int64_t mag = rhs[r] < 0 ? -rhs[r] : rhs[r];
      for (int64_t q = row_ptr[r]; q < row_ptr[r + 1]; ++q) {
        const int64_t a = coef[q];
        if (a <= -kMag || a >= kMag || (a < 0 ? -a : a) >= kMag - mag)
          return set_error(BDDMP_INVALID_ARG, "row " + std::to_string(r) + ": sum of |coefficients| + |rhs| >= 2^62");
        mag += a < 0 ? -a : a;
      }
    }
    const int64_t off = p.row_ptr.back();
    for (int32_t r = 0; r < n_rows; ++r) p.row_ptr.push_back(off + row_ptr[r + 1] - base);
    p.col.insert(p.col.end(), col + base, col + base + nnz);
    p.coef.insert(p.coef.end(), coef + base, coef + base + nnz);
    p.sense.insert(p.sense.end(), sense, sense + n_rows);
    p.rhs.insert(p.rhs.end(), rhs, rhs + n_rows);
    return int32_t(BDDMP_OK);
  });
}

int32_t bddmp_problem_add_rows_real(bddmp_problem *h, int32_t n_rows, const int64_t *row_ptr, const int32_t *col,
                                    const double *coef, const int8_t *sense, const double *rhs) {
  return guarded([&] {
    if (!h || n_rows < 0) return set_error(BDDMP_INVALID_ARG, "null problem or negative row count");
    if (n_rows == 0) return int32_t(BDDMP_OK);
    if (!row_ptr || !sense || !rhs) return set_error(BDDMP_INVALID_ARG, "null row array");
    for (int32_t r = 0; r < n_rows; ++r)
      if (row_ptr[r + 1] < row_ptr[r]) return set_error(BDDMP_INVALID_ARG, "row_ptr not non-decreasing");
    const int64_t base = row_ptr[0], nnz = row_ptr[n_rows] - base;
    if (nnz > 0 && !coef) return set_error(BDDMP_INVALID_ARG, "null coef");
    constexpr double kExact = 9007199254740992.0;  // 2^53: every integer below it is a double
    auto integral = [&](double v) { return std::isfinite(v) && std::fabs(v) < kExact && std::trunc(v) == v; };
    std::vector<int64_t> ci(static_cast<size_t>(nnz)), bi(static_cast<size_t>(n_rows));
    for (int64_t q = 0; q < nnz; ++q) {
      if (!integral(coef[base + q]))
        return set_error(BDDMP_NOT_INTEGER, "coefficient " + std::to_string(base + q) + " is not an integer below 2^53");
      ci[size_t(q)] = int64_t(coef[base + q]);
    }
    for (int32_t r = 0; r < n_rows; ++r) {
      if (!integral(rhs[r]))
        return set_error(BDDMP_NOT_INTEGER, "right-hand side " + std::to_string(r) + " is not an integer below 2^53");
      bi[size_t(r)] = int64_t(rhs[r]);
    }
    std::vector<int64_t> rp(size_t(n_rows) + 1);
    for (int32_t r = 0; r <= n_rows; ++r) rp[size_t(r)] = row_ptr[r] - base;
    return bddmp_problem_add_rows(h, n_rows, rp.data(), col ? col + base : nullptr, ci.data(), sense, bi.data());
  });
}

int32_t bddmp_problem_set_order(bddmp_problem *h, const int32_t *perm) {
  return guarded([&] {
    if (!h) return set_error(BDDMP_INVALID_ARG, "null problem");
    bddmp::Problem &p = h->p;
    if (!perm) {
      p.order.clear();
      return int32_t(BDDMP_OK);
    }
    std::vector<char> seen(size_t(p.n), 0);
    for (int32_t r = 0; r < p.n; ++r) {
      if (perm[r] < 0 || perm[r] >= p.n || seen[perm[r]]) return set_error(BDDMP_INVALID_ARG, "order is not a permutation");
      seen[perm[r]] = 1;
    }
    p.order.assign(perm, perm + p.n);
    return int32_t(BDDMP_OK);
  });
}

int32_t bddmp_plan_create(const bddmp_problem *h, const bddmp_options *opt, bddmp_plan **out) {
  return guarded([&] {
    if (!h || !out) return set_error(BDDMP_INVALID_ARG, "null problem or out");
    *out = nullptr;
    bddmp_options o;
    if (opt) o = *opt;
    else bddmp_options_default(&o);
    auto *pl = new bddmp_plan();
    const int32_t rc = bddmp::make_plan(h->p, o, pl->plan);
    if (rc != BDDMP_OK) {
      delete pl;
      return rc;
    }
    *out = pl;
    return int32_t(BDDMP_OK);
  });
}

int32_t bddmp_plan_create_batch(const bddmp_problem *const *probs, int32_t n_inst, const bddmp_options *opt,
                                bddmp_plan **out) {
  return guarded([&] {
    if (!out) return set_error(BDDMP_INVALID_ARG, "null out");
    *out = nullptr;
    if (n_inst < 1 || !probs) return set_error(BDDMP_INVALID_ARG, "need at least one instance");
    bddmp::Problem cat;
    cat.inst_var.push_back(0);
    cat.inst_row.push_back(0);
    int64_t nv = 0;
    for (int32_t k = 0; k < n_inst; ++k) {
      if (!probs[k]) return set_error(BDDMP_INVALID_ARG, "null instance " + std::to_string(k));
      const bddmp::Problem &q = probs[k]->p;
      if (nv + q.n > INT32_MAX) return set_error(BDDMP_INVALID_ARG, "more than 2^31 - 1 variables in the batch");
      const int32_t v0 = int32_t(nv);
      cat.cost.insert(cat.cost.end(), q.cost.begin(), q.cost.end());
      const int64_t e0 = cat.row_ptr.back();
      for (size_t r = 1; r < q.row_ptr.size(); ++r) cat.row_ptr.push_back(e0 + q.row_ptr[r]);
      for (int32_t c : q.col) cat.col.push_back(v0 + c);
      cat.coef.insert(cat.coef.end(), q.coef.begin(), q.coef.end());
      cat.sense.insert(cat.sense.end(), q.sense.begin(), q.sense.end());
      cat.rhs.insert(cat.rhs.end(), q.rhs.begin(), q.rhs.end());
      if (q.order.empty())
        for (int32_t i = 0; i < q.n; ++i) cat.order.push_back(v0 + i);
      else
        for (int32_t i : q.order) cat.order.push_back(v0 + i);
      nv += q.n;
      cat.inst_var.push_back(nv);
      cat.inst_row.push_back(int64_t(cat.row_ptr.size()) - 1);
    }
    cat.n = int32_t(nv);
    bddmp_options o;
    if (opt) o = *opt;
    else bddmp_options_default(&o);
    auto *pl = new bddmp_plan();
    const int32_t rc = bddmp::make_plan(cat, o, pl->plan);
    if (rc != BDDMP_OK) {
      delete pl;
      return rc;
    }
    *out = pl;
    return int32_t(BDDMP_OK);
  });
}

int32_t bddmp_plan_instances(const bddmp_plan *h, int64_t *var_off, int64_t *row_off, int64_t *inc_off) {
  if (!h) return set_error(BDDMP_INVALID_ARG, "null plan");
  const bddmp::Plan &P = h->plan;
  const size_t k = P.inst_var.size();
  if (var_off) std::memcpy(var_off, P.inst_var.data(), 8 * k);
  if (row_off) std::memcpy(row_off, P.inst_row.data(), 8 * k);
  if (inc_off) std::memcpy(inc_off, P.inst_inc.data(), 8 * k);
  return BDDMP_OK;
}

int32_t bddmp_plan_primal_search(const bddmp_plan *h, const float *M, int32_t score_mode, int64_t max_dead_ends,
                                 int8_t *x, double *obj, int32_t *feasible, int64_t *n_implied) {
  if (!h) return set_error(BDDMP_INVALID_ARG, "null plan");
  if (max_dead_ends < 0) return set_error(BDDMP_INVALID_ARG, "negative dead-end budget");
  return guarded([&] {
    return bddmp::primal_search(h->plan, M, score_mode, max_dead_ends, x, obj, feasible, n_implied);
  });
}

int32_t bddmp_plan_restrict_row(const bddmp_plan *h, int32_t row, int32_t n_fix, const int32_t *vars,
                                const int8_t *vals, uint8_t *alive, int32_t *lo, int32_t *hi, int32_t *feasible) {
  if (!h) return set_error(BDDMP_INVALID_ARG, "null plan");
  return guarded([&] { return bddmp::restrict_row(h->plan, row, n_fix, vars, vals, alive, lo, hi, feasible); });
}

int32_t bddmp_plan_stats(const bddmp_plan *h, bddmp_stats *out) {
  if (!h || !out) return set_error(BDDMP_INVALID_ARG, "null plan or out");
  const bddmp::Plan &P = h->plan;
  std::memset(out, 0, sizeof *out);
  out->n_vars = P.n;
  out->n_bdds = P.m;
  out->n_nodes = P.N;
  out->n_arcs_live = P.live;
  out->n_arcs_bot = P.bot;
  out->n_incidences = P.I;
  out->waves_fwd = P.Df;
  out->waves_bwd = P.Db;
  out->device_bytes = int64_t(P.lay.total);
  out->max_width = P.max_width;
  out->n_shapes = int32_t(P.shapes.size());
  out->max_rows_per_var = P.max_j;
  out->bwd_contiguous = P.bwd_contiguous ? 1 : 0;
  out->fwd_tiles = int64_t(P.fwd_tiles.size() / 2 + P.fwd_big.size() / 2);
  out->bwd_tiles = int64_t(P.bwd_tiles.size() / 2 + P.bwd_big.size() / 2);
  out->n_instances = int32_t(P.inst_var.size() - 1);
  out->n_intervals = P.split_k;
  out->n_cuts = P.n_cuts;
  out->n_copy_pairs = P.n_copy;
  out->fused_turn = P.fuse_turn ? 1 : 0;
  out->fused_wrap = P.fuse_wrap ? 1 : 0;
  out->dataflow = P.pers_ok ? 1 : 0;
  out->n_groups = P.n_groups;
  out->tile_deps_fwd = int64_t(P.fdep_list.size());
  out->tile_deps_bwd = int64_t(P.bdep_list.size());
  for (const auto *ptr : {&P.fdep_ptr, &P.bdep_ptr})
    for (size_t t = 0; t + 1 < ptr->size(); ++t) out->max_tile_deps = std::max(out->max_tile_deps, (*ptr)[t + 1] - (*ptr)[t]);
  return BDDMP_OK;
}

int32_t bddmp_plan_export_order(const bddmp_plan *h, int32_t *perm_out) {
  if (!h || (!perm_out && h->plan.n)) return set_error(BDDMP_INVALID_ARG, "null plan or output");
  std::memcpy(perm_out, h->plan.order.data(), sizeof(int32_t) * size_t(h->plan.n));
  return BDDMP_OK;
}

int32_t bddmp_plan_export_structure(const bddmp_plan *h, int32_t *level_width, int32_t *level_var, int32_t *lo,
                                    int32_t *hi) {
  if (!h) return set_error(BDDMP_INVALID_ARG, "null plan");
  const bddmp::Plan &P = h->plan;
  int64_t qi = 0, qn = 0;
  for (int32_t j = 0; j < P.m; ++j) {
    if (P.row_shape[j] < 0) continue;
    const bddmp::Shape &sh = P.shapes[P.row_shape[j]];
    for (int32_t l = 0; l < sh.k; ++l, ++qi) {
      if (level_width) level_width[qi] = sh.first[l + 1] - sh.first[l];
      if (level_var) level_var[qi] = P.inc_var[qi];
    }
    for (size_t u = 0; u < sh.lo.size(); ++u, ++qn) {
      if (lo) lo[qn] = sh.lo[u];
      if (hi) hi[qn] = sh.hi[u];
    }
  }
  return BDDMP_OK;
}

int32_t bddmp_plan_export_tile_deps(const bddmp_plan *h, int32_t pass, int32_t *dep_ptr, int32_t *dep_list,
                                    int32_t *tile_group) {
  if (!h) return set_error(BDDMP_INVALID_ARG, "null plan");
  if (pass != 0 && pass != 1) return set_error(BDDMP_INVALID_ARG, "pass must be 0 (forward) or 1 (backward)");
  const bddmp::Plan &P = h->plan;
  if (!P.pers_ok) return set_error(BDDMP_INVALID_ARG, "the plan has no dataflow launch");
  const auto &ptr = pass ? P.bdep_ptr : P.fdep_ptr;
  const auto &lst = pass ? P.bdep_list : P.fdep_list;
  if (dep_ptr) std::memcpy(dep_ptr, ptr.data(), sizeof(int32_t) * ptr.size());
  if (dep_list && !lst.empty()) std::memcpy(dep_list, lst.data(), sizeof(int32_t) * lst.size());
  if (tile_group) {
    const auto &qptr = pass ? P.bqptr : P.fqptr;
    const auto &qtile = pass ? P.bqtile : P.fqtile;
    for (size_t g = 0; g + 1 < qptr.size(); ++g)
      for (int32_t k = qptr[g]; k < qptr[g + 1]; ++k) tile_group[qtile[size_t(k)]] = int32_t(g);
  }
  return BDDMP_OK;
}

int32_t bddmp_plan_export_wave_split(const bddmp_plan *h, int32_t pass, int32_t *tile_begin, int32_t *mid,
                                     int32_t *b_wait) {
  if (!h) return set_error(BDDMP_INVALID_ARG, "null plan");
  if (pass != 0 && pass != 1) return set_error(BDDMP_INVALID_ARG, "pass must be 0 (forward) or 1 (backward)");
  const bddmp::Plan &P = h->plan;
  if (!P.pers_ok) return set_error(BDDMP_INVALID_ARG, "the plan has no tile dependency lists");
  const auto &waves = pass ? P.bwd_waves : P.fwd_waves;
  const auto &split = pass ? P.bsplit : P.fsplit;
  for (size_t w = 0; w < waves.size(); ++w) {
    if (tile_begin) tile_begin[w] = waves[w].tile_begin;
    if (mid) mid[w] = split[w].mid;
    if (b_wait) b_wait[w] = split[w].b_wait;
  }
  if (tile_begin) tile_begin[waves.size()] = waves.empty() ? 0 : waves.back().tile_end;
  return BDDMP_OK;
}

int32_t bddmp_plan_digest(const bddmp_plan *h, uint64_t *digest) {
  if (!h || !digest) return set_error(BDDMP_INVALID_ARG, "null plan or digest");
  const bddmp::Plan &P = h->plan;
  uint64_t d = 1469598103934665603ull;
  const std::vector<int64_t> sizes{P.n, P.m, P.N, P.I, P.S, P.Sc, P.Df, P.Db, P.n_general, int64_t(P.lay.total)};
  digest_add(d, sizes);
  digest_add(d, P.meta); digest_add(d, P.child); digest_add(d, P.parent); digest_add(d, P.garcs);
  digest_add(d, P.grec); digest_add(d, P.gnb); digest_add(d, P.rbeg); digest_add(d, P.rin); digest_add(d, P.rarc);
  digest_add(d, P.canon_of); digest_add(d, P.layer_of); digest_add(d, P.layer_var); digest_add(d, P.root_slot);
  digest_add(d, P.fwd_tiles); digest_add(d, P.bwd_tiles); digest_add(d, P.fwd_big); digest_add(d, P.bwd_big);
  digest_add(d, P.bwd_list); digest_add(d, P.bdd_canon_off); digest_add(d, P.var_first); digest_add(d, P.var_nj);
  digest_add(d, P.own_slot); digest_add(d, P.cslot); digest_add(d, P.cuts); digest_add(d, P.cut_slots);
  digest_add(d, P.cut_live); digest_add(d, P.cut_rb); digest_add(d, P.cut_arc); digest_add(d, P.inst_cut);
  digest_add(d, P.inst_cut_idx); digest_add(d, P.exit_rec); digest_add(d, P.fdep_ptr); digest_add(d, P.fdep_list);
  digest_add(d, P.bdep_ptr); digest_add(d, P.bdep_list); digest_add(d, P.ftinfo); digest_add(d, P.btinfo);
  digest_add(d, P.ftrec); digest_add(d, P.btrec); digest_add(d, P.fqptr); digest_add(d, P.fqtile);
  digest_add(d, P.bqptr); digest_add(d, P.bqtile); digest_add(d, P.fgt); digest_add(d, P.bgt); digest_add(d, P.fgm);
  digest_add(d, P.bgm); digest_add(d, P.wave_f); digest_add(d, P.wave_b); digest_add(d, P.order); digest_add(d, P.rank);
  digest_add(d, P.cost); digest_add(d, P.inc_var); digest_add(d, P.var_group); digest_add(d, P.inst_row32);
  digest_add(d, P.inst_lb_const);
  *digest = d;
  return BDDMP_OK;
}

int32_t bddmp_plan_export_waves(const bddmp_plan *h, int32_t *wave_fwd, int32_t *wave_bwd) {
  if (!h) return set_error(BDDMP_INVALID_ARG, "null plan");
  const bddmp::Plan &P = h->plan;
  if (wave_fwd) std::memcpy(wave_fwd, P.wave_f.data(), sizeof(int32_t) * size_t(P.n));
  if (wave_bwd) std::memcpy(wave_bwd, P.wave_b.data(), sizeof(int32_t) * size_t(P.n));
  return BDDMP_OK;
}

int32_t bddmp_solver_bind(const bddmp_plan *h, void *dev_arena, size_t bytes, void *hip_stream, bddmp_solver **out) {
  return guarded([&] {
    if (!h || !out) return set_error(BDDMP_INVALID_ARG, "null plan or out");
    *out = nullptr;
    bddmp::Solver *s = nullptr;
    const int32_t rc = bddmp::solver_bind(h->plan, dev_arena, bytes, hip_stream, s);
    if (rc != BDDMP_OK) return rc;
    auto *w = new bddmp_solver();
    w->s = s;
    *out = w;
    return int32_t(BDDMP_OK);
  });
}

#define SOLVER_OR_FAIL(h)                                                   \
  if (!(h) || !(h)->s) return set_error(BDDMP_BAD_STATE, "null or unbound solver")

int32_t bddmp_solver_reset(bddmp_solver *h) {
  SOLVER_OR_FAIL(h);
  return guarded([&] { return bddmp::solver_reset(*h->s); });
}

int32_t bddmp_solver_iterate(bddmp_solver *h, int32_t n_iters) {
  SOLVER_OR_FAIL(h);
  return guarded([&] { return bddmp::solver_iterate(*h->s, n_iters); });
}

int32_t bddmp_solver_iterate_until(bddmp_solver *h, int32_t max_iters, double min_rel_impr, int32_t check_every,
                                   int32_t *iters_done, int32_t *stop_at, double *lb) {
  SOLVER_OR_FAIL(h);
  return guarded([&] {
    return bddmp::solver_iterate_until(*h->s, max_iters, min_rel_impr, check_every, iters_done, stop_at, lb);
  });
}

int32_t bddmp_solver_lower_bound(bddmp_solver *h, double *lb, double *residual, double *any_lambda_bound) {
  SOLVER_OR_FAIL(h);
  return guarded([&] { return bddmp::solver_lower_bound(*h->s, lb, residual, any_lambda_bound); });
}

int32_t bddmp_solver_instance_bounds(bddmp_solver *h, double *lb_host, int32_t n) {
  SOLVER_OR_FAIL(h);
  return guarded([&] { return bddmp::solver_instance_bounds(*h->s, lb_host, n); });
}

int32_t bddmp_solver_lb_history(bddmp_solver *h, double *lb_host, int32_t cap, int32_t *n_out) {
  SOLVER_OR_FAIL(h);
  if (cap < 0 || (cap > 0 && !lb_host)) return set_error(BDDMP_INVALID_ARG, "bad history buffer");
  return guarded([&] { return bddmp::solver_lb_history(*h->s, lb_host, cap, n_out); });
}

int32_t bddmp_solver_min_marginals(bddmp_solver *h, float *m0_dev, float *m1_dev) {
  SOLVER_OR_FAIL(h);
  return guarded([&] { return bddmp::solver_min_marginals(*h->s, m0_dev, m1_dev); });
}

int32_t bddmp_solver_get_lambda(bddmp_solver *h, float *lam_dev) {
  SOLVER_OR_FAIL(h);
  if (!lam_dev) return set_error(BDDMP_INVALID_ARG, "null output");
  return guarded([&] { return bddmp::solver_get_lambda(*h->s, lam_dev); });
}

int32_t bddmp_solver_set_lambda(bddmp_solver *h, const float *lam_dev) {
  SOLVER_OR_FAIL(h);
  if (!lam_dev) return set_error(BDDMP_INVALID_ARG, "null input");
  return guarded([&] { return bddmp::solver_set_lambda(*h->s, lam_dev); });
}

int32_t bddmp_solver_get_copy_duals(bddmp_solver *h, float *mu_bar_dev, float *mu_dev, float *dfw_dev, float *dbw_dev) {
  SOLVER_OR_FAIL(h);
  return guarded([&] { return bddmp::solver_copy_duals(*h->s, true, mu_bar_dev, mu_dev, dfw_dev, dbw_dev); });
}

int32_t bddmp_solver_set_copy_duals(bddmp_solver *h, const float *mu_bar_dev, const float *mu_dev, const float *dfw_dev,
                                    const float *dbw_dev) {
  SOLVER_OR_FAIL(h);
  return guarded([&] {
    return bddmp::solver_copy_duals(*h->s, false, const_cast<float *>(mu_bar_dev), const_cast<float *>(mu_dev),
                                    const_cast<float *>(dfw_dev), const_cast<float *>(dbw_dev));
  });
}

int32_t bddmp_solver_round_primal(bddmp_solver *h, float *M_dev, int8_t *x_host, double *obj, int64_t *n_violated) {
  SOLVER_OR_FAIL(h);
  return guarded([&] { return bddmp::solver_round_primal(*h->s, M_dev, x_host, obj, n_violated); });
}

int32_t bddmp_smooth_workspace_bytes(const bddmp_plan *h, int32_t n_iters, size_t *bytes) {
  if (!h) return set_error(BDDMP_INVALID_ARG, "null plan");
  return bddmp::solver_smooth_workspace(h->plan, n_iters, bytes);
}

int32_t bddmp_solver_smooth_run(bddmp_solver *h, float alpha, int32_t n_iters, void *ws, size_t ws_bytes) {
  SOLVER_OR_FAIL(h);
  return guarded([&] { return bddmp::solver_smooth_run(*h->s, alpha, n_iters, ws, ws_bytes); });
}

int32_t bddmp_solver_smooth_grad(bddmp_solver *h, float alpha, int32_t n_iters, void *ws, size_t ws_bytes,
                                 double dlb, float *grad_dev) {
  SOLVER_OR_FAIL(h);
  return guarded([&] { return bddmp::solver_smooth_grad(*h->s, alpha, n_iters, ws, ws_bytes, dlb, grad_dev); });
}

int32_t bddmp_solver_smooth_grad_noalloc(bddmp_solver *h, float alpha, int32_t n_iters, double dlb, float *grad_dev) {
  SOLVER_OR_FAIL(h);
  return guarded([&] { return bddmp::solver_smooth_grad_noalloc(*h->s, alpha, n_iters, dlb, grad_dev); });
}

int32_t bddmp_solver_set_costs(bddmp_solver *h, const double *cost_dev) {
  SOLVER_OR_FAIL(h);
  return bddmp::solver_set_costs(*h->s, cost_dev);
}

int32_t bddmp_solver_set_graphs(bddmp_solver *h, int32_t enable) {
  SOLVER_OR_FAIL(h);
  return bddmp::solver_set_graphs(*h->s, enable);
}

int32_t bddmp_solver_set_launch(bddmp_solver *h, int32_t mode, int32_t chunk) {
  SOLVER_OR_FAIL(h);
  return guarded([&] { return bddmp::solver_set_launch(*h->s, mode, chunk); });
}

int32_t bddmp_solver_get_launch(const bddmp_solver *h, int32_t *mode, int32_t *chunk) {
  SOLVER_OR_FAIL(h);
  return bddmp::solver_get_launch(*h->s, mode, chunk);
}

int32_t bddmp_solver_set_groups(bddmp_solver *h, const int32_t *lanes) {
  SOLVER_OR_FAIL(h);
  return bddmp::solver_set_groups(*h->s, lanes);
}

int32_t bddmp_solver_get_groups(const bddmp_solver *h, int32_t *lanes) {
  SOLVER_OR_FAIL(h);
  return bddmp::solver_get_groups(*h->s, lanes);
}

int32_t bddmp_solver_autotune(bddmp_solver *h, int32_t iters, int32_t *lanes) {
  SOLVER_OR_FAIL(h);
  return guarded([&] { return bddmp::solver_autotune(*h->s, iters, lanes); });
}

int32_t bddmp_solver_time_kernels(bddmp_solver *h, int32_t n_iters, bddmp_kernel_times *out) {
  SOLVER_OR_FAIL(h);
  if (!out || n_iters < 0) return set_error(BDDMP_INVALID_ARG, "bad arguments");
  return guarded([&] { return bddmp::solver_time_kernels(*h->s, n_iters, out); });
}

void bddmp_solver_destroy(bddmp_solver *h) {
  if (!h) return;
  bddmp::solver_destroy(h->s);
  delete h;
}

void bddmp_plan_destroy(bddmp_plan *h) { delete h; }

void bddmp_problem_destroy(bddmp_problem *h) { delete h; }

}  // extern "C"
