// Primal heuristic (Sec. 4; App. "Primal heuristic" and "Variable fixations"): variables are fixed
// to their preferred values in descending order of a score, each fixation restricting every
// diagram that holds the variable and propagating the values the restricted diagrams imply.
//
// A fixation x_i = beta sends the (1 - beta)-arcs of the level of x_i to FALSE in each diagram of
// J_i (Alg. "Variable Fixation"); a node that loses its last in-arc is removed with its out-arcs
// (Alg. "Remove-Forward"), a node whose arcs both lead to FALSE is removed and its in-arcs sent to
// FALSE (Alg. "Remove-Backward"). A diagram whose root or TRUE terminal is cut off has an empty
// restricted feasible set. After the changes, a level whose remaining arcs all carry one label
// implies that value for its variable (the set F of Alg. "Restriction-Propagation").
//
// The search follows Alg. "Primal-Heuristic" as a depth-first search: fix the open variable of
// largest score to its preferred value and propagate; if that empties a feasible set, undo and try
// the other value; when both fail, return to the latest fixation whose other value is untried (the
// backtracking the text of Sec. 4 describes) until a complete solution or a budget of dead ends
// is reached. Every change goes on an undo trail.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"

namespace bddmp {

namespace {

constexpr int32_t kArcBot = -1, kArcTop = -2;

struct Restrictor {
  const Plan &P;
  // per canonical node: current children (global node index, kArcBot or kArcTop), alive flag,
  // number of live in-arcs; per canonical incidence (level): live 0-arcs and 1-arcs
  std::vector<int32_t> arc;      // [2N]
  std::vector<uint8_t> alive;    // [N]
  std::vector<int32_t> indeg;    // [N]
  std::vector<int32_t> cnt;      // [2I]
  std::vector<int32_t> top_in;   // [m] live arcs into TRUE per row
  std::vector<int32_t> node_row, node_lvl;  // [N]
  std::vector<int64_t> in_ptr;   // [N+1] static in-arcs: (parent << 1) | label
  std::vector<int64_t> in_arc;
  std::vector<int8_t> value;     // [n] -1 open, 0 / 1 fixed
  std::vector<int64_t> var_ptr;  // [n+1] canonical incidences of each variable
  std::vector<int32_t> var_inc;
  // undo trail: (kind, index, old value)
  struct Undo {
    int32_t kind;
    int64_t idx;
    int32_t old;
  };
  std::vector<Undo> trail;
  std::vector<int32_t> touched;  // rows restricted since the last check
  bool failed = false;

  explicit Restrictor(const Plan &plan) : P(plan) {
    const int64_t N = P.N, I = P.I;
    arc.assign(2 * size_t(N), kArcBot);
    alive.assign(size_t(N), 1);
    indeg.assign(size_t(N), 0);
    cnt.assign(2 * size_t(I), 0);
    top_in.assign(size_t(P.m), 0);
    node_row.assign(size_t(N), 0);
    node_lvl.assign(size_t(N), 0);
    std::vector<int64_t> deg(size_t(N) + 1, 0);
    for (int32_t j = 0; j < P.m; ++j) {
      if (P.row_shape[j] < 0) continue;
      const Shape &sh = P.shapes[P.row_shape[j]];
      const int64_t n0 = P.canon_node[j];
      for (int32_t l = 0; l < sh.k; ++l)
        for (int32_t u = sh.first[l]; u < sh.first[l + 1]; ++u) {
          const int64_t g = n0 + u;
          node_row[g] = j;
          node_lvl[g] = int32_t(P.canon_off[j] + l);
          const int32_t ch[2] = {sh.lo[u], sh.hi[u]};
          for (int b = 0; b < 2; ++b) {
            int32_t t = kArcBot;
            if (ch[b] == -2) t = kArcTop;
            else if (ch[b] >= 0) t = int32_t(n0 + sh.first[l + 1] + ch[b]);
            arc[2 * g + b] = t;
            if (t != kArcBot) cnt[2 * size_t(node_lvl[g]) + b]++;
            if (t >= 0) {
              indeg[t]++;
              deg[size_t(t) + 1]++;
            }
            if (t == kArcTop) top_in[j]++;
          }
        }
    }
    in_ptr.assign(size_t(N) + 1, 0);
    for (int64_t g = 0; g < N; ++g) in_ptr[g + 1] = in_ptr[g] + deg[g + 1];
    in_arc.assign(size_t(in_ptr[N]), 0);
    std::vector<int64_t> fill(in_ptr.begin(), in_ptr.end() - 1);
    for (int64_t g = 0; g < N; ++g)
      for (int b = 0; b < 2; ++b)
        if (arc[2 * g + b] >= 0) in_arc[fill[arc[2 * g + b]]++] = (g << 1) | b;
    value.assign(size_t(P.n), -1);
    var_ptr.assign(size_t(P.n) + 1, 0);
    for (int64_t c = 0; c < I; ++c) var_ptr[P.inc_var[c] + 1]++;
    for (int32_t i = 0; i < P.n; ++i) var_ptr[i + 1] += var_ptr[i];
    var_inc.assign(size_t(I), 0);
    std::vector<int64_t> vf(var_ptr.begin(), var_ptr.end() - 1);
    for (int64_t c = 0; c < I; ++c) var_inc[vf[P.inc_var[c]]++] = int32_t(c);
  }

  bool is_root(int64_t g) const {
    const int32_t j = node_row[g];
    return node_lvl[g] == P.canon_off[j] && g == P.canon_node[j];
  }

  void set_arc(int64_t g, int b, int32_t t) {
    trail.push_back({0, 2 * g + b, arc[2 * g + b]});
    arc[2 * g + b] = t;
  }
  void add_cnt(int64_t lvl, int b, int32_t d) {
    trail.push_back({1, 2 * lvl + b, cnt[2 * lvl + b]});
    cnt[2 * lvl + b] += d;
  }
  void add_indeg(int64_t g, int32_t d) {
    trail.push_back({2, g, indeg[g]});
    indeg[g] += d;
  }
  void kill(int64_t g) {
    trail.push_back({3, g, alive[g]});
    alive[g] = 0;
    if (is_root(g)) failed = true;
  }
  void add_top(int32_t j, int32_t d) {
    trail.push_back({4, j, top_in[j]});
    top_in[j] += d;
    if (top_in[j] == 0) failed = true;
  }
  void set_value(int32_t i, int8_t v) {
    trail.push_back({5, i, value[i]});
    value[i] = v;
  }

  void undo_to(size_t mark) {
    while (trail.size() > mark) {
      const Undo u = trail.back();
      trail.pop_back();
      switch (u.kind) {
        case 0: arc[u.idx] = u.old; break;
        case 1: cnt[u.idx] = u.old; break;
        case 2: indeg[u.idx] = u.old; break;
        case 3: alive[u.idx] = uint8_t(u.old); break;
        case 4: top_in[u.idx] = u.old; break;
        default: value[u.idx] = int8_t(u.old); break;
      }
    }
    touched.clear();
    failed = false;
  }

  // an arc of a live node stops being live (redirected to FALSE or its tail removed)
  void drop_arc_target(int64_t g, int b) {
    const int32_t t = arc[2 * g + b];
    if (t == kArcBot) return;
    add_cnt(node_lvl[g], b, -1);
    if (t == kArcTop) {
      add_top(node_row[g], -1);
    } else {
      add_indeg(t, -1);
      if (indeg[t] == 0 && alive[t]) remove_forward(t);
    }
  }

  // Alg. "Remove-Forward": a node no longer reachable from the root
  void remove_forward(int64_t g) {
    kill(g);
    for (int b = 0; b < 2; ++b) drop_arc_target(g, b);
  }

  // Alg. "Remove-Backward": a node with no path to TRUE; its in-arcs go to FALSE
  void remove_backward(int64_t g) {
    kill(g);
    for (int64_t q = in_ptr[g]; q < in_ptr[g + 1]; ++q) {
      const int64_t p = in_arc[q] >> 1;
      const int b = int(in_arc[q] & 1);
      if (alive[p] && arc[2 * p + b] == int32_t(g)) redirect(p, b);
    }
  }

  // send the b-arc of live node g to FALSE (Alg. "Variable Fixation")
  void redirect(int64_t g, int b) {
    if (arc[2 * g + b] == kArcBot) return;
    drop_arc_target(g, b);
    set_arc(g, b, kArcBot);
    if (alive[g] && arc[2 * g] == kArcBot && arc[2 * g + 1] == kArcBot) remove_backward(g);
  }

  // restrict every diagram of x_i to x_i = v
  void fix_level(int64_t c, int v) {
    // the row and level of canonical incidence c
    const int32_t row = node_row[first_node_of(c)];
    const Shape &sh = P.shapes[P.row_shape[row]];
    const int32_t l = int32_t(c - P.canon_off[row]);
    const int64_t n0 = P.canon_node[row];
    for (int32_t u = sh.first[l]; u < sh.first[l + 1]; ++u) {
      const int64_t g = n0 + u;
      if (alive[g]) redirect(g, 1 - v);
      if (failed) return;
    }
  }

  std::vector<int64_t> inc_first_node;  // [I] first canonical node of each level
  int64_t first_node_of(int64_t c) const { return inc_first_node[c]; }

  void build_level_index() {
    inc_first_node.assign(size_t(P.I), 0);
    for (int32_t j = 0; j < P.m; ++j) {
      if (P.row_shape[j] < 0) continue;
      const Shape &sh = P.shapes[P.row_shape[j]];
      for (int32_t l = 0; l < sh.k; ++l) inc_first_node[P.canon_off[j] + l] = P.canon_node[j] + sh.first[l];
    }
  }

  // Alg. "Restriction-Propagation" from x_i = v: false if some restricted feasible set is empty
  bool propagate(int32_t i0, int v0) {
    std::vector<std::pair<int32_t, int>> queue{{i0, v0}};
    size_t head = 0;
    while (head < queue.size()) {
      const int32_t i = queue[head].first;
      const int v = queue[head].second;
      ++head;
      if (value[i] >= 0) {
        if (value[i] != v) return false;
        continue;
      }
      set_value(i, int8_t(v));
      touched.clear();
      for (int64_t q = var_ptr[i]; q < var_ptr[i + 1]; ++q) {
        fix_level(var_inc[q], v);
        if (failed) return false;
        touched.push_back(node_row[first_node_of(var_inc[q])]);
      }
      // implied values of each restricted row: a level whose live arcs all carry one label
      for (int32_t row : touched)
        for (int64_t lvl = P.canon_off[row]; lvl < P.canon_off[row + 1]; ++lvl) {
          const int c0 = cnt[2 * lvl], c1 = cnt[2 * lvl + 1];
          const int32_t iv = P.inc_var[lvl];
          if (c0 == 0 && c1 == 0) return false;
          const int forced = c1 == 0 ? 0 : (c0 == 0 ? 1 : -1);
          if (forced < 0) continue;
          if (value[iv] >= 0) {
            if (value[iv] != forced) return false;
          } else {
            queue.push_back({iv, forced});
          }
        }
      touched.clear();
    }
    return !failed;
  }
};

}  // namespace

int32_t primal_search(const Plan &P, const float *M, int32_t mode, int64_t max_dead_ends, int8_t *x, double *obj,
                      int32_t *feasible, int64_t *implied) {
  if (!M || !x) return set_error(BDDMP_INVALID_ARG, "null M or x");
  if (mode < 0 || mode > 2) return set_error(BDDMP_INVALID_ARG, "score mode must be 0, 1 or 2");
  Restrictor R(P);
  R.build_level_index();
  const int32_t n = P.n;
  // scores (Sec. 4 and App. "Search strategies"): |M_i|, -M_i, or sign(R_i) M_i with R_i the
  // search space reduction coefficient from solution counts (Table "algebras", counting algebra)
  std::vector<double> score(size_t(n), 0.0);
  std::vector<double> rdiff(size_t(n), 0.0);
  if (mode == 2) {
    for (int32_t j = 0; j < P.m; ++j) {
      if (P.row_shape[j] < 0) continue;
      const Shape &sh = P.shapes[P.row_shape[j]];
      const int32_t nn = sh.first[sh.k];
      std::vector<double> fw(size_t(nn), 0.0), bw(size_t(nn), 0.0);
      auto bval = [&](int32_t l, int32_t ch) { return ch == -2 ? 1.0 : (ch < 0 ? 0.0 : bw[size_t(sh.first[l + 1] + ch)]); };
      for (int32_t l = sh.k - 1; l >= 0; --l)
        for (int32_t u = sh.first[l]; u < sh.first[l + 1]; ++u) bw[u] = bval(l, sh.lo[u]) + bval(l, sh.hi[u]);
      fw[0] = 1.0;
      for (int32_t l = 0; l + 1 < sh.k; ++l)
        for (int32_t u = sh.first[l]; u < sh.first[l + 1]; ++u)
          for (int32_t ch : {sh.lo[u], sh.hi[u]})
            if (ch >= 0) fw[size_t(sh.first[l + 1] + ch)] += fw[u];
      for (int32_t l = 0; l < sh.k; ++l) {
        double c1 = 0.0, c0 = 0.0;
        for (int32_t u = sh.first[l]; u < sh.first[l + 1]; ++u) {
          c0 += fw[u] * bval(l, sh.lo[u]);
          c1 += fw[u] * bval(l, sh.hi[u]);
        }
        rdiff[P.inc_var[P.canon_off[j] + l]] += c1 - c0;
      }
    }
  }
  for (int32_t i = 0; i < n; ++i) {
    const double m = double(M[i]);
    score[i] = mode == 0 ? std::fabs(m) : (mode == 1 ? -m : (rdiff[i] > 0 ? m : (rdiff[i] < 0 ? -m : 0.0)));
  }
  std::vector<int32_t> order(static_cast<size_t>(n));
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return score[a] > score[b]; });
  // variables in no row take their own best value (eq. "preferred-variable-value")
  int64_t n_free = 0;
  for (int32_t i = 0; i < n; ++i)
    if (R.var_ptr[i] == R.var_ptr[i + 1]) {
      R.set_value(i, int8_t(P.cost[i] < 0));
      ++n_free;
    }
  struct Decision {
    int32_t pos;   // position in the order
    int8_t value;  // value in force
    bool last;     // no other value left to try
    size_t mark;   // trail length before the fixation
  };
  std::vector<Decision> stack;
  int64_t dead_ends = 0;
  bool ok = true;
  int32_t pos = 0;
  for (;;) {
    while (pos < n && R.value[order[pos]] >= 0) ++pos;
    if (pos == n) break;
    const int32_t i = order[pos];
    const int beta = M[i] <= 0.0f ? 1 : 0;
    const size_t mark = R.trail.size();
    if (R.propagate(i, beta)) {
      stack.push_back({pos, int8_t(beta), false, mark});
      continue;
    }
    R.undo_to(mark);
    if (R.propagate(i, 1 - beta)) {
      stack.push_back({pos, int8_t(1 - beta), true, mark});
      continue;
    }
    R.undo_to(mark);
    // dead end: back to the latest fixation with an untried value
    ++dead_ends;
    bool resumed = false;
    while (!stack.empty() && dead_ends <= max_dead_ends) {
      const Decision d = stack.back();
      stack.pop_back();
      R.undo_to(d.mark);
      if (d.last) continue;
      const int32_t vi = order[d.pos];
      if (R.propagate(vi, 1 - d.value)) {
        stack.push_back({d.pos, int8_t(1 - d.value), true, d.mark});
        pos = d.pos;
        resumed = true;
        break;
      }
      R.undo_to(d.mark);
      ++dead_ends;
    }
    if (!resumed) {
      ok = false;
      break;
    }
  }
  int64_t fixed = 0;
  for (int32_t i = 0; i < n; ++i) fixed += R.value[i] >= 0;
  const int64_t n_implied = fixed - int64_t(stack.size()) - n_free;
  double o = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    x[i] = R.value[i] < 0 ? int8_t(-1) : R.value[i];
    if (x[i] == 1) o += P.cost[i];
  }
  if (obj) *obj = o;
  if (feasible) *feasible = ok ? 1 : 0;
  if (implied) *implied = n_implied;
  return BDDMP_OK;
}

int32_t restrict_row(const Plan &P, int32_t row, int32_t n_fix, const int32_t *vars, const int8_t *vals,
                     uint8_t *alive, int32_t *lo, int32_t *hi, int32_t *feasible) {
  if (row < 0 || row >= P.m) return set_error(BDDMP_INVALID_ARG, "row out of range");
  if (n_fix < 0 || (n_fix > 0 && (!vars || !vals))) return set_error(BDDMP_INVALID_ARG, "bad fixations");
  Restrictor R(P);
  R.build_level_index();
  bool ok = true;
  for (int32_t q = 0; q < n_fix && ok; ++q) {
    if (vars[q] < 0 || vars[q] >= P.n || (vals[q] != 0 && vals[q] != 1))
      return set_error(BDDMP_INVALID_ARG, "fixation out of range");
    const int32_t i = vars[q];
    for (int64_t k = R.var_ptr[i]; k < R.var_ptr[i + 1] && ok; ++k) {
      const int64_t c = R.var_inc[k];
      if (R.node_row[R.first_node_of(c)] != row) continue;
      R.fix_level(c, vals[q]);
      ok = !R.failed;
    }
  }
  if (feasible) *feasible = ok ? 1 : 0;
  if (P.row_shape[row] < 0) return BDDMP_OK;
  const Shape &sh = P.shapes[P.row_shape[row]];
  const int64_t n0 = P.canon_node[row];
  for (int32_t l = 0; l < sh.k; ++l)
    for (int32_t u = sh.first[l]; u < sh.first[l + 1]; ++u) {
      const int64_t g = n0 + u;
      if (alive) alive[u] = R.alive[g];
      for (int b = 0; b < 2; ++b) {
        const int32_t t = R.arc[2 * g + b];
        const int32_t code = t == kArcBot ? -1 : (t == kArcTop ? -2 : int32_t(t - (n0 + sh.first[l + 1])));
        if (b == 0 && lo) lo[u] = code;
        if (b == 1 && hi) hi[u] = code;
      }
    }
  return BDDMP_OK;
}

}  // namespace bddmp
