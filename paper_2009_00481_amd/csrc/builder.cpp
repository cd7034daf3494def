// Host BDD builder: linear row -> canonical quasi-reduced BDD (threshold construction).
//
// The diagram of  sum_t a_t x_t (sense) b  over levels t = 0..k-1 (Sec. 5.1 Def. "Binary
// decision diagram": consecutive indices on every path, FALSE reachable from any level, TRUE only
// after the last one, no dead nodes, no isomorphic nodes; canonical by Prop. "Canonicity").
//
// Construction (the threshold idea the paper takes from Behle, Sec. 5.2): with R_t the sorted
// set of sums the suffix a_t..a_{k-1} can reach, a prefix with partial sum s leaves the residual
// threshold beta = b - s. Its feasible completions are the suffixes whose sum r satisfies
// r <= beta ('<='), r >= beta ('>=') or r = beta ('='), so the prefix's class is fixed by how many
// elements of R_t pass the threshold (or by beta's position in R_t for '='): one binary search
// per arc, O(N log W) for the whole diagram. Classes are numbered in breadth-first discovery
// order, 0-arc child first, which is the canonical in-level node order of the library.
#include <algorithm>
#include <string>

#include "internal.h"

namespace bddmp {

namespace {

bool holds(int32_t sense, int64_t lhs, int64_t rhs) {
  return sense == BDDMP_EQ ? lhs == rhs : (sense == BDDMP_LE ? lhs <= rhs : lhs >= rhs);
}

// Class of a prefix with partial sum s against the sorted suffix sums R, or -1 if no completion
// satisfies the row (the arc goes to FALSE).
int64_t threshold_class(const std::vector<int64_t> &R, int32_t sense, int64_t b, int64_t s) {
  const int64_t beta = b - s;
  if (sense == BDDMP_LE) {
    const int64_t c = std::upper_bound(R.begin(), R.end(), beta) - R.begin();  // #{r <= beta}
    return c - 1;
  }
  if (sense == BDDMP_GE) {
    const int64_t c = R.end() - std::lower_bound(R.begin(), R.end(), beta);   // #{r >= beta}
    return c - 1;
  }
  auto it = std::lower_bound(R.begin(), R.end(), beta);
  return (it != R.end() && *it == beta) ? int64_t(it - R.begin()) : -1;
}

}  // namespace

int32_t build_shape(const int64_t *a, int32_t k, int32_t sense, int64_t b, int64_t budget, Shape &out,
                    std::string &err) {
  out = Shape{};
  out.k = k;
  out.first.assign(size_t(k) + 1, 0);
  if (k == 0) {
    if (!holds(sense, 0, b)) {
      err = "row without variables does not hold";
      return BDDMP_ROW_INFEASIBLE;
    }
    return BDDMP_OK;
  }
  // suffix sum sets, merged from the back
  std::vector<std::vector<int64_t>> R(size_t(k) + 1);
  R[k] = {0};
  for (int32_t t = k - 1; t >= 0; --t) {
    const auto &nx = R[t + 1];
    std::vector<int64_t> shifted(nx.size());
    for (size_t q = 0; q < nx.size(); ++q) shifted[q] = nx[q] + a[t];
    std::vector<int64_t> merged;
    merged.reserve(nx.size() * 2);
    std::merge(nx.begin(), nx.end(), shifted.begin(), shifted.end(), std::back_inserter(merged));
    merged.erase(std::unique(merged.begin(), merged.end()), merged.end());
    if (budget > 0 && int64_t(merged.size()) > budget) {
      err = "suffix sums exceed the node budget";
      return BDDMP_BDD_TOO_LARGE;
    }
    R[t] = std::move(merged);
  }
  if (threshold_class(R[0], sense, b, 0) < 0) {
    err = "row has no 0/1 solution";
    return BDDMP_ROW_INFEASIBLE;
  }
  std::vector<int64_t> rep{0}, next_rep;
  std::vector<int32_t> slot;
  int64_t total = 0;
  for (int32_t t = 0; t < k; ++t) {
    const int32_t w = int32_t(rep.size());
    out.first[t + 1] = out.first[t] + w;
    out.max_width = std::max(out.max_width, w);
    total += w;
    if (budget > 0 && total > budget) {
      err = "node budget exceeded";
      return BDDMP_BDD_TOO_LARGE;
    }
    if (w > kMaxWidth) {
      err = "level wider than 32767 nodes";
      return BDDMP_BDD_TOO_LARGE;
    }
    const bool last = t == k - 1;
    if (!last) slot.assign(R[t + 1].size(), -1);
    next_rep.clear();
    for (int32_t u = 0; u < w; ++u) {
      int32_t child[2];
      for (int beta = 0; beta < 2; ++beta) {
        const int64_t s = rep[u] + (beta ? a[t] : 0);
        if (last) {
          child[beta] = holds(sense, s, b) ? -2 : -1;
          continue;
        }
        const int64_t c = threshold_class(R[t + 1], sense, b, s);
        if (c < 0) {
          child[beta] = -1;
          continue;
        }
        if (slot[c] < 0) {
          slot[c] = int32_t(next_rep.size());
          next_rep.push_back(s);
        }
        child[beta] = slot[c];
      }
      out.lo.push_back(child[0]);
      out.hi.push_back(child[1]);
    }
    rep.swap(next_rep);
  }
  return BDDMP_OK;
}

}  // namespace bddmp
