// Internal types of the bddmp library (host builder, planner, solver).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "bddmp.h"

namespace bddmp {

// Child codes of the 16-bit packed arcs: an in-level index of the next level, or a terminal.
constexpr uint32_t kBot = 0xFFFFu;
constexpr uint32_t kTop = 0xFFFEu;
constexpr int32_t kMaxWidth = 0x7FFF;   // widest level the 16-bit child codes can address
constexpr int kTile = 256;              // layers per workgroup of the wave kernels
constexpr int kBigMax = 4096;           // max rows of one variable (J_i) a wave kernel handles
constexpr int kLbBlocks = 1024;         // fixed partial count of the deterministic fp64 reductions

struct Error {
  int32_t code;
  std::string msg;
};

// Records the message for bddmp_last_error and returns code.
int32_t set_error(int32_t code, const std::string &msg);

// One canonical diagram shape: levels, per-level widths, level-relative children (-1 BOT, -2 TOP).
struct Shape {
  int32_t k = 0;
  std::vector<int32_t> first;  // [k+1]
  std::vector<int32_t> lo, hi; // [nodes]
  int32_t max_width = 0;
};

// Threshold construction of the BDD of  sum_t a[t] x_t (sense) b  (levels t = 0..k-1).
// Returns BDDMP_OK, ROW_INFEASIBLE or BDD_TOO_LARGE (budget > 0 caps the node count).
int32_t build_shape(const int64_t *a, int32_t k, int32_t sense, int64_t b, int64_t budget, Shape &out,
                    std::string &err);

struct Problem {
  int32_t n = 0;
  std::vector<double> cost;
  std::vector<int64_t> row_ptr{0};
  std::vector<int32_t> col;
  std::vector<int64_t> coef;
  std::vector<int8_t> sense;
  std::vector<int64_t> rhs;
  std::vector<int32_t> order;  // empty = identity
};

// Byte offsets of the solver's arrays inside the device arena.
struct ArenaLayout {
  size_t arcs, mf, mb, node_off, child_off, lam, seg, canon_of, layer_of, layer_var;
  size_t fwd_tiles, bwd_tiles, bwd_list, fwd_big, bwd_big;
  size_t root_node, bdd_canon_off, cost, var_first, var_nj;
  size_t d_fresh, mbuf, xbuf, part, ipart, lb_hist, scal;
  size_t total;
};

struct WaveRange {
  int32_t tile_begin, tile_end;  // normal tiles [begin, end) in the pass's tile list
  int32_t big_begin, big_end;    // big tiles (one variable with more than kTile rows)
  int32_t list;                  // backward pass: 1 if positions go through bwd_list
};

struct Plan {
  int32_t n = 0, m = 0;
  int64_t N = 0, I = 0, live = 0, bot = 0;
  int32_t max_width = 0, max_j = 0;
  std::vector<Shape> shapes;
  std::vector<int32_t> row_shape;     // [m], -1 for a row without variables
  std::vector<int64_t> canon_off;     // [m+1] first canonical incidence of row j
  std::vector<int64_t> canon_node;    // [m+1] first canonical node of row j
  std::vector<int32_t> inc_var;       // [I] variable of each canonical incidence
  std::vector<int32_t> order, rank;   // processing order and its inverse
  std::vector<int32_t> wave_f, wave_b; // [n], 1-based, 0 = no rows
  int32_t Df = 0, Db = 0;
  double lb_const = 0.0;              // sum of min(0, c_i) over variables in no row
  std::vector<double> cost;
  // host images of the device arrays (storage = forward-wave-major layer order)
  std::vector<uint32_t> arcs;         // [N] lo | hi << 16
  std::vector<int32_t> node_off;      // [I+1]
  std::vector<int32_t> child_off;     // [I], -1 on a last level
  std::vector<uint32_t> seg;          // [I] position in the variable's segment | length << 16
  std::vector<int32_t> canon_of;      // [I] storage layer -> canonical incidence
  std::vector<int32_t> layer_of;      // [I] canonical incidence -> storage layer
  std::vector<int32_t> layer_var;     // [I] variable of a storage layer
  std::vector<int32_t> fwd_tiles, bwd_tiles;  // tile start positions (+ end sentinel)
  std::vector<int32_t> fwd_big, bwd_big;      // big tiles as (start, end) position pairs
  std::vector<int32_t> bwd_list;      // [I] backward position -> storage layer (used if not contiguous)
  std::vector<WaveRange> fwd_waves, bwd_waves;
  bool bwd_contiguous = true;
  std::vector<int32_t> root_node;     // [m] node of the root, -1 for rows without variables
  std::vector<int32_t> bdd_canon_off; // [m+1] as int32 for the device
  std::vector<int32_t> var_first;     // [n] first storage layer of the variable, -1 if none
  std::vector<int32_t> var_nj;        // [n] |J_i|
  int32_t hist_cap = 4096;
  ArenaLayout lay{};
};

int32_t make_plan(const Problem &p, const bddmp_options &opt, Plan &out);
void greedy_colour_order(const Problem &p, std::vector<int32_t> &order);

}  // namespace bddmp
