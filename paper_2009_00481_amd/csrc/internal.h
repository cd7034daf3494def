// Internal types of the bddmp library (host builder, planner, solver).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "bddmp.h"

namespace bddmp {

// 16-bit child codes of the general arc array: an in-level index of the next level, or a terminal.
constexpr uint32_t kBot = 0xFFFFu;
constexpr uint32_t kTop = 0xFFFEu;
constexpr int32_t kMaxWidth = 0x7FFF;   // widest level the 16-bit child codes can address
constexpr int kTile = 256;              // layers per workgroup of the wave kernels
constexpr int kBigMax = 4096;           // max rows of one variable (J_i) a wave kernel handles
constexpr int kLbBlocks = 1024;         // fixed partial count of the deterministic fp64 reductions
constexpr int kCutsPerBlock = 4;        // wide cuts per workgroup of the copy-arc kernels (one wavefront each)

// Control words of one pass's dataflow launch (uint32 offsets): generation of the last launch,
// workgroups gone, error word, then kPassQueues ticket counters, each on a 128-byte line of its own.
constexpr int kPassGen = 0, kPassGone = 1, kPassErr = 2, kPassQueue0 = 32, kPassQueues = 32, kPassQueueStride = 32;
constexpr int kPassCtlWords = kPassQueue0 + kPassQueues * kPassQueueStride;

// 2-bit child codes of a narrow layer (both its level and the next have at most 2 nodes)
constexpr uint32_t kC2Bot = 2u, kC2Top = 3u;

// Layer record meta word: bits 0-7 arcs of a narrow layer (node u: lo at 4u, hi at 4u+2),
// bits 8-9 own width of a narrow layer (0 marks a general layer), bit 10 root level,
// bits 11-20 position in the variable's segment, bits 21-30 segment length (<= 1023 in tiles).
constexpr uint32_t kMetaWidthShift = 8, kMetaRootBit = 1u << 10, kMetaPosShift = 11, kMetaLenShift = 21;
constexpr uint32_t kMetaField = 0x3FFu;

// Bit 31 of a backward tile's end position: the tile holds a root level (contributes to the bound).
constexpr uint32_t kTileRootBit = 0x80000000u;
// Bits 29-30 of a tile's start position: width class of its widest general level (0: <= 8 nodes,
// 1: <= 32, 2: <= 128, 3: wider), which selects the lanes per general layer. Positions stay
// below 2^29.
constexpr uint32_t kTileClsShift = 29, kTilePosMask = (1u << 29) - 1u;
constexpr int kWidthClasses = 4;
// A tile closes early once its general layers hold this many nodes (own plus child level), so
// that tiles with wide levels carry comparable work (default; options.tile_work overrides).
constexpr int64_t kTileWideWork = 2048;
// nodes of a tile's general own levels, and of their child levels, that the node-parallel (flat)
// path stages at most (kFlatCap / kTile per lane)
constexpr int kFlatCap = 2048;
// Packed in-arcs of a next-level node with at most two (two in-arc codes, kNoArc16 for none);
// kManyInArcs marks a node with more, whose in-arcs are read from the offset lists.
constexpr uint32_t kNoArc16 = 0xFFFFu, kManyInArcs = 0xFFFFFFFFu;
// Per tile width class, 4 bits: log2 of the lanes per general layer (0..6), or kGselFlat for the
// node-parallel tile path. Default: the node-parallel path for every class.
constexpr uint32_t kGselFlat = 7u;
constexpr uint32_t kDefaultGsel = kGselFlat | (kGselFlat << 4) | (kGselFlat << 8) | (kGselFlat << 12);
// Lanes value <-> 4-bit code: 0 (node-parallel) <-> kGselFlat, 2^k (k <= 6) <-> k; false if invalid.
bool gsel_code(int32_t lanes, uint32_t &code);
// Parses "g0,g1,g2,g3" (each 0 or a power of two up to 64) into a gsel word; false if malformed.
bool parse_groups(const char *s, uint32_t &gsel);
// In-arc codes of the pull-form forward step: source node index (15 bits) | arc label << 15.
constexpr uint32_t kInArcHi = 0x8000u;

// Records bddmp_last_error's message and returns code.
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
  // independent instances concatenated into this problem (empty = one instance): offsets of each
  // instance's variables and rows, [n_inst + 1]
  std::vector<int64_t> inst_var, inst_row;
};

// Byte offsets of the solver's arrays inside the device arena.
struct ArenaLayout {
  size_t meta, child, parent, lam, mf, mbc, garcs, grec, gnb, rbeg, rin, rarc, canon_of, layer_of, layer_var, root_slot;
  size_t fdep_list, bdep_list, ftrec, btrec, fqptr, fqtile, bqptr, bqtile, fflag, bflag, pctl;
  size_t fgt, bgt, fgm, bgm;
  size_t fwd_tiles, bwd_tiles, bwd_list, fwd_big, bwd_big;
  size_t bdd_canon_off, cost, var_first, var_nj;
  size_t d_fresh, mbuf, xbuf, part, lbpart, lb_hist, scal;
  size_t inst_row, inst_lb;
  size_t cuts, cut_slots, cut_live, cut_rb, cut_arc, mu_in, dfw, dbw, cut_e, inst_cut, inst_cut_idx, exit_rec;
  size_t total;
};

struct WaveRange {
  int32_t tile_begin, tile_end;  // normal tiles [begin, end) in the pass's tile list
  int32_t big_begin, big_end;    // big tiles (one variable with more than kTile rows)
  int32_t list;                  // backward pass: 1 if positions go through bwd_list
  bool narrow_only;              // every layer of the wave is narrow
  int64_t nodes, layers;         // work of the wave (for the byte model)
};

struct Plan {
  int32_t n = 0, m = 0;
  int64_t N = 0, I = 0, live = 0, bot = 0;
  int64_t S = 0;                      // own-level slots: 2 per layer, then the nodes of wider levels
  int64_t Sc = 0;                     // child-level slots, the same way for the next level
  int64_t n_general = 0;              // layers outside the narrow class
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
  // host images of the device arrays (layers in forward-wave-major order)
  std::vector<uint32_t> meta;         // [I] meta word of each layer
  std::vector<int32_t> child, parent; // [I] next / previous level of the same row, -1 at the ends
  std::vector<uint32_t> garcs;        // [S] lo | hi << 16 (16-bit codes) at every node slot
  // [4I] or empty: own slot, child slot, own width | child width << 16, base of the child level's
  // in-arc offsets in rbeg (-1 without child level)
  std::vector<int32_t> grec;
  std::vector<int32_t> gnb;           // [2I] with grec: child layer's own slot, parent layer's child slot (-1 at row ends)
  std::vector<int32_t> rbeg;          // per general layer with a child: child width + 1 offsets into rarc
  std::vector<uint32_t> rin;          // same indexing as rbeg: up to two in-arcs packed, or kManyInArcs
  std::vector<uint16_t> rarc;         // in-arcs of those child levels (kInArcHi marks 1-arcs)
  std::vector<int32_t> canon_of;      // [I] storage layer -> canonical incidence
  std::vector<int32_t> layer_of;      // [I] canonical incidence -> storage layer
  std::vector<int32_t> layer_var;     // [I] variable of a storage layer
  std::vector<int32_t> root_slot;     // [m] slot of the root node, -1 for rows without variables
  std::vector<int32_t> fwd_tiles, bwd_tiles;  // tiles as (start, end) position pairs
  std::vector<int32_t> fwd_big, bwd_big;      // big tiles (one variable each) as (start, end) pairs
  std::vector<int32_t> bwd_list;      // [I] backward position -> storage layer (used if not contiguous)
  std::vector<WaveRange> fwd_waves, bwd_waves;
  bool bwd_contiguous = true;
  // the last forward wave and the first backward wave hold the same layers in the same tiles (every
  // layer a last level, all narrow, no split): one launch runs both passes' steps on them
  bool fuse_turn = false;
  // wrap-around: the first forward wave and the last backward wave hold the same levels in the same
  // tiles (every layer a root level, all narrow, no split): inside a run of iterations, one launch
  // runs the last backward step of one iteration and the first forward step of the next
  bool fuse_wrap = false;
  std::vector<int32_t> bdd_canon_off; // [m+1] as int32 for the device
  std::vector<int32_t> var_first;     // [n] first storage layer of the variable, -1 if none
  std::vector<int32_t> var_nj;        // [n] |J_i|
  // own slot of a layer (device code derives it the same way)
  std::vector<int64_t> own_slot, cslot; // [I] own-level slot and child-level slot
  int32_t hist_cap = 4096;
  int64_t n_lbpart = 0;               // backward tiles (normal + big) = bound partials per sweep
  // instances: offsets of variables, rows and canonical incidences [n_inst + 1], and each
  // instance's constant bound term (sum of min(0, c_i) over its variables in no row)
  std::vector<int64_t> inst_var, inst_row, inst_inc;
  std::vector<double> inst_lb_const;
  std::vector<int32_t> inst_row32;    // inst_row as int32 for the device
  // Sec. 6 split (n_cuts = 0 without one). A cut separates levels l and l+1 of a row whose variables
  // lie in different intervals. The layer of level l (exit layer) then has no child layer: its arcs
  // lead to a virtual child level with one slot per arc (2u + beta), holding the copy-arc duals
  // mu_bar in the child-slot space; the layer of level l+1 (cut root) has no parent layer and
  // takes its forward messages from the arc duals mu. Per cut, in canonical (row, level) order:
  // cuts = {exit layer, root layer, first arc index, exit width | root width << 16},
  // cut_slots = {exit own slot, exit child slot, root own slot, root child slot}, cut_live = index
  // of its first live pair among all live pairs (canonical order); cut_arc[arc] = the arc's child in
  // the root level (kBot for an arc into BOT), arcs numbered in canonical cut order. Records list
  // the n_cut_narrow narrow cuts (both levels at most 2 nodes) first, then the wide ones; cut_rb =
  // base of a wide cut's root-level in-arc lists in rbeg / rin (-1 for narrow cuts).
  int32_t split_k = 0;
  float split_gamma = 0.5f;
  int64_t n_cuts = 0, n_cut_narrow = 0, n_arcs_cut = 0, n_copy = 0, n_cut_parts = 0;
  std::vector<int32_t> var_interval;  // [n] interval of each variable (split only)
  std::vector<int32_t> cuts, cut_slots, cut_live, cut_rb;
  // per instance: its cut records in canonical order (offsets [n_inst + 1], record indices), for
  // the per-instance bounds (the sub-BDD after a cut adds its E to its row's instance)
  std::vector<int32_t> inst_cut, inst_cut_idx;
  std::vector<int32_t> cut_row;       // [n_cuts] row of each cut record (host)
  std::vector<int32_t> exit_rec;      // [I] with a split: the cut record whose exit layer this is, or -1
  std::vector<uint16_t> cut_arc;
  // Dataflow launch of a pass (one persistent launch; workgroups take tiles in pass order through a
  // device ticket): per normal tile of each pass, the tiles that write the messages it reads (the
  // tiles holding the parent layers of its layers in the forward pass, the child layers' tiles in
  // the backward pass), deduplicated and ascending, as CSR (dep_ptr [tiles + 1], dep_list). All of
  // them lie in earlier waves, so their indices are smaller than the tile's own. tinfo per tile: bit
  // 0 every layer is narrow, bit 1 positions go through bwd_list, bits 2-3 wave priority (3 for tiles
  // on the pass's longest dependency chains, lower with more slack). Plans with big tiles have none
  // (pers_ok false).
  bool pers_ok = false;
  std::vector<int32_t> fdep_ptr, fdep_list, bdep_ptr, bdep_list;
  std::vector<uint32_t> ftinfo, btinfo;
  // the same per tile as the kernel reads it, 8 words: start word, end word, tinfo | dependency
  // count << 8, offset of its dependencies in dep_list, then the first four dependencies (-1 pads)
  std::vector<int32_t> ftrec, btrec;
  // groups of instances (one ticket queue each in the dataflow launch): group of each variable, and
  // per pass each group's tiles in pass order (CSR over groups)
  int32_t n_groups = 1;
  std::vector<int32_t> var_group;
  std::vector<int32_t> fqptr, fqtile, bqptr, bqtile;
  // Two-branch wave launches (plans with dependency lists): each wave's tiles split at mid into a
  // part A [tile_begin, mid) and a part B [mid, tile_end). Every tile of an A part depends only on
  // tiles of earlier A parts, so the A parts run in order on one stream without waiting for B; the
  // B parts run in order on a second stream, part B of wave w after part A of wave b_wait (-1: no
  // A tile). A part is at most half of its wave (rounded up).
  struct WaveSplit {
    int32_t mid, b_wait;
  };
  std::vector<WaveSplit> fsplit, bsplit;
  // Node maps of the node-parallel (flat) path: per normal tile of each pass two words, the byte
  // offset of the tile's maps in the pass's map array (a multiple of 16) and its general own nodes
  // | child nodes << 16, or {-1, 0} when it has no general layer or its levels exceed the flat stage.
  // The maps hold, per own node and then per child node (the concatenated levels of the tile's
  // general layers in position order), the rank of the node's layer among the tile's general
  // layers; each tile's maps are padded to a multiple of 16 bytes.
  std::vector<int32_t> fgt, bgt;
  std::vector<uint8_t> fgm, bgm;
  // lanes per general layer for each tile width class (log2, 4 bits each), and the normal tiles
  // of each class over both passes
  uint32_t gsel = kDefaultGsel;
  int64_t tile_work = kTileWideWork;
  int64_t class_tiles[kWidthClasses] = {0, 0, 0, 0};
  ArenaLayout lay{};
};

int32_t make_plan(const Problem &p, const bddmp_options &opt, Plan &out);
int32_t primal_search(const Plan &P, const float *M, int32_t mode, int64_t max_dead_ends, int8_t *x, double *obj,
                      int32_t *feasible, int64_t *implied);
int32_t restrict_row(const Plan &P, int32_t row, int32_t n_fix, const int32_t *vars, const int8_t *vals,
                     uint8_t *alive, int32_t *lo, int32_t *hi, int32_t *feasible);
void greedy_colour_order(const Problem &p, std::vector<int32_t> &order);

}  // namespace bddmp
